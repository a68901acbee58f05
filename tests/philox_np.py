"""Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) in numpy, written from
the published definition, for test inputs that need a chosen random draw:
e.g. the packet whose first optical-depth draw is exactly 1 in FP32.
Pinned to the published known-answer vectors by test_oracle_pins."""
import numpy as np

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Counters as uint32 arrays (broadcastable), key as two ints; returns
    the four output words as uint32 arrays."""
    c = [np.asarray(x, dtype=np.uint64) for x in (c0, c1, c2, c3)]
    c0, c1, c2, c3 = np.broadcast_arrays(*c)
    k0, k1 = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        n0 = (p1 >> np.uint64(32)) ^ c1 ^ np.uint64(k0)
        n2 = (p0 >> np.uint64(32)) ^ c3 ^ np.uint64(k1)
        c0, c1, c2, c3 = n0, p1 & MASK, n2, p0 & MASK
        k0 = (k0 + W0) & 0xFFFFFFFF
        k1 = (k1 + W1) & 0xFFFFFFFF
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def fp32_draw_is_one(word):
    """The FP32 path maps a word w to ((w >> 8) + 1/2) / 2^24, which rounds to
    exactly 1 when the top 24 bits are all set."""
    return (np.asarray(word, dtype=np.uint32) >> np.uint32(8)) == np.uint32(0xFFFFFF)


def find_launch_tau_zero(seed, start=0, chunk=1 << 22, limit=1 << 28):
    """First packet id >= start whose launch optical-depth draw (draw 4: word
    0 of Philox block 1) is exactly 1 in the FP32 path, i.e. tau = -ln 1 = 0."""
    for lo in range(start, start + limit, chunk):
        pid = np.arange(lo, lo + chunk, dtype=np.uint64)
        w0, _, _, _ = philox4x32_10(pid & MASK, pid >> np.uint64(32), 1, 0, seed, seed >> 32)
        hit = np.nonzero(fp32_draw_is_one(w0))[0]
        if hit.size:
            return int(pid[hit[0]])
    return None
