"""The numpy Philox used to choose test packets: the published known-answer
vectors, and the packet whose FP32 launch optical depth is exactly 0."""
import json
import os

import numpy as np

import philox_np as P

HERE = os.path.dirname(__file__)
# packet of seed 1 whose launch optical-depth draw is 1 in FP32 (found by
# philox_np.find_launch_tau_zero(1)); used by the GPU regression test
TAU_ZERO_SEED, TAU_ZERO_PID = 1, 25324145


def test_known_answer_vectors():
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.json")) as fh:
        kat = json.load(fh)
    for case in kat["cases"]:
        c = [int(x, 16) for x in case["ctr"]]
        k = [int(x, 16) for x in case["key"]]
        out = P.philox4x32_10(*c, k[0], k[1])
        assert [int(x) for x in out] == [int(x, 16) for x in case["out"]]


def test_tau_zero_packet():
    pid = np.uint64(TAU_ZERO_PID)
    w0, _, _, _ = P.philox4x32_10(pid & P.MASK, pid >> np.uint64(32), 1, 0, TAU_ZERO_SEED, 0)
    assert P.fp32_draw_is_one(w0)
    u = np.float32((int(w0) >> 8) + 0.5) * np.float32(1.0 / 16777216.0)
    assert u == np.float32(1.0) and -np.log(u) == 0.0
    # the packets before it do not draw 1 there
    assert P.find_launch_tau_zero(TAU_ZERO_SEED, start=TAU_ZERO_PID - (1 << 20),
                                  chunk=1 << 20, limit=1 << 20) is None
