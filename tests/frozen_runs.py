"""Frozen-temperature runs of the same packets on the GPU (through the C-ABI)
and on the oracle, restricted to the packets whose events agree.

With a fixed temperature field no packet depends on another, and both sides
draw the same Philox numbers, so a packet's events are the same on both --
except, rarely, where a face is reached within rounding and the two sides'
different arithmetic decides it differently.  This helper finds the agreeing
packets from per-packet records and traces only the maximal ranges of them
again (by packet offset, same energy per packet), so the tallies of the two
sides can be compared cell by cell."""
import numpy as np

REC_FIELDS = ("fate", "k", "n_cross", "n_scat", "n_abs", "n_mrw", "n_draws")


def same_records(g, o):
    s = np.ones(len(g), bool)
    for f in REC_FIELDS:
        s &= g[f] == o[f]
    return s


def runs_of(mask):
    """Maximal [start, stop) ranges where mask is true."""
    out, start = [], None
    for i, v in enumerate(list(mask) + [False]):
        if v and start is None:
            start = i
        if not v and start is not None:
            out.append((start, i))
            start = None
    return out


def agreeing_runs(mcrt, make_ctx, ora, n, seed, T_frozen, torch, ctx=None, **kw):
    """Trace packets [0, n) frozen at T_frozen on a fresh context from
    make_ctx() and on the oracle, then again only the agreeing ranges on
    another fresh context (or on `ctx`, its tallies cleared) and on the
    oracle.  Returns (ctx, oracle state, fraction of packets that agreed)."""
    Tg = torch.from_numpy(np.ascontiguousarray(T_frozen)).cuda()
    probe = make_ctx()
    g = mcrt.Context.records_numpy(probe.trace(n, seed, frozen_T=Tg, n_recs=n))
    o = ora.run(n, seed, frozen_T=T_frozen, n_recs=n, **kw)["recs"]
    same = same_records(g, o)
    del probe
    if ctx is None:
        ctx = make_ctx()
    ctx.reset()
    st = None
    for a, b in runs_of(same):
        ctx.trace(b - a, seed, n_total=n, offset=a, frozen_T=Tg)
        st = ora.run(b - a, seed, n_total=n, offset=a, frozen_T=T_frozen, state=st, **kw)
    torch.cuda.synchronize()
    return ctx, st, float(same.mean())
