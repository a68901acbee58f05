"""Pick launch and solver options for a disk by timing them on the GPU, and
cache the choice per problem shape.

Knobs (`mcrt_options` fields, so a tuned context is an ordinary one, and
the packets per trace call, which the caller applies):
  * Trace launch shape: `block_size` and `blocks_per_cu` -- 512-thread
    workgroups, one per compute unit with the emission CDF in LDS (the
    default); 768-thread ones (3 wavefronts per SIMD, fewer registers); or
    256-thread ones, two per compute unit with the CDF in L2, or one.  FP32
    tracking only (the FP64 kernels are built for 512).
  * Trace hand-off: `wave_events`, the event count after which a packet still
    going once all packets are handed out moves to the whole-wavefront launch.
  * Packets per `mcrt_trace` call: a pass of n packets as 1, 2 or 4 calls
    (same packets, by offset); each call pays the tail of its longest walk,
    so one call is expected to win -- the tuner measures it.
  * PDA: `pda_solver` (1 grid-wide CG kernels, 2 one workgroup) and, for the
    one-workgroup solver, `pda_precond` (0 point Jacobi, 1 theta-line blocks).
    Timed on the region and Monte Carlo temperature of a real pass, restored
    before every solve, so every candidate solves the same system.
The trace candidates are timed as whole passes on the same seeds, so they
trace the same packets; each stage keeps the winner of the one before.

Nothing here runs implicitly: `options_for` only reads a cache, and `tune`
is called by the user (or `bench.py --autotune`).  `PACKAGED_CACHE` holds
choices measured on an MI355X, which `options_for` falls back to.
"""
import json
import math
import os
import time
from typing import Dict, Optional, Sequence

import numpy as np

CACHE_ENV = "MCRT_AUTOTUNE_CACHE"
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_0902_3092_amd",
                             "autotune.json")
PACKAGED_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_mi355x.json")
# what a choice holds beyond the mcrt_options fields
NON_OPTIONS = ("calls_per_pass",)
# physics options that must be equal between the tuned and the timed contexts
PHYSICS = ("precision", "mrw", "gamma", "n_int_min", "n_T", "pda_visits")


def cache_path(path: Optional[str] = None) -> str:
    return path or os.environ.get(CACHE_ENV) or DEFAULT_CACHE


def shape_key(disk, n_packets: int, **phys) -> str:
    """Cache key: grid and bin counts, physics options, the density scale and
    the packet count, both to the nearest decade."""
    rho = np.asarray(disk.rho, dtype=np.float64)
    top = float(rho.max()) if rho.size else 0.0
    dec = "none" if top <= 0.0 else "%d" % round(math.log10(top))
    n_r, n_mu = len(disk.r_edges) - 1, len(disk.mu_edges) - 1
    n_l = len(disk.lambda_edges) - 1
    ph = ",".join("%s=%s" % (k, phys[k]) for k in PHYSICS if k in phys)
    return "%dx%dx%d|rho1e%s|pk1e%d|%s" % (n_r, n_mu, n_l, dec,
                                           round(math.log10(max(n_packets, 1))), ph)


def load(path: Optional[str] = None) -> Dict[str, dict]:
    p = cache_path(path)
    try:
        with open(p) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return {}
    return data if isinstance(data, dict) else {}


def store(key: str, entry: dict, path: Optional[str] = None) -> None:
    p = cache_path(path)
    data = load(p)
    data[key] = entry
    os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, p)


def lookup(disk, n_packets: int, path: Optional[str] = None, **phys) -> Optional[dict]:
    """The cached entry for this shape (the user's cache, else the packaged
    one), or None."""
    key = shape_key(disk, n_packets, **phys)
    e = load(path).get(key)
    if e is None and path is None:
        e = load(PACKAGED_CACHE).get(key)
    return e


def options_for(disk, n_packets: int, path: Optional[str] = None, **phys) -> dict:
    """The cached mcrt_options fields for this shape, or {} (library
    defaults)."""
    e = lookup(disk, n_packets, path, **phys)
    return {k: v for k, v in e["options"].items() if k not in NON_OPTIONS} if e else {}


# what a batched pass takes from a disk's context: its hand-off threshold and
# PDA solver (the batched trace has one launch shape for all disks)
BATCH_KEYS = ("wave_events", "pda_solver", "pda_precond")


def batch_options(disk, n_packets: int, path: Optional[str] = None, **phys) -> dict:
    """The cached choices of this disk shape that a batched pass uses, or {}."""
    return {k: v for k, v in options_for(disk, n_packets, path, **phys).items()
            if k in BATCH_KEYS}


def calls_per_pass(disk, n_packets: int, path: Optional[str] = None, **phys) -> int:
    """The cached number of trace calls per pass for this shape (1 if none)."""
    e = lookup(disk, n_packets, path, **phys)
    return int(e["options"].get("calls_per_pass", 1)) if e else 1


def trace_pass(ctx, n_packets: int, seed: int, calls: int = 1, stream=None):
    """One pass of n packets as `calls` trace calls (packets by offset)."""
    per = -(-n_packets // calls)
    for off in range(0, n_packets, per):
        ctx.trace(min(per, n_packets - off), seed, n_total=n_packets, offset=off, stream=stream)


def pick(timings: Dict[str, float], ok: Dict[str, bool], default: str,
         margin: float = 0.03) -> str:
    """The fastest candidate that succeeded; the default unless another one is
    faster by more than `margin` (timing noise must not flip the choice)."""
    good = {k: t for k, t in timings.items() if ok.get(k, False) and math.isfinite(t)}
    if not good:
        return default
    best = min(good, key=good.get)
    if default in good and good[best] >= (1.0 - margin) * good[default]:
        return default
    return best


def _label(opts: dict) -> str:
    return ",".join("%s=%s" % kv for kv in sorted(opts.items()))


def tune(disk, *, n_packets: int = 200000, seeds: Sequence[int] = (11, 12),
         wave_events: Sequence[int] = (512, 2048, 8192),
         shapes: Sequence[tuple] = ((512, 0), (768, 0), (256, 0), (256, 1)),
         calls: Sequence[int] = (1, 2, 4), handoff: Sequence[int] = (0, 4096, 8192),
         pda_repeats: int = 3,
         path: Optional[str] = None, save: bool = True, log=None, **phys) -> dict:
    """Time the candidates on this disk and return (and cache) the choice:
    {"key", "options", "shape_s", "trace_s", "handoff_s", "calls_s", "pda_s",
    "pda_iters"}.  shapes: (block_size, blocks_per_cu) pairs, tried with FP32
    tracking; handoff: live counts at which hand-offs begin (0: the hand-off
    launch's wavefronts)."""
    import torch
    from . import mcrt as M

    say = log or (lambda s: None)
    phys = dict(phys)
    phys.setdefault("precision", "fp32")
    phys.setdefault("mrw", True)
    key = shape_key(disk, n_packets, **phys)

    def passes(opts, n_calls=1):
        """(median seconds of a pass over the seeds, every packet traced and
        none capped).  A pass lasts as long as its longest walk, which the
        running temperature makes differ from run to run even on one seed, so
        the median of several is taken."""
        ctx = M.Context(disk, **phys, **opts)
        ts = []
        for s in seeds:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.reset()
            trace_pass(ctx, n_packets, int(s), n_calls)
            ctx.update_T()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        c = ctx.counters()
        del ctx
        return float(np.median(ts)), c["capped"] == 0 and c["launch"] == n_packets

    # launch shape (FP32 only), then the hand-off threshold, then calls per pass
    shape_s, shape_ok = {}, {}
    if phys["precision"] != "fp32":
        shapes = ((512, 0),)
    for bs, per_cu in shapes:
        lab = "%d/%d" % (bs, per_cu)
        shape_s[lab], shape_ok[lab] = passes(dict(block_size=bs, blocks_per_cu=per_cu))
        say("autotune: block_size/blocks_per_cu %s: %.3f s" % (lab, shape_s[lab]))
    bs_best, cu_best = (int(x) for x in pick(shape_s, shape_ok, "512/0").split("/"))
    shape = dict(block_size=bs_best, blocks_per_cu=cu_best)
    trace_s, trace_ok = {}, {}
    for we in wave_events:
        trace_s[str(we)], trace_ok[str(we)] = passes(dict(wave_events=int(we), **shape))
        say("autotune: wave_events=%d: %.3f s" % (we, trace_s[str(we)]))
    we_best = int(pick(trace_s, trace_ok, str(2048 if 2048 in wave_events else wave_events[0])))
    handoff_s, handoff_ok = {}, {}
    for hl in handoff:
        handoff_s[str(hl)], handoff_ok[str(hl)] = passes(dict(wave_events=we_best,
                                                              handoff_live=int(hl), **shape))
        say("autotune: handoff_live=%d: %.3f s" % (hl, handoff_s[str(hl)]))
    hl_best = int(pick(handoff_s, handoff_ok, str(handoff[0]))) if handoff else 0
    shape = dict(shape, handoff_live=hl_best)
    calls_s, calls_ok = {}, {}
    for k in calls:
        calls_s[str(k)], calls_ok[str(k)] = passes(dict(wave_events=we_best, **shape), int(k))
        say("autotune: %d trace call(s) per pass: %.3f s" % (k, calls_s[str(k)]))
    calls_best = int(pick(calls_s, calls_ok, "1"))

    # PDA: the region and MC temperature of one pass, the same system for all
    base = M.Context(disk, wave_events=we_best, **shape, **phys)
    base.reset()
    base.trace(n_packets, int(seeds[0]))
    base.update_T()
    T_mc = base.get(M.GET_T).clone()
    base.pda_solve()
    mask = (base.get(M.GET_REGION) == 1).to(torch.uint8).contiguous()
    n_cells = base.n_cells
    del base
    cands = [dict(pda_solver=1, pda_precond=0)]
    if n_cells <= 65536:
        cands += [dict(pda_solver=2, pda_precond=0), dict(pda_solver=2, pda_precond=1)]
    if int(mask.sum().item()) == 0:
        cands = []   # no region at this packet count: nothing to time, library defaults
    pda_s, pda_ok, pda_it = {}, {}, {}
    for cand in cands:
        ctx = M.Context(disk, wave_events=we_best, **shape, **phys, **cand)
        best = float("inf")
        st = None
        for _ in range(pda_repeats):
            ctx.set_T(T_mc)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                st = ctx.pda_solve(mask)
            except M.McrtError:  # not converged: this candidate fails
                st = None
                break
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        lab = _label(cand)
        pda_s[lab] = best
        pda_ok[lab] = st is not None and st["rc"] == M.OK and \
            (st["n_region"] == 0 or st["last_change"] < 1e-6)
        pda_it[lab] = int(st["cg_iters_total"]) if st is not None else -1
        say("autotune: %s: %.4f s, %d CG iterations" % (lab, best, pda_it[lab]))
        del ctx
    opts = {"wave_events": we_best, "calls_per_pass": calls_best}
    opts.update(shape)
    if cands:
        default_pda = _label(dict(pda_solver=2, pda_precond=1)) if n_cells <= 65536 else \
            _label(cands[0])
        pda_best = pick(pda_s, pda_ok, default_pda)
        opts.update({k: int(v) for k, v in (kv.split("=") for kv in pda_best.split(","))})
    entry = {"key": key, "options": opts, "shape_s": shape_s, "trace_s": trace_s,
             "handoff_s": handoff_s, "calls_s": calls_s, "pda_s": pda_s,
             "pda_iters": pda_it, "n_packets": n_packets, "seeds": list(seeds),
             "device": torch.cuda.get_device_name(0),
             "when": time.strftime("%Y-%m-%dT%H:%M:%S")}
    if save:
        store(key, entry, path)
    return entry
