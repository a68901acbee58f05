"""Benchmark of the hot path on one MI355X.

One step = one pass of the whole path over one disk: clear the tallies, trace
the step's photon packets with immediate reemission and the modified random
walk (gamma = 3, 20 interactions in the cell first) in one call, invert the
cell temperatures, and solve the partial diffusion approximation on cells
entered by fewer than 100 packets.  Workload: the 1e-2 Msun disk on 0.1-100
AU, 100 r x 60 theta cells, 100 wavelength bins, kappa ~ 1/lambda beyond 1
micron, albedo 0.5, midplane radial optical depth 1e5 (inputs synthetic and
seeded).  A step holds 1e8 packets by default: the count at which a run's
midplane temperature comes within 1 % (the metric's condition), which the same
run measures.

Printed: one JSON line with
* packets/s of the whole step (the value) and the roofline of the trace call
  (events x FP operations per event over the HIP-event duration of the call);
* the midplane-T error of the last timed step against an FP64 no-MRW
  reference of as many packets in two independent halves, the reference's
  own noise removed in quadrature, and whether it is <= 1 %;
* the plain FP64 path on the same step, and the configuration's own
  1e6-packet step;
* the 64-disk batched workload at its drawn packet counts, five passes in one
  HIP graph, beside the plain FP64 path one disk at a time on a sample of the
  disks; the batched PDA of the last pass alone, in GB/s;
* the vertical-structure loop with the hydrostatic step run to convergence
  on the device (passes and the statistic of each);
* the ray-traced SED (source function of the Monte Carlo T and mean
  intensity) with and without the MRW at 1e6 packets, and the ray tracer's
  time;
* the PDA and its adjoint on the 200 x 120 differentiation workload;
* the CPU oracle on a bounded sample of the step on this host.
Stage lines go to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# FP operations per event of the transport, counted on the reference
# implementation (adds, multiplies, divides, square roots and transcendental
# calls each count one): a face crossing evaluates two sphere and two cone
# quadratics and moves the packet; an interaction moves, draws the scattering
# decision, a new direction and a new optical depth; an absorption adds two
# temperature inversions and the reemission-bin search; an MRW step adds the
# distance to the cell boundary, the escape-time solve, the deposit, the jump
# and a reemission; a launch places the packet on the star.
FLOPS_PER_EVENT = {"cross": 62, "scat": 25, "abs": 90, "mrw": 270, "launch": 40}
PEAK = {"fp64": 78.6e12, "fp32": 157.3e12}
HBM_PEAK = 8.0e12
# BiCGSTAB on the transposed Jacobian, bytes per unknown and iteration (FP64):
# two operator products, each reading the diagonal, four couplings and the
# vector at the cell and its four neighbours and writing the product (11
# words, 88 B); the updates p, y (read r, p, v, diagonal; write p, y), s, z
# (read r, v, diagonal; write s, z), lambda, r (read lambda, y, z, s, t;
# write lambda, r) and the dot products' extra reads of rh (2): 6 + 5 + 7 + 2
# = 20 words.
BICGSTAB_BYTES_PER_UNKNOWN = 2 * 88 + 20 * 8
# PCG bytes per unknown and iteration (FP64).  Jacobi: the operator product
# reads diag, two couplings and p and writes q (40 B); the update reads x, r,
# p, q and diag and writes x, r and p (64 B).  Theta-line preconditioner: the
# update no longer reads diag (-8 B); the forward sweep reads r, the pivot and
# a coupling and writes y, the backward sweep reads y, the pivot and a
# coupling and writes z (+64 B).
PCG_BYTES_PER_UNKNOWN = {0: 104, 1: 160}
# per unknown and Picard sweep: assembly reads T, rho of the cell (its four
# neighbours come from cache) and writes diag, two couplings, b and x (56 B);
# the T update reads x and writes T (16 B)
PDA_SWEEP_BYTES = 72
PDA_COUNTERS_JSON = os.path.join(ROOT, "profiles", "pda_batched_counters.json")


# Sources of the FP32 trace kernel; HBM traffic measured with rocprofv3
# counters is reported only while they are unchanged.
TRACE32_SOURCES = ("trace_fp32.hip", "trace_common.h", "rng.h", "mcrt_internal.h")
COUNTERS_JSON = os.path.join(ROOT, "profiles", "trace_fp32_counters.json")
# the two kernels of one FP32 trace call, whose counters the summary adds up
TRACE32_KERNELS = "trace_fp32_kernel + trace_fp32_tail_kernel"


def trace32_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in TRACE32_SOURCES:
        with open(os.path.join(ROOT, "paper_0902_3092_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, packets):
    """(HBM bytes per launch from the committed counter summary, or None when
    it covers another kernel, launch size or source; and why)."""
    try:
        with open(COUNTERS_JSON) as fh:
            c = json.load(fh)
    except (OSError, ValueError) as e:
        return None, "no counter summary (%s)" % type(e).__name__
    if c.get("kernel") != kernel or c.get("packets") != packets:
        return None, "the counter summary covers another kernel or launch size"
    h = trace32_source_hash()
    if c.get("source_sha256") != h:
        return None, "the kernel sources changed since the counters were taken (%s)" % h[:12]
    return (1024.0 * (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]),
            "profiles/trace_fp32_counters.json")


T_START = time.perf_counter()


def log(msg):
    print("bench: [%6.1f s] %s" % (time.perf_counter() - T_START, msg), file=sys.stderr,
          flush=True)


def elapsed():
    return time.perf_counter() - T_START


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--precision", default="fp32", choices=["fp64", "fp32"])
    p.add_argument("--packets", type=int, default=100000000,
                   help="packets per timed step")
    p.add_argument("--ref-packets", type=int, default=0,
                   help="packets of the midplane-T reference, two halves (0: as a step)")
    p.add_argument("--c1-steps", type=int, default=3,
                   help="timed steps at the configuration's own 1e6 packets (0: skip)")
    p.add_argument("--c3-plain-every", type=int, default=8,
                   help="the plain FP64 comparison of the 64-disk workload runs every n-th disk")
    p.add_argument("--cpu-packets", type=int, default=1000000)
    p.add_argument("--budget-s", type=float, default=540.0,
                   help="wall-clock budget of the whole run: a leg after the timed steps "
                        "whose expected length would pass it is skipped and reported so")
    p.add_argument("--tune-out", default="",
                   help="time the autotuner's candidates on the step at --packets, write "
                        "the choice to this file and exit")
    p.add_argument("--sed-study", type=int, default=0,
                   help="the MRW's effect on the ray-traced SED at this many packets per run "
                        "and exit")
    p.add_argument("--pda-probe", action="store_true",
                   help="the 64-disk workload, one pass at its drawn packets, then the batched "
                        "PDA of that pass alone (for counter runs) and exit")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--no-hydro", action="store_true")
    p.add_argument("--no-sed", action="store_true")
    p.add_argument("--no-ref", action="store_true")
    p.add_argument("--no-batch", action="store_true")
    p.add_argument("--no-pda", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--large", type=int, default=0,
                   help="only run the large disk (400 x 200 cells, 200 bins, 3 species) with this "
                        "many packets, FP32 and FP64, and exit")
    p.add_argument("--autotune", action="store_true",
                   help="time the tuner's candidates on the step's disk first (2e5-packet "
                        "passes) and run the step with its choice")
    p.add_argument("--c3", type=float, default=0.0,
                   help="only run the 64-disk batched workload at this fraction of its drawn "
                        "packets, --c3-passes passes in one graph, and exit")
    p.add_argument("--c3-passes", type=int, default=5)
    p.add_argument("--c3-split", action="store_true",
                   help="with --c3: submit each pass as a graph of its own")
    p.add_argument("--c3-plain", action="store_true",
                   help="with --c3: also one pass of each disk alone on the FP64 path")
    p.add_argument("--large-chunk", type=int, default=0,
                   help="with --large: packets per mcrt_trace call (0: all in one call)")
    p.add_argument("--accuracy-g", type=float, default=0.0,
                   help="asymmetry parameter of the accuracy study's scattering")
    p.add_argument("--hydro", type=int, default=0,
                   help="only run this many passes of the vertical-structure loop (trace, T, "
                        "PDA, hydrostatic equilibrium) and exit")
    p.add_argument("--hydro-batched", type=int, default=0,
                   help="only run this many passes of that loop as one graph-captured "
                        "mcrt_batch_run call and exit")
    p.add_argument("--aniso", type=float, default=0.0,
                   help="only time the step with Henyey-Greenstein scattering of this asymmetry "
                        "parameter beside the isotropic one, and exit")
    p.add_argument("--accuracy", type=int, default=0,
                   help="only compare MRW gamma = 1/3/10 and PDA on/off runs of --packets "
                        "packets with an FP64 no-MRW, no-PDA reference of this many packets, "
                        "and exit")
    p.add_argument("--event-mix", action="store_true",
                   help="only fit the per-event cost of each event type from three albedos, "
                        "and exit")
    p.add_argument("--tail-probe", action="store_true",
                   help="only time the longest packet of a frozen-temperature sample of the step, "
                        "alone, per lane and in whole-wavefront mode, and exit")
    p.add_argument("--source-hash", action="store_true",
                   help="print the hash of the FP32 trace kernel sources and exit")
    p.add_argument("--handoff-live", type=int, default=-1,
                   help="override the hand-off live count of the timed step (0: the hand-off "
                        "launch's wavefronts)")
    p.add_argument("--runahead", type=int, default=-1,
                   help="override wave_runahead of the timed step (0 or 1)")
    p.add_argument("--block-size", type=int, default=-1,
                   help="override block_size of the timed step (0, 256, 512, 768)")
    p.add_argument("--copy-mib", type=int, default=0,
                   help="only copy this many MiB device to device once (a plain copy kernel of "
                        "known size, to scale the HBM byte counters) and exit")
    return p.parse_args()


def host_cpu():
    """Host CPU model and the number of processors this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0)), os.cpu_count()


def cpu_baseline(disk, opts, n_packets):
    """The CPU oracle (single thread) on a bounded sample of the same step."""
    import oracle
    oracle.build(force=False)
    ora = oracle.Oracle(disk, n_T=opts.n_T)
    t0 = time.perf_counter()
    st = ora.run(n_packets, opts.seed, mrw=True, gamma=opts.gamma, n_int_min=opts.n_int_min)
    T = ora.update_T(st["E_abs"])
    region = ora.pda_region(st["visits"], st["n_abs"], st["n_mrw"], visits_min=opts.pda_visits)
    ora.pda(T, region)
    dt = time.perf_counter() - t0
    model, usable, total = host_cpu()
    return {"value": n_packets / dt, "unit": "photon packets/s", "cores": 1, "kind": "oracle",
            "host_cpu_model": model, "host_nproc_usable": usable, "host_cpu_count": total,
            "sample": "%d packets of the timed step's disk (trace + T + PDA), one thread, %.1f s"
                      % (n_packets, dt)}


def run_once(ctx, n, seed):
    ctx.reset()
    ctx.trace(n, seed)
    ctx.update_T()
    return ctx.pda_solve()


def fields(ctx, mcrt):
    return (ctx.get(mcrt.GET_T).cpu().numpy(), ctx.get(mcrt.GET_VISITS).cpu().numpy(),
            ctx.get(mcrt.GET_REGION).cpu().numpy(), ctx.get(mcrt.GET_N_ABS).cpu().numpy())


def c3(mcrt, W, torch, scale, iters, plain, split=False):
    """The 64-disk batched workload at `scale` of its drawn packets: `iters`
    passes (trace, T, PDA) in one graph-captured submission, the MRW
    coefficients of pass k > 0 taken from the temperature after pass k-1;
    then, with `plain`, one pass of each disk alone on the FP64 path
    (no graph), the same packet counts."""
    draws = W.batch_draws()
    npk = [max(1000, int(round(b["n_packets"] * scale))) for b in draws]
    seeds = [b["seed"] for b in draws]
    ctxs = batch_contexts(mcrt, W, draws)
    torch.cuda.synchronize()
    log("c3: %d disks, %d packets per pass, %d passes in %s" %
        (len(ctxs), sum(npk), iters, "one graph each" if split else "one graph"))
    t0 = time.perf_counter()
    if split:
        # one graph per pass (a pass takes the previous pass's T through the
        # contexts), so that each pass reports when it ends
        for it in range(iters):
            st = mcrt.batch_run(ctxs, npk, [sd + (it << 32) for sd in seeds], n_iter=1,
                                use_graph=True)
            torch.cuda.synchronize()
            log("c3: pass %d done (%.1f s)" % (it + 1, time.perf_counter() - t0))
    else:
        st = mcrt.batch_run(ctxs, npk, seeds, n_iter=iters, use_graph=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log("c3: batched done (%.1f s)" % dt)
    out = {"workload": "64 disks, log10 M ~ U(-5,-1), 50x40 to 200x120 cells, 100 bins, "
                       "MRW gamma=3, PDA < 100 visits",
           "packet_scale": scale, "packets_per_pass": sum(npk), "passes": iters,
           "batched_fp32": {"value": iters * sum(npk) / dt, "unit": "photon packets/s",
                            "s": dt, "graph": "one per pass" if split else "all passes",
                            "mrw_coef_T": "previous pass",
                            "pda_region_cells_last_pass": int(sum(x["n_region"] for x in st)),
                            "pda_cg_iters_max": int(max(x["cg_iters_total"] for x in st))}}
    del ctxs
    if plain:
        tp = 0.0
        for q, (b, n, sd) in enumerate(zip(draws, npk, seeds)):
            ctx = mcrt.Context(W.batch_disk(b), precision="fp64", mrw=True, gamma=3.0,
                               n_int_min=20, pda_visits=100)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            run_once(ctx, n, sd)
            torch.cuda.synchronize()
            tp += time.perf_counter() - t1
            del ctx
            log("c3: plain FP64, %d disks done (%.1f s)" % (q + 1, tp))
        out["plain_fp64_one_at_a_time"] = {"value": sum(npk) / tp, "unit": "photon packets/s",
                                           "s": tp, "passes": 1, "graph": False}
    return out


def large(mcrt, W, torch, n_packets, chunk_packets=0):
    """The large disk: one pass (trace, T, PDA) with FP32 tracking and with the
    all-FP64 path at the same packet count; their temperature difference
    against the photon noise of both runs."""
    import numpy as np
    d, o = W.config("large")
    out = {"workload": "disk 1e-1 Msun, 0.1-500 AU, 400 r x 200 theta, 200 lambda bins, "
                       "3 species, MRW gamma=3, PDA < 100 visits", "packets": n_packets,
           "packets_per_call": chunk_packets if chunk_packets > 0 else n_packets}
    T, NA, VIS = {}, {}, {}
    for prec in ("fp32", "fp64"):
        ctx = mcrt.Context(d, precision=prec, mrw=True, gamma=o.gamma, n_int_min=o.n_int_min,
                           pda_visits=o.pda_visits, n_T=o.n_T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.reset()
        # one call unless chunked: every call ends with its longest walks
        chunk = chunk_packets if chunk_packets > 0 else n_packets
        for off in range(0, n_packets, chunk):
            ctx.trace(min(chunk, n_packets - off), o.seed, n_total=n_packets, offset=off)
            torch.cuda.synchronize()
            log("large %s: %d packets traced (%.1f s)" % (prec, min(off + chunk, n_packets),
                                                        time.perf_counter() - t0))
        ctx.update_T()
        st = ctx.pda_solve()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        T[prec] = ctx.get(mcrt.GET_T).cpu().numpy()
        NA[prec] = ctx.get(mcrt.GET_N_ABS).cpu().numpy().view(np.uint32).astype(np.float64)
        VIS[prec] = ctx.get(mcrt.GET_VISITS).cpu().numpy().view(np.uint32)
        out[prec] = {"value": n_packets / dt, "unit": "photon packets/s", "s": dt,
                     "pda_region": st["n_region"], "counters": ctx.counters()}
        del ctx
    ok = (NA["fp32"] >= 100) & (NA["fp64"] >= 100) & (T["fp64"] > 0)
    rel = np.abs(T["fp32"][ok] / T["fp64"][ok] - 1.0)
    noise = np.sqrt(1.0 / (16.0 * NA["fp32"][ok]) + 1.0 / (16.0 * NA["fp64"][ok]))
    out["T_fp32_vs_fp64"] = {"cells": int(ok.sum()), "median_rel": float(np.median(rel)),
                             "median_photon_noise": float(np.median(noise)),
                             "frac_within_3_noise": float(np.mean(rel <= 3 * noise))}
    return out


def tail_probe(mcrt, W, torch):
    """Latency of one long random walk: on the step's disk with a frozen
    power-law temperature field (so a packet's events do not depend on the
    others), find the longest of 3e5 packets, then trace it alone, once per
    lane (wave_events = 0) and in whole-wavefront mode, FP32 both one event
    at a time and with runs of interactions traced lane-parallel."""
    import numpy as np
    d, o = W.config("mrw_pda")
    rc = 0.5 * (d.r_edges[:-1] + d.r_edges[1:]) / W.AU
    Tf = torch.from_numpy(np.ascontiguousarray(
        (300.0 * rc[:, None] ** -0.5 * (1 + 0.3 * d.mu_edges[None, 1:])).reshape(-1))).cuda()
    out = {"workload": "disk 1e-2 Msun, 100 r x 60 theta, frozen T = 300 K (r/AU)^-1/2 (1 + 0.3 mu)"}
    for prec in ("fp32", "fp64"):
        kw = dict(precision=prec, mrw=True, gamma=o.gamma, n_int_min=o.n_int_min, n_T=o.n_T)
        ctx = mcrt.Context(d, **kw)
        n = 300000
        recs = mcrt.Context.records_numpy(ctx.trace(n, 7, n_total=1000000, frozen_T=Tf, n_recs=n))
        ev = recs["n_cross"] + recs["n_scat"] + recs["n_abs"] + recs["n_mrw"]
        pid = int(np.argmax(ev))
        modes = (("per_lane", 0, 0), ("whole_wave", 32, 0))
        if prec == "fp32":
            modes += (("whole_wave_runahead", 32, 1),)
        res = {"pid": pid}
        for name, we, ra in modes:
            c1 = mcrt.Context(d, wave_events=we, wave_runahead=ra, **kw)
            c1.trace(1, 7, n_total=1000000, offset=pid, frozen_T=Tf)   # warm-up
            c1.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c1.trace(1, 7, n_total=1000000, offset=pid, frozen_T=Tf)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            c = c1.counters()
            e = c["cross"] + c["scat"] + c["abs"] + c["mrw"]
            res[name] = {"events": e, "s": dt, "us_per_event": dt / e * 1e6,
                         "counters": {k: c[k] for k in ("cross", "scat", "abs", "mrw")}}
            log("tail probe %s %s: %d events, %.2f us/event" % (prec, name, e, dt / e * 1e6))
        out[prec] = res
    return out


def accuracy(mcrt, W, torch, n_ref, n_run, g=0.0):
    """Synthetic analogue of the paper's accuracy study (Sect. 3.1-3.2): on the step's
    disk, runs of n_run packets with MRW at gamma = 1, 3, 10 (PDA on), with
    gamma = 3 and no PDA, and with no MRW, against an FP64 reference of n_ref
    packets with neither MRW nor PDA.  Reported over the cells the reference
    entered at least 1000 times: the mass-weighted mean |T/T_ref - 1|, its
    signed mean, its 5th and 95th percentiles, the photon noise 1/(4 sqrt N_abs)
    of both runs (mass-weighted), and the same on the midplane row.  Runs are
    traced in calls of at most 1e7 packets, one log line each.  g != 0: every
    run and the reference scatter by the Henyey-Greenstein phase function, so
    the MRW rows test the diffusion coefficient's (1 - g) sigma correction."""
    import numpy as np
    d, o = W.config("mrw_pda")
    m = d.rho * W.cell_volumes(d)
    chunk = 10000000

    def trace_all(ctx, n, seed, tag):
        t0 = time.perf_counter()
        for off in range(0, n, chunk):
            ctx.trace(min(chunk, n - off), seed, n_total=n, offset=off)
            torch.cuda.synchronize()
            log("accuracy: %s: %d of %d packets (%.1f s)" % (tag, min(off + chunk, n), n,
                                                            time.perf_counter() - t0))

    def noise(n_abs):
        return 1.0 / (4.0 * np.sqrt(np.maximum(n_abs, 1)))

    ref = mcrt.Context(d, precision="fp64", mrw=False, n_T=o.n_T, g_asym=g)
    ref.reset()
    t0 = time.perf_counter()
    trace_all(ref, n_ref, o.seed + 99, "reference")
    T_ref = ref.update_T().cpu().numpy()
    vis_ref = ref.get(mcrt.GET_VISITS).cpu().numpy().view(np.uint32)
    nz_ref = noise(ref.get(mcrt.GET_N_ABS).cpu().numpy())
    ok = (vis_ref >= 1000) & (T_ref > 0) & (m > 0)
    mid = np.zeros_like(ok)
    mid[0::d.n_mu] = True
    out = {"workload": "disk 1e-2 Msun, 100 r x 60 theta, 100 bins", "g": g, "reference":
           {"packets": n_ref, "precision": "fp64", "mrw": False, "pda": False,
            "s": time.perf_counter() - t0, "cells": int(ok.sum())}, "runs": []}
    del ref
    cases = [("no MRW, PDA", False, 3.0, True), ("MRW gamma=1, PDA", True, 1.0, True),
             ("MRW gamma=3, PDA", True, 3.0, True), ("MRW gamma=10, PDA", True, 10.0, True),
             ("MRW gamma=3, no PDA", True, 3.0, False)]
    for name, mrw, gamma, pda in cases:
        ctx = mcrt.Context(d, precision="fp32", mrw=mrw, gamma=gamma, n_int_min=o.n_int_min,
                           pda_visits=o.pda_visits, n_T=o.n_T, g_asym=g)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.reset()
        trace_all(ctx, n_run, o.seed + 7, name)
        T = ctx.update_T().clone()
        n_reg = 0
        if pda:
            n_reg = ctx.pda_solve()["n_region"]
            T = ctx.get(mcrt.GET_T)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        T = T.cpu().numpy()
        nz = noise(ctx.get(mcrt.GET_N_ABS).cpu().numpy())
        rel = T / np.where(T_ref > 0, T_ref, 1.0) - 1.0
        row = {"case": name, "packets": n_run, "s": dt, "pda_cells": int(n_reg)}
        for tag, sel in (("all", ok), ("midplane", ok & mid)):
            if sel.any():
                w = m[sel] / m[sel].sum()
                row[tag] = {"mean_abs": float((np.abs(rel[sel]) * w).sum()),
                            "mean_signed": float((rel[sel] * w).sum()),
                            "p05": float(np.percentile(rel[sel], 5)),
                            "p95": float(np.percentile(rel[sel], 95)),
                            "noise_run": float((nz[sel] * w).sum()),
                            "noise_ref": float((nz_ref[sel] * w).sum()),
                            "cells": int(sel.sum())}
        out["runs"].append(row)
        log("accuracy: %s: %.1f s, mean |dT/T| %.4f" % (name, dt, row["all"]["mean_abs"]))
        del ctx
    return out


def aniso(mcrt, W, torch, g, steps):
    """The step (1e6 packets, FP32 tracking, MRW, PDA) on the step's disk with
    Henyey-Greenstein scattering of asymmetry g, and the same step with
    isotropic scattering, `steps` timed steps each after one warm-up."""
    d, o = W.config("mrw_pda")
    out = {"workload": "disk 1e-2 Msun, 100 r x 60 theta, 100 bins, 1e6 packets, MRW gamma=3, "
                       "PDA < 100 visits", "g": g}
    for name, gg in (("hg", g), ("isotropic", 0.0)):
        ctx = mcrt.Context(d, precision="fp32", mrw=True, gamma=o.gamma, n_int_min=o.n_int_min,
                           pda_visits=o.pda_visits, n_T=o.n_T, g_asym=gg)
        run_once(ctx, o.n_packets, o.seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            run_once(ctx, o.n_packets, o.seed + 1000 * (i + 1))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        c = ctx.counters()
        out[name] = {"value": o.n_packets / dt, "unit": "photon packets/s", "ms_per_step": dt * 1e3,
                     "steps": steps, "events_last_step": c}
        log("aniso: %s: %.3g packets/s" % (name, o.n_packets / dt))
    return out


def hydro(mcrt, W, torch, n_iter):
    """The vertical-structure loop of the method (Sect. 2.5, applied in Sect. 3.4) on the step's disk:
    n_iter passes of trace (1e6 packets, FP32, MRW) -> T -> PDA -> hydrostatic
    equilibrium (M_star = 2.5 Msun, mu = 2.3, shell masses kept).  After each
    pass: its time, the hydrostatic kernel's, and the convergence statistic,
    the mean over cells with >= 100 absorptions of |T_k - T_k-1| / sigma with
    sigma^2 the sum of both passes' 1 / (16 N_abs) T^2 (converged below 3)."""
    import numpy as np
    d, o = W.config("mrw_pda")
    ctx = mcrt.Context(d, precision="fp32", mrw=True, gamma=o.gamma, n_int_min=o.n_int_min,
                       pda_visits=o.pda_visits, n_T=o.n_T)
    stream = torch.cuda.current_stream()
    out = {"workload": "disk 1e-2 Msun, 100 r x 60 theta, 100 bins, 1e6 packets per pass, MRW "
                       "gamma=3, PDA < 100 visits; M_star 2.5 Msun, mu 2.3", "passes": []}
    prev = None
    for k in range(n_iter):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_once(ctx, o.n_packets, o.seed + 100 * k)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        T = ctx.get(mcrt.GET_T).cpu().numpy()
        nab = ctx.get(mcrt.GET_N_ABS).cpu().numpy().astype(np.float64)
        e0.record(stream)
        ctx.hydrostatic(2.5 * W.M_SUN, 2.3)
        e1.record(stream)
        torch.cuda.synchronize()
        row = {"s": time.perf_counter() - t0, "hydrostatic_ms": e0.elapsed_time(e1)}
        if prev is not None:
            Tp, np_ = prev
            ok = (nab >= 100) & (np_ >= 100) & (T > 0) & (Tp > 0)
            sig = np.sqrt(T[ok] ** 2 / (16 * nab[ok]) + Tp[ok] ** 2 / (16 * np_[ok]))
            row["mean_dT_over_sigma"] = float(np.mean(np.abs(T[ok] - Tp[ok]) / sig))
            row["cells"] = int(ok.sum())
        prev = (T, nab)
        out["passes"].append(row)
        log("hydro: pass %d: %.1f s %s" % (k, row["s"], row.get("mean_dT_over_sigma", "")))
    return out


def vertical_structure(mcrt, W, torch, max_iter):
    """The vertical-structure loop run to convergence on the device
    (mcrt_batch_converge): the step's disk with the hydrostatic step
    (M_star 2.5 Msun, mu 2.3), 1e6 packets per pass, one HIP graph per pass,
    stopped when the statistic R (the change of T against its photon noise
    from the split tallies, Sect. 2.5) is below 3."""
    d, o = W.config("mrw_pda")
    ctx = mcrt.Context(d, precision="fp32", mrw=True, gamma=o.gamma, n_int_min=o.n_int_min,
                       pda_visits=o.pda_visits, n_T=o.n_T, hydro_M_star=2.5 * W.M_SUN,
                       hydro_mu=2.3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, rec, rc = mcrt.batch_converge([ctx], [o.n_packets], [o.seed], max_iter=max_iter)
    torch.cuda.synchronize()
    s = time.perf_counter() - t0
    r = rec[0]
    return {"workload": "disk 1e-2 Msun, 100 r x 60 theta, 100 bins, 1e6 packets per pass, MRW "
                        "gamma=3, PDA < 100 visits; hydrostatic step M_star 2.5 Msun, mu 2.3",
            "passes": r["passes"], "converged_pass": r["converged_pass"],
            "R_per_pass": [round(x, 3) for x in r["R"]], "threshold": 3.0,
            "dT_rms_last": r["dT_rms"], "noise_rms_last": r["noise_rms"],
            "cells_compared": r["cells"], "return_code": rc, "s": s,
            "packets_per_s": r["passes"] * o.n_packets / s}


def sed_study(mcrt, W, torch, n_packets, cos_i=(0.7071067811865476, 0.2588190451025208,
                                                  0.9659258262890683)):
    """The effect of the MRW on the ray-traced SED (Sect. 3.3): the step's
    disk traced with the MRW (FP32, gamma = 3) and without it (FP64, the
    reference), n_packets each with the path-length tallies; the SED of each
    from its Monte Carlo T (before the PDA) and its mean intensity, at 45
    degrees and two more inclinations; the relative difference per bin.  Also
    the ray tracer's time."""
    import numpy as np
    d, o = W.config("mrw_pda")
    out = {"workload": "disk 1e-2 Msun, 100 r x 60 theta, 100 bins, %.3g packets each, "
                       "MRW gamma=3 (FP32) against no MRW (FP64)" % n_packets,
           "cos_i": list(cos_i)}
    seds = {}
    for name, kw in (("mrw", dict(precision="fp32", mrw=True)),
                     ("reference", dict(precision="fp64", mrw=False))):
        ctx = mcrt.Context(d, gamma=o.gamma, n_int_min=o.n_int_min, pda_visits=o.pda_visits,
                           n_T=o.n_T, j_tally=1, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.reset()
        ctx.trace(n_packets, o.seed + 5150)
        T = ctx.update_T()
        J = ctx.mean_intensity(T)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L = ctx.raytrace_sed(T, J, cos_i=list(cos_i), n_sub=4, n_phi=32)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        seds[name] = L.cpu().numpy()
        out[name + "_trace_s"] = t1 - t0
        out[name + "_raytrace_ms"] = (t2 - t1) * 1e3
        if name == "mrw":
            # the image behind the same rays at 45 degrees and its visibility
            # amplitudes for a 100 m baseline at 150 pc (two position angles)
            img = ctx.raytrace_image(T, J, cos_i=[cos_i[0]], n_sub=4, n_phi=32)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            V = ctx.visibility(img, [cos_i[0]], 4, 32, [[1e4, 0.0], [1e4, 1.5707963267948966]],
                               150 * 3.0857e18)
            torch.cuda.synchronize()
            t4 = time.perf_counter()
            lam = np.sqrt(d.lambda_edges[:-1] * d.lambda_edges[1:])
            nband = (lam >= 8e-4) & (lam <= 13e-4)
            Vn = V.cpu().numpy()[0][:, nband]
            out["visibility_100m_150pc_nband"] = {
                "position_angles_rad": [0.0, 1.5707963267948966],
                "min": [float(v.min()) for v in Vn], "max": [float(v.max()) for v in Vn],
                "visibility_ms": (t4 - t3) * 1e3, "bins": int(nband.sum())}
        log("sed study: %s done (%.1f s trace, %.1f ms ray tracing)" % (name, t1 - t0,
                                                                      (t2 - t1) * 1e3))
        del ctx
    a, b = seds["mrw"], seds["reference"]
    rel = a / np.where(b > 0, b, 1) - 1
    keep = b > 1e-6 * b.max(axis=1, keepdims=True)   # bins that carry light
    out["max_abs_rel_diff"] = [float(np.abs(rel[q][keep[q]]).max()) for q in range(len(cos_i))]
    out["mean_abs_rel_diff"] = [float(np.abs(rel[q][keep[q]]).mean()) for q in range(len(cos_i))]
    out["rays"] = len(cos_i) * (d.n_r + 1) * 4 * 32
    return out


def hydro_batched(mcrt, W, torch, n_iter):
    """The same loop as one mcrt_batch_run call: n_iter passes of trace (1e6
    packets) -> T -> PDA -> hydrostatic equilibrium captured in one HIP graph
    on the step's disk; the call's time and the shell masses kept."""
    import numpy as np
    d, o = W.config("mrw_pda")
    ctx = mcrt.Context(d, precision="fp32", mrw=True, gamma=o.gamma, n_int_min=o.n_int_min,
                       pda_visits=o.pda_visits, n_T=o.n_T, hydro_M_star=2.5 * W.M_SUN,
                       hydro_mu=2.3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = mcrt.batch_run([ctx], [o.n_packets], [o.seed], n_iter=n_iter, use_graph=True)
    torch.cuda.synchronize()
    s = time.perf_counter() - t0
    rho = ctx.get(mcrt.GET_RHO).cpu().numpy()
    return {"workload": "disk 1e-2 Msun, 100 r x 60 theta, 100 bins, 1e6 packets per pass, MRW "
                        "gamma=3, PDA < 100 visits; M_star 2.5 Msun, mu 2.3; one graph",
            "passes": n_iter, "s": s, "packets_per_s": n_iter * o.n_packets / s,
            "pda_region_last_pass": stats[0]["n_region"],
            "rho_finite": bool(np.all(np.isfinite(rho))),
            "midplane_rho_ratio_max": float(np.max(rho.reshape(d.n_r, -1)[:, 0] /
                                                   np.maximum(d.rho.reshape(d.n_r, -1)[:, 0], 1e-300)))}


def event_mix(mcrt, W, torch):
    """Per-event cost by event type: the longest frozen-T walk (of 1e5
    packets) on the step's disk with albedo 0.1, 0.5 and 0.9 at the same
    extinction, traced alone per lane and in whole-wavefront mode; a
    least-squares fit of the times against the event counts gives the cost
    of a scattering, an absorption, and a crossing or MRW step."""
    import numpy as np
    rows = []
    for om in (0.1, 0.5, 0.9):
        d = W.make_disk("mix", M_dust_msun=1e-2, n_r=100, n_mu=60, n_lambda=100,
                        species=(((1.0 - om) / 0.5, om),))
        rc = 0.5 * (d.r_edges[:-1] + d.r_edges[1:]) / W.AU
        Tf = torch.from_numpy(np.ascontiguousarray(
            (300.0 * rc[:, None] ** -0.5 * (1 + 0.3 * d.mu_edges[None, 1:])).reshape(-1))).cuda()
        for prec in ("fp32", "fp64"):
            kw = dict(precision=prec, mrw=True, gamma=3.0, n_int_min=20)
            ctx = mcrt.Context(d, **kw)
            n = 100000
            recs = mcrt.Context.records_numpy(ctx.trace(n, 7, n_total=1000000, frozen_T=Tf,
                                                        n_recs=n))
            ev = recs["n_cross"] + recs["n_scat"] + recs["n_abs"] + recs["n_mrw"]
            pid = int(np.argmax(ev))
            for name, we in (("per_lane", 0), ("whole_wave", 32)):
                c1 = mcrt.Context(d, wave_events=we, **kw)
                c1.trace(1, 7, n_total=1000000, offset=pid, frozen_T=Tf)   # warm-up
                c1.reset()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                c1.trace(1, 7, n_total=1000000, offset=pid, frozen_T=Tf)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                c = c1.counters()
                rows.append(dict(albedo=om, precision=prec, mode=name, s=dt,
                                 **{k: c[k] for k in ("cross", "scat", "abs", "mrw")}))
                log("event mix: albedo %.1f %s %s: %.3f s" % (om, prec, name, dt))
    fits = {}
    for prec in ("fp32", "fp64"):
        for name in ("per_lane", "whole_wave"):
            sel = [r for r in rows if r["precision"] == prec and r["mode"] == name]
            A = np.array([[r["scat"], r["abs"], r["cross"] + r["mrw"]] for r in sel], float)
            t = np.array([r["s"] for r in sel])
            x = np.linalg.lstsq(A, t, rcond=None)[0] * 1e6
            fits["%s_%s" % (prec, name)] = {"us_scattering": x[0], "us_absorption": x[1],
                                            "us_crossing_or_mrw": x[2]}
    return {"rows": rows, "fit": fits}


def midplane_error_vs_halves(disk, T, visits, region, R1, R2):
    """Midplane-T error of a run against a reference made of two independent
    halves R1, R2 (FP64, no MRW): the mass-weighted mean |T/R - 1| over the
    midplane row (cells with >= 100 packet entries or in the PDA region), R the
    mean of the halves.  The reference's own photon noise is estimated cell by
    cell from the halves' difference, (R1 - R2)/(2R), and removed in
    quadrature: the run's RMS error is sqrt(RMS(d)^2 - RMS(ref noise)^2) (an
    unbiased estimate of its mean squared error, bias included), and its mean
    |error| is the measured mean |d| scaled by the same factor."""
    import numpy as np
    from paper_0902_3092_amd import workloads as W
    n_mu = disk.n_mu
    m = (disk.rho * W.cell_volumes(disk))[0::n_mu]
    T, R1, R2 = T[0::n_mu], R1[0::n_mu], R2[0::n_mu]
    R = 0.5 * (R1 + R2)
    ok = ((visits[0::n_mu] >= 100) | (region[0::n_mu] == 1)) & (R1 > 0) & (R2 > 0) & (m > 0)
    w = m[ok] / m[ok].sum()
    d = T[ok] / R[ok] - 1.0
    s_ref2 = ((R1[ok] - R2[ok]) / (2.0 * R[ok])) ** 2
    ms_d = float((w * d * d).sum())
    ms_ref = float((w * s_ref2).sum())
    ms_run = max(ms_d - ms_ref, 0.0)
    mean_abs_d = float((w * np.abs(d)).sum())
    scale = np.sqrt(ms_run / ms_d) if ms_d > 0 else 0.0
    mean_abs_run = mean_abs_d * scale
    return {"cells": int(ok.sum()), "pda_cells": int((ok & (region[0::n_mu] == 1)).sum()),
            "mean_abs_vs_reference": mean_abs_d, "rms_vs_reference": float(np.sqrt(ms_d)),
            "reference_noise_rms": float(np.sqrt(ms_ref)),
            "run_error_rms": float(np.sqrt(ms_run)), "run_error_mean_abs": float(mean_abs_run),
            "signed_mean": float((w * d).sum()), "max_abs_vs_reference": float(np.abs(d).max()),
            "meets_1pct": bool(mean_abs_run <= 0.01)}


def reference_halves(mcrt, disk, o, n_total, torch):
    """The reference of the midplane-T error: FP64 tracking, no MRW, the same
    PDA rule, n_total packets as two independent halves (each one call)."""
    out = []
    t0 = time.perf_counter()
    for h in range(2):
        ref = mcrt.Context(disk, precision="fp64", mrw=False, pda_visits=o.pda_visits, n_T=o.n_T)
        ref.reset()
        ref.trace(n_total // 2, o.seed + 4242 + 17 * h)
        ref.update_T()
        ref.pda_solve()
        torch.cuda.synchronize()
        out.append(ref.get(mcrt.GET_T).cpu().numpy())
        log("reference half %d of %d packets done (%.1f s)" % (h + 1, n_total // 2,
                                                             time.perf_counter() - t0))
        del ref
    return out, time.perf_counter() - t0


BATCH_PHYS = dict(precision="fp32", mrw=True, gamma=3.0, n_int_min=20, pda_visits=100)


def batch_contexts(mcrt, W, draws):
    """Contexts of the 64-disk workload, each with the autotuner's cached
    choices for its shape where there are any (MRW coefficients from the
    previous pass's T)."""
    from paper_0902_3092_amd import autotune
    out = []
    for b in draws:
        d = W.batch_disk(b)
        out.append(mcrt.Context(d, mrw_coef_T=1, **BATCH_PHYS,
                                **autotune.batch_options(d, b["n_packets"], **BATCH_PHYS)))
    return out


def batch_tuned_count(W, draws):
    from paper_0902_3092_amd import autotune
    return sum(1 for b in draws
               if autotune.batch_options(W.batch_disk(b), b["n_packets"], **BATCH_PHYS))


def c3_full(mcrt, W, torch, passes):
    """The 64-disk batched workload at its drawn packet counts: `passes`
    passes (trace, T, PDA) captured in one HIP graph, the MRW coefficients of
    pass k > 0 from the temperature after pass k - 1; then the batched PDA of
    the last pass alone (mcrt_batch_pda, HIP events)."""
    import numpy as np
    draws = W.batch_draws()
    npk = [b["n_packets"] for b in draws]
    seeds = [b["seed"] for b in draws]
    ctxs = batch_contexts(mcrt, W, draws)
    torch.cuda.synchronize()
    log("c3: %d disks, %.3g packets per pass, %d passes in one graph" %
        (len(ctxs), sum(npk), passes))
    t0 = time.perf_counter()
    st, rc = mcrt.batch_run_rc(ctxs, npk, seeds, n_iter=passes, use_graph=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log("c3: batched done (%.1f s, rc %d)" % (dt, rc))
    cnt = [c.counters() for c in ctxs]
    out = {"workload": "64 disks, log10 M ~ U(-5,-1), H/r0 ~ U(0.02,0.05), 50x40 to 200x120 "
                       "cells, 100 bins, 1e6-1e7 packets each per pass, MRW gamma=3, PDA < 100 "
                       "visits, MRW coefficients of pass k from pass k-1",
           "batched_fp32": {"value": passes * sum(npk) / dt, "unit": "photon packets/s",
                            "s": dt, "passes": passes, "packets_per_pass": sum(npk),
                            "graph": "all passes in one", "return_code": rc,
                            "capped_last_pass": int(sum(c["capped"] for c in cnt)),
                            "handed_off_last_pass": int(sum(c["handed"] for c in cnt)),
                            "cells": int(sum(c.n_cells for c in ctxs)),
                            "pda_region_cells_last_pass": int(sum(x["n_region"] for x in st)),
                            "disks_with_tuned_options": batch_tuned_count(W, draws)}}
    # the PDA of the last pass again, alone: Monte Carlo T from the tallies,
    # then all disks' PDA in one launch
    for c in ctxs:
        c.update_T()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    pst, prc = mcrt.batch_pda(ctxs, allow=(mcrt.E_SINGULAR_REGION, mcrt.E_NOT_CONVERGED))
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    bpu = PCG_BYTES_PER_UNKNOWN[ctxs[0].options.pda_precond]
    nbytes = sum(x["n_region"] * (x["cg_iters_total"] * bpu + x["sweeps"] * PDA_SWEEP_BYTES)
                 for x in pst)
    gbs = nbytes / (ms * 1e-3)
    out["batched_pda"] = {"kernel": "pda_wg_kernel (one workgroup per disk, 64 disks)",
                          "ms": ms, "unknowns": int(sum(x["n_region"] for x in pst)),
                          "cg_iters_total_max": int(max(x["cg_iters_total"] for x in pst)),
                          "sweeps_max": int(max(x["sweeps"] for x in pst)),
                          "algorithmic_bytes": nbytes, "achieved_GBps": gbs / 1e9,
                          "frac_hbm_peak": gbs / HBM_PEAK, "return_code": prc,
                          "bytes_model": "per unknown: %d B per CG iteration + %d B per Picard "
                                         "sweep (assembly, T update)" % (bpu, PDA_SWEEP_BYTES)}
    hit = pda_l2_hit_rate()
    if hit:
        out["batched_pda"].update(hit)
    del ctxs
    return out


def c3_plain(mcrt, W, torch, c3out, plain_every):
    """The plain FP64 path on every `plain_every`-th disk of the 64-disk
    workload, one at a time (one pass each, no graph), beside the batched
    passes of `c3out`."""
    draws = W.batch_draws()
    out = c3out
    sel = list(range(0, len(draws), plain_every))
    tp, npl = 0.0, 0
    for q in sel:
        b = draws[q]
        ctx = mcrt.Context(W.batch_disk(b), precision="fp64", mrw=True, gamma=3.0, n_int_min=20,
                           pda_visits=100)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        run_once(ctx, b["n_packets"], b["seed"])
        torch.cuda.synchronize()
        tp += time.perf_counter() - t1
        npl += b["n_packets"]
        del ctx
        log("c3: plain FP64 disk %d done (%.1f s so far)" % (q, tp))
    out["plain_fp64_one_at_a_time"] = {
        "value": npl / tp, "unit": "photon packets/s", "s": tp, "disks": len(sel),
        "disk_indices": "every %d-th of the 64" % plain_every, "packets": npl, "passes": 1,
        "graph": False}
    out["batched_vs_plain"] = out["batched_fp32"]["value"] / out["plain_fp64_one_at_a_time"]["value"]
    return out


def pda_probe(mcrt, W, torch):
    """One pass of the 64-disk workload at its drawn packets (batched, one
    graph), then the batched PDA of that pass on its own: the launch that the
    PDA counter runs select by kernel name."""
    draws = W.batch_draws()
    ctxs = batch_contexts(mcrt, W, draws)
    mcrt.batch_run_rc(ctxs, [b["n_packets"] for b in draws], [b["seed"] for b in draws],
                      n_iter=1, use_graph=True)
    torch.cuda.synchronize()
    log("pda probe: pass done")
    for c in ctxs:
        c.update_T()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pst, prc = mcrt.batch_pda(ctxs, allow=(mcrt.E_SINGULAR_REGION, mcrt.E_NOT_CONVERGED))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    bpu = PCG_BYTES_PER_UNKNOWN[ctxs[0].options.pda_precond]
    nbytes = sum(x["n_region"] * (x["cg_iters_total"] * bpu + x["sweeps"] * PDA_SWEEP_BYTES)
                 for x in pst)
    return {"s": dt, "unknowns": int(sum(x["n_region"] for x in pst)),
            "algorithmic_bytes": nbytes, "return_code": prc}


def pda_l2_hit_rate():
    """L2 and MALL hit rates of the batched PDA kernel from the committed
    counter summary, while the PDA source hashes the same."""
    try:
        with open(PDA_COUNTERS_JSON) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    import hashlib
    with open(os.path.join(ROOT, "paper_0902_3092_amd", "csrc", "pda.hip"), "rb") as fh:
        h = hashlib.sha256(fh.read()).hexdigest()
    if c.get("source_sha256") != h:
        return {"l2_hit_rate": None, "l2_note": "pda.hip changed since the counters were taken"}
    return {k: c[k] for k in ("l2_hit_rate", "mall_hit_rate", "counter_source") if k in c}


def pda_grad(mcrt, W, torch):
    import numpy as np
    d, _ = W.config("pda_grad")
    ctx = mcrt.Context(d)
    tb = ctx.tables()
    chi = lambda T: np.interp(T, tb["T"], 1.0 / (3.0 * tb["Drho"]))
    T_D, T_bc, mask, ks, w = W.pda_grad_inputs(d, chi)
    dev = lambda a, dt=None: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).cuda()
    m_t, TD_t, Tbc_t, ks_t, w_t = dev(mask, np.uint8), dev(T_D), dev(T_bc), dev(ks), dev(w)
    ctx.pda_linear(m_t, TD_t, Tbc_t, kscale=ks_t)          # warm-up
    ctx.pda_adjoint(w_t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = ctx.pda_linear(m_t, TD_t, Tbc_t, kscale=ks_t)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.pda_adjoint(w_t)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    bpu = PCG_BYTES_PER_UNKNOWN[ctx.options.pda_precond]
    nbytes = st["cg_iters_total"] * st["n_region"] * bpu
    gbs = nbytes / (t1 - t0)
    # the nonlinear PDA (D follows T) and the adjoint of its Jacobian
    ctx.pda_nonlinear(m_t, Tbc_t, kscale=ks_t)                 # warm-up
    ctx.pda_nonlinear_adjoint(w_t)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    _, nst = ctx.pda_nonlinear(m_t, Tbc_t, kscale=ks_t)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    _, _, ast = ctx.pda_nonlinear_adjoint(w_t, stats=True)
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    nl_bytes = ast["cg_iters_total"] * nst["n_region"] * BICGSTAB_BYTES_PER_UNKNOWN
    return {"workload": "200 r x 120 theta, 1e-1 Msun, region tau_R > 10",
            "preconditioner": "theta lines" if ctx.options.pda_precond else "Jacobi",
            "n_region": st["n_region"], "cg_iters": st["cg_iters_total"],
            "forward_ms": (t1 - t0) * 1e3, "adjoint_ms": (t2 - t1) * 1e3,
            "pcg_bytes_per_unknown_iter": bpu,
            "achieved_GBps": gbs / 1e9, "frac_hbm_peak": gbs / HBM_PEAK,
            "nonlinear": {"forward_ms": (t4 - t3) * 1e3, "picard_sweeps": nst["sweeps"],
                          "cg_iters_total": nst["cg_iters_total"],
                          "adjoint_ms": (t5 - t4) * 1e3,
                          "bicgstab_iters": ast["cg_iters_total"],
                          "bicgstab_bytes_per_unknown_iter": BICGSTAB_BYTES_PER_UNKNOWN,
                          "adjoint_GBps": nl_bytes / (t5 - t4) / 1e9}}


def main():
    a = parse()
    if a.source_hash:
        print(trace32_source_hash())
        return
    if a.gpus != 1:
        print("bench.py: the benchmark runs on one GPU; --gpus %d is not supported" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if a.copy_mib > 0:
        n = a.copy_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4}), flush=True)
        return

    from paper_0902_3092_amd import mcrt
    from paper_0902_3092_amd import workloads as W

    if a.tail_probe:
        print(json.dumps({"tail_probe": tail_probe(mcrt, W, torch)}), flush=True)
        return
    if a.event_mix:
        print(json.dumps({"event_mix": event_mix(mcrt, W, torch)}), flush=True)
        return
    if a.hydro > 0:
        print(json.dumps({"hydro": hydro(mcrt, W, torch, a.hydro)}), flush=True)
        return
    if a.hydro_batched > 0:
        print(json.dumps({"hydro_batched": hydro_batched(mcrt, W, torch, a.hydro_batched)}),
              flush=True)
        return
    if a.aniso != 0.0:
        print(json.dumps({"aniso": aniso(mcrt, W, torch, a.aniso, a.steps)}), flush=True)
        return
    if a.accuracy > 0:
        print(json.dumps({"accuracy": accuracy(mcrt, W, torch, a.accuracy, a.packets,
                                               a.accuracy_g)}), flush=True)
        return
    if a.large > 0:
        print(json.dumps({"large": large(mcrt, W, torch, a.large, a.large_chunk)}), flush=True)
        return
    if a.c3 > 0:
        print(json.dumps({"c3": c3(mcrt, W, torch, a.c3, a.c3_passes, a.c3_plain, a.c3_split)}),
              flush=True)
        return

    if a.pda_probe:
        print(json.dumps({"pda_probe": pda_probe(mcrt, W, torch)}), flush=True)
        return
    if a.sed_study > 0:
        print(json.dumps({"sed_study": sed_study(mcrt, W, torch, a.sed_study)}), flush=True)
        return

    disk, o = W.config("mrw_pda")
    N = a.packets
    from paper_0902_3092_amd import autotune
    phys = dict(precision=a.precision, mrw=True, gamma=o.gamma, n_int_min=o.n_int_min,
                pda_visits=o.pda_visits, n_T=o.n_T)
    if a.tune_out:
        # measure the choices for this step and write them where the package
        # keeps them (the caller copies the file into the package)
        log("autotune: timing candidates at %.3g packets" % N)
        e = autotune.tune(disk, n_packets=N, seeds=(11, 12, 13), path=a.tune_out, log=log,
                          **phys)
        print(json.dumps({"autotune": e}), flush=True)
        return
    if a.autotune:
        log("autotune: timing candidates")
        tuned = autotune.tune(disk, n_packets=N, seeds=(11,), log=log, **phys)
        tuned_src = "measured in this run"
    else:
        tuned = autotune.lookup(disk, N, **phys)
        tuned_src = ("the package's cache (%s), measured on an MI355X"
                     % os.path.basename(autotune.PACKAGED_CACHE))
    t_opts = autotune.options_for(disk, N, **phys) if tuned and not a.autotune else (
        {k: v for k, v in tuned["options"].items() if k not in autotune.NON_OPTIONS}
        if tuned else {})
    n_calls = int(tuned["options"].get("calls_per_pass", 1)) if tuned else 1
    t_opts = dict(t_opts)
    if a.handoff_live >= 0:
        t_opts["handoff_live"] = a.handoff_live
    if a.runahead >= 0:
        t_opts["wave_runahead"] = a.runahead
    if a.block_size >= 0:
        t_opts["block_size"] = a.block_size
    ctx = mcrt.Context(disk, **phys, **t_opts)
    stream = torch.cuda.current_stream()

    def step(i, ev=None):
        ctx.reset()
        if ev is not None:
            ev[0].record(stream)
        autotune.trace_pass(ctx, N, o.seed + 1000 * i, n_calls)
        if ev is not None:
            ev[1].record(stream)
        ctx.update_T()
        return ctx.pda_solve()

    log("warmup %d step(s) of %.3g packets" % (a.warmup, N))
    for i in range(a.warmup):
        step(i)
        torch.cuda.synchronize()
        log("warmup step %d done" % (i + 1))
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(a.steps)]
    counters = []
    pda = None
    log("timing %d step(s)" % a.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        pda = step(a.warmup + i, evs[i])
        counters.append(ctx.counters())     # waits for the step
        log("timed step %d done (%.1f s)" % (i + 1, time.perf_counter() - t0))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / a.steps
    trace_ms = [e0.elapsed_time(e1) for e0, e1 in evs]
    T_meas, vis_meas, reg_meas, nabs_meas = fields(ctx, mcrt)

    def sigma_rule_fields():
        """The same tallies with the PDA region of both tests of Sect. 3.1:
        fewer than 100 visits, or photon noise above 5 % (or no absorption) in
        an opaque cell."""
        ctx.update_T()
        st_s = ctx.pda_solve(ctx.region_mask(o.pda_visits, 0.05))
        f = fields(ctx, mcrt)
        return f, st_s

    (T_sig, vis_sig, reg_sig, _), pda_sig = sigma_rule_fields()
    c = counters[-1]
    flops = sum(FLOPS_PER_EVENT[k] * c[k] for k in FLOPS_PER_EVENT)
    traffic, traffic_src = (measured_traffic(TRACE32_KERNELS, N) if a.precision == "fp32"
                            else (None, "counters are taken for the FP32 kernels only"))
    t_trace = float(np.mean(trace_ms)) * 1e-3
    achieved = flops / t_trace
    peak = PEAK[a.precision]
    out = {
        "metric": "photon packets/s (MRW on) at <=1% midplane-T error; batched vs plain",
        "value": N / (ms_step * 1e-3),
        "unit": "photon packets/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "disk 1e-2 Msun, 0.1-100 AU, 100 r x 60 theta cells, 100 lambda "
                               "bins, MRW gamma=3, PDA on cells with <100 visits, %.3g packets "
                               "per step (the count at which the run meets the midplane-T "
                               "condition; the configuration's own 1e6 is c1_1e6_step)" % N,
                   "precision": a.precision, "packets_per_step": N},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": traffic,
                     "traffic_source": traffic_src,
                     "kernel": "trace_%s_kernel + trace_%s_tail_kernel (one mcrt_trace call)"
                               % (a.precision, a.precision),
                     "kernel_ms": float(np.mean(trace_ms)),
                     "flops_per_launch": flops},
        "events_per_step": c,
        "options": (dict(t_opts, calls_per_pass=n_calls) if tuned else "library defaults"),
        "pda": {k: pda[k] for k in ("sweeps", "cg_iters_total", "n_region")},
    }
    if tuned:
        out["autotune"] = {"source": tuned_src, "choice": tuned["options"],
                           **{k: tuned[k] for k in ("shape_s", "trace_s", "handoff_s", "calls_s", "pda_s",
                                                    "pda_iters", "n_packets", "when")
                              if k in tuned}}
    else:
        out["autotune"] = {"source": "no cached choice for this step: library defaults"}
    # the legs after the timed steps, in order of importance; each is skipped
    # (and reported so) when its expected length would pass the budget
    leg_s, skipped = {}, {}

    def leg(name, est_s, fn):
        if elapsed() + est_s > a.budget_s:
            skipped[name] = "expected ~%.0f s at %.0f s elapsed, budget %.0f s" % (
                est_s, elapsed(), a.budget_s)
            log("skipping %s (%s)" % (name, skipped[name]))
            return False
        t = time.perf_counter()
        fn()
        leg_s[name] = time.perf_counter() - t
        return True

    step_s = ms_step * 1e-3
    ref = {}

    def do_ref():
        nref = a.ref_packets if a.ref_packets > 0 else N
        log("reference: FP64, no MRW, %.3g packets in two independent halves" % nref)
        ref["halves"], dt = reference_halves(mcrt, disk, o, nref, torch)
        R1, R2 = ref["halves"]
        err = midplane_error_vs_halves(disk, T_meas, vis_meas, reg_meas, R1, R2)
        err["reference"] = ("FP64, no MRW, same PDA rule, %.3g packets as two independent "
                            "halves of one call each (%.1f s)" % (nref, dt))
        err["run"] = "the last timed step"
        err["pda_rule"] = "visits < 100 (the step's rule)"
        out["midplane_T_error"] = err
        out["meets_1pct_midplane"] = err["meets_1pct"]
        err_s = midplane_error_vs_halves(disk, T_sig, vis_sig, reg_sig, R1, R2)
        err_s["pda_rule"] = ("visits < 100, or noise 1/(4 sqrt N) > 5 % or no absorption in an "
                             "opaque cell (Sect. 3.1), on the same tallies")
        err_s["pda_region_cells"] = pda_sig["n_region"]
        out["midplane_T_error_sigma_rule"] = err_s

    if not a.no_ref:
        # FP64 without MRW takes ~17 times the FP32 step with it
        leg("reference", 17.0 * step_s * (a.ref_packets or N) / N, do_ref)

    def do_c1():
        n1 = o.n_packets
        log("the configuration's own step: %d packets, %d steps" % (n1, a.c1_steps))
        run_once(ctx, n1, o.seed + 31)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(a.c1_steps):
            run_once(ctx, n1, o.seed + 37 + i)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.c1_steps
        c1 = {"value": n1 / dt, "unit": "photon packets/s", "packets": n1,
              "ms_per_step": dt * 1e3, "steps": a.c1_steps}
        if "halves" in ref:
            Tm, vm, rm, _ = fields(ctx, mcrt)
            c1["midplane_T_error"] = midplane_error_vs_halves(disk, Tm, vm, rm, *ref["halves"])
            (Ts, vs, rs, _), st_s = sigma_rule_fields()
            c1["midplane_T_error_sigma_rule"] = midplane_error_vs_halves(disk, Ts, vs, rs,
                                                                         *ref["halves"])
            c1["midplane_T_error_sigma_rule"]["pda_region_cells"] = st_s["n_region"]
        out["c1_1e6_step"] = c1

    if a.c1_steps > 0:
        leg("c1_1e6_step", 3.0 * (a.c1_steps + 1), do_c1)
    del ctx
    torch.cuda.empty_cache()

    def do_c3():
        out["c3"] = c3_full(mcrt, W, torch, a.c3_passes)

    if not a.no_batch:
        leg("c3_batched", 30.0 * a.c3_passes, do_c3)

    def do_cpu():
        log("CPU oracle, %d packets" % a.cpu_packets)
        out["cpu_baseline"] = cpu_baseline(disk, o, a.cpu_packets)

    if not a.no_cpu:
        leg("cpu_baseline", a.cpu_packets / 5e4, do_cpu)

    def do_vertical():
        log("vertical-structure loop to convergence")
        out["vertical_structure"] = vertical_structure(mcrt, W, torch, 10)

    if not a.no_hydro:
        leg("vertical_structure", 40.0, do_vertical)

    def do_sed():
        log("ray-traced SED, MRW against no MRW, 1e6 packets")
        out["sed_study_1e6"] = sed_study(mcrt, W, torch, o.n_packets)

    if not a.no_sed:
        leg("sed_study_1e6", 40.0, do_sed)

    def do_grad():
        log("PDA and adjoint on the differentiation workload")
        out["pda_grad"] = pda_grad(mcrt, W, torch)

    if not a.no_pda:
        leg("pda_grad", 10.0, do_grad)

    def do_plain():
        log("plain FP64 step, %.3g packets" % N)
        ctx64 = mcrt.Context(disk, precision="fp64", mrw=True, gamma=o.gamma,
                             n_int_min=o.n_int_min, pda_visits=o.pda_visits, n_T=o.n_T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_once(ctx64, N, o.seed + 777)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["plain_fp64"] = {"value": N / dt, "ms_per_step": dt * 1e3, "steps": 1,
                             "packets": N}
        if "halves" in ref:
            T64, vis64, reg64, _ = fields(ctx64, mcrt)
            out["plain_fp64"]["midplane_T_error"] = midplane_error_vs_halves(
                disk, T64, vis64, reg64, *ref["halves"])
        del ctx64

    if not a.no_plain and a.precision != "fp64":
        leg("plain_fp64", 3.0 * step_s + 5.0, do_plain)

    def do_c3_plain():
        c3_plain(mcrt, W, torch, out["c3"], a.c3_plain_every)

    if not a.no_batch and "c3" in out and not a.no_plain:
        leg("c3_plain_fp64", 6.0 * (64 // a.c3_plain_every), do_c3_plain)
    out["legs_s"] = leg_s
    out["legs_skipped"] = skipped
    out["wall_s"] = elapsed()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
