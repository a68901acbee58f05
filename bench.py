"""Benchmark of the hot path on one MI355X.

One step = one pass of the whole path over one disk: clear the tallies, trace
1e6 photon packets with immediate reemission and the modified random walk
(gamma = 3, 20 interactions in the cell first), invert the cell temperatures,
and solve the partial diffusion approximation on cells entered by fewer than
100 packets.  Workload: the 1e-2 Msun disk on 0.1-100 AU, 100 r x 60 theta
cells, 100 wavelength bins, kappa ~ 1/lambda beyond 1 micron, albedo 0.5,
midplane radial optical depth 1e5 (inputs synthetic and seeded).

Printed: one JSON line with packets/s of the whole step, the roofline of the
trace kernel (events x FP operations per event, from the HIP-event duration
of the kernel), and the CPU oracle timed on a bounded sample of the same
workload on this host.
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


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--precision", default="fp32", choices=["fp64", "fp32"])
    p.add_argument("--no-plain", action="store_true", help="skip the plain FP64 comparison step")
    p.add_argument("--packets", type=int, default=1000000)
    p.add_argument("--cpu-packets", type=int, default=300000)
    p.add_argument("--no-cpu", action="store_true")
    return p.parse_args()


def cpu_baseline(disk, opts, n_packets):
    """The CPU oracle (single thread) on a bounded sample of the same step."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    ora = oracle.Oracle(disk, n_T=opts.n_T)
    t0 = time.perf_counter()
    st = ora.run(n_packets, opts.seed, mrw=True, gamma=opts.gamma, n_int_min=opts.n_int_min)
    T = ora.update_T(st["E_abs"])
    region = (st["visits"] < opts.pda_visits).astype(np.uint8)
    ora.pda(T, region)
    dt = time.perf_counter() - t0
    return {"value": n_packets / dt, "unit": "photon packets/s", "cores": 1, "kind": "oracle",
            "sample": "%d packets of the same disk (trace + T + PDA), one thread, %.1f s"
                      % (n_packets, dt)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_0902_3092_amd import mcrt
    from paper_0902_3092_amd import workloads as W

    disk, o = W.config("mrw_pda")
    N = a.packets
    ctx = mcrt.Context(disk, precision=a.precision, mrw=True, gamma=o.gamma,
                       n_int_min=o.n_int_min, pda_visits=o.pda_visits, n_T=o.n_T)
    stream = torch.cuda.current_stream()

    def step(i, ev=None):
        ctx.reset()
        if ev is not None:
            ev[0].record(stream)
        ctx.trace(N, o.seed + 1000 * i)
        if ev is not None:
            ev[1].record(stream)
        ctx.update_T()
        return ctx.pda_solve()

    for i in range(a.warmup):
        step(i)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(a.steps)]
    counters = []
    pda = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        pda = step(a.warmup + i, evs[i])
        counters.append(ctx.counters())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / a.steps
    trace_ms = [e0.elapsed_time(e1) for e0, e1 in evs]
    c = counters[-1]
    flops = sum(FLOPS_PER_EVENT[k] * c[k] for k in FLOPS_PER_EVENT)
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
        "config": {"workload": "disk 1e-2 Msun, 100 r x 60 theta cells, 100 lambda bins, "
                               "1e6 packets, MRW gamma=3, PDA on cells with <100 visits",
                   "precision": a.precision, "packets_per_step": N},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "kernel": "trace_%s_kernel" % a.precision,
                     "kernel_ms": float(np.mean(trace_ms)),
                     "flops_per_launch": flops},
        "events_per_step": c,
        "pda": {k: pda[k] for k in ("sweeps", "cg_iters_total", "n_region")},
    }
    if not a.no_plain and a.precision != "fp64":
        # the plain FP64 path on the same step, for comparison (one timed step)
        ctx64 = mcrt.Context(disk, precision="fp64", mrw=True, gamma=o.gamma,
                             n_int_min=o.n_int_min, pda_visits=o.pda_visits, n_T=o.n_T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx64.reset()
        ctx64.trace(N, o.seed + 777)
        ctx64.update_T()
        ctx64.pda_solve()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["plain_fp64"] = {"value": N / dt, "ms_per_step": dt * 1e3, "steps": 1}
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(disk, o, a.cpu_packets)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
