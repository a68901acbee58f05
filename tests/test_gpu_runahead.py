"""Runs of interactions traced lane-parallel in the whole-wavefront launch
(option wave_runahead, FP32 tracking) against the same launch one event at a
time.

A run takes the same decisions as event-at-a-time tracing from the same
tally: the kind of each interaction (albedo draw against the albedo of the
current bin), each reemission bin (the difference spectrum between the
temperatures before and after the deposit, Sect. 2.1), the positions flight
by flight, the first face crossing or start of the MRW (Sect. 2.2.2), and the
cell's tally after the run's deposits.  Packets traced one per launch move to
the whole-wavefront launch after their first event, so each packet's walk is
compared, with its draws (the record's draw count).

* Frozen temperature: packet by packet, and the tallies when every packet
  agrees.
* Running temperature: each packet starts from the tallies the earlier ones
  left, so the comparison is on the packets before the first that differs,
  with the absorbed energy of every cell after them; with MRW coefficients
  from the running cell temperature and from a fixed field.
* Many packets in one launch (hand-offs from the per-lane launch, runs that
  find another packet's deposit in their cell and are redone): energy is
  conserved and the handed-off walks' interactions ran mostly in runs.
"""
import os
import sys

import numpy as np
import pytest

from paper_0902_3092_amd import workloads as W

sys.path.insert(0, os.path.dirname(__file__))
from frozen_runs import same_records  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def mcrt(torch_cuda):
    from paper_0902_3092_amd import mcrt as M
    M.lib()
    return M


def _frozen_field(d, T1=300.0):
    rc = 0.5 * (d.r_edges[:-1] + d.r_edges[1:]) / W.AU
    T = T1 * rc[:, None] ** -0.5 * (1 + 0.3 * d.mu_edges[None, 1:])
    return np.ascontiguousarray(T.reshape(-1))


def _thick_disk():
    return W.small_disk(M_dust_msun=1e-1, n_r=14, n_mu=10, n_lambda=24)


def _one_per_launch(mcrt, ctx, n, seed, tallies=False, **kw):
    recs, E = [], []
    for p in range(n):
        r = ctx.trace(1, seed, n_total=n, offset=p, n_recs=1, **kw)
        recs.append(mcrt.Context.records_numpy(r)[0])
        if tallies:
            E.append(ctx.get(mcrt.GET_E_ABS).cpu().numpy())
    return np.array(recs, dtype=recs[0].dtype), E


def _interactions(c):
    return c["scat"] + c["abs"]


@pytest.mark.parametrize("mrw", [False, True])
def test_runs_follow_the_same_events_frozen_T(mcrt, torch_cuda, mrw):
    torch = torch_cuda
    d = _thick_disk()
    Tf = torch.from_numpy(_frozen_field(d)).cuda()
    n = 300
    kw = dict(precision="fp32", mrw=mrw, gamma=2.0, n_int_min=5, wave_events=1)
    serial = mcrt.Context(d, wave_runahead=0, **kw)
    runs = mcrt.Context(d, wave_runahead=1, **kw)
    serial.reset()
    runs.reset()
    a, _ = _one_per_launch(mcrt, serial, n, 31, frozen_T=Tf)
    b, _ = _one_per_launch(mcrt, runs, n, 31, frozen_T=Tf)
    torch.cuda.synchronize()
    cs, cr = serial.counters(), runs.counters()
    print("serial", cs, "runs", cr)
    assert cs["in_runs"] == 0
    assert cr["in_runs"] > 0.5 * _interactions(cr)
    same = same_records(a, b)
    assert same.mean() >= 0.99, same.mean()
    if mrw:
        assert b["n_mrw"].sum() > 0
    pa = np.stack([a["x"], a["y"], a["z"]], 1)
    pb = np.stack([b["x"], b["y"], b["z"]], 1)
    assert np.array_equal(pa[same], pb[same])
    if same.all():
        for what in (mcrt.GET_VISITS, mcrt.GET_N_ABS, mcrt.GET_N_MRW):
            assert torch.equal(serial.get(what), runs.get(what))
        Ea = serial.get(mcrt.GET_E_ABS).cpu().numpy()
        Eb = runs.get(mcrt.GET_E_ABS).cpu().numpy()
        assert np.array_equal(Ea, Eb)


@pytest.mark.parametrize("coef_T", [0, 1])
def test_runs_follow_the_same_events_running_T(mcrt, torch_cuda, coef_T):
    torch = torch_cuda
    d = _thick_disk()
    N, seed = 300, 19
    kw = dict(precision="fp32", mrw=True, gamma=2.0, n_int_min=5, wave_events=1,
              mrw_coef_T=coef_T)
    out = {}
    for ra in (0, 1):
        ctx = mcrt.Context(d, wave_runahead=ra, **kw)
        if coef_T:
            ctx.set_T(torch.from_numpy(_frozen_field(d, 200.0)).cuda())
        ctx.reset()
        recs, E = _one_per_launch(mcrt, ctx, N, seed, tallies=True)
        torch.cuda.synchronize()
        out[ra] = (recs, E, ctx.counters())
    (a, Ea, cs), (b, Eb, cr) = out[0], out[1]
    print("serial", cs, "runs", cr)
    assert cs["in_runs"] == 0
    assert cr["in_runs"] > 0.5 * _interactions(cr)
    same = same_records(a, b)
    m = N if same.all() else int(np.argmin(same))
    print("packets agreeing before the first difference: %d of %d" % (m, N))
    assert m >= 0.97 * N, m
    assert a["n_abs"][:m].sum() > 200 and a["n_mrw"][:m].sum() > 20
    # the tallies after the agreeing packets: deposit for deposit
    assert np.array_equal(Ea[m - 1], Eb[m - 1])


def test_runs_in_a_full_launch_conserve_energy(mcrt, torch_cuda):
    torch = torch_cuda
    d = _thick_disk()
    kw = dict(precision="fp32", mrw=True, gamma=2.0, n_int_min=5, wave_events=64)
    res = {}
    for ra in (0, 1):
        ctx = mcrt.Context(d, wave_runahead=ra, **kw)
        ctx.reset()
        ctx.trace(40000, 5)
        torch.cuda.synchronize()
        c = ctx.counters()
        sed = ctx.sed().cpu().numpy()
        E_star = float(ctx.get(mcrt.GET_E_STAR).cpu()[0])
        L = float(ctx.tables()["L_star"])
        assert c["capped"] == 0
        assert (sed.sum() + E_star) / L == pytest.approx(1.0, abs=1e-9)
        res[ra] = c
    c0, c1 = res[0], res[1]
    print("serial", c0, "runs", c1)
    assert c1["handed"] > 0 and c1["in_runs"] > 0
    assert c0["in_runs"] == 0
    # most interactions of the handed-off walks (which carry most of the
    # launch's interactions) ran in runs; the totals of one launch are set by
    # its few longest walks, so they are not compared between the two
    assert c1["in_runs"] > 0.3 * _interactions(c1)
