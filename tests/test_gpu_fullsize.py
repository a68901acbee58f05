"""The named workloads at their full sizes, in the launch configurations the
benchmark times: what the oracle can check one by one (tables, cell
location, packets under a frozen temperature field) and the properties that
hold at any size (energy conservation, exact integer tallies, converged PDA
regions)."""
import math

import numpy as np
import pytest

from paper_0902_3092_amd import workloads as W

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


def _power_law_T(d, T1=300.0):
    rc = 0.5 * (d.r_edges[:-1] + d.r_edges[1:]) / W.AU
    return np.ascontiguousarray((T1 * rc[:, None] ** -0.5 *
                                 (1 + 0.3 * d.mu_edges[None, 1:])).reshape(-1))


def _energy(ctx, mcrt):
    sed = ctx.sed().cpu().numpy()
    E_star = ctx.get(mcrt.GET_E_STAR).cpu().numpy()[0]
    return (sed.sum() + E_star) / ctx.tables()["L_star"]


@pytest.mark.parametrize("name", ["mrw_pda", "large"])
def test_tables_and_locate_full_size(mcrt, oracle_mod, torch_cuda, name):
    torch = torch_cuda
    d, o = W.config(name)
    ctx = mcrt.Context(d, n_T=o.n_T)
    ora = oracle_mod.Oracle(d, n_T=o.n_T)
    t = ctx.tables()
    nz = ora.cdf > 1e-300
    assert np.allclose(t["cdf"][nz], ora.cdf[nz], rtol=1e-9)
    assert np.allclose(t["Drho"], ora.Drho, rtol=1e-9, atol=0)
    assert np.allclose(t["kbar"], ora.kbar, rtol=1e-9)
    rng = np.random.default_rng(9)
    n = 50000
    r = np.exp(rng.uniform(np.log(d.r_edges[0] * 0.9), np.log(d.r_edges[-1] * 1.1), n))
    mu = np.concatenate([rng.uniform(-1, 1, n // 2),
                         rng.choice(d.mu_edges, n - n // 2) * rng.choice([-1, 1], n - n // 2)])
    ph = rng.uniform(0, 2 * np.pi, n)
    st = np.sqrt(1 - mu * mu)
    xyz = np.ascontiguousarray(np.stack([r * st * np.cos(ph), r * st * np.sin(ph), r * mu], 1))
    got = ctx.locate(torch.from_numpy(xyz).cuda()).cpu().numpy()
    assert np.array_equal(got, ora.locate(xyz))


@pytest.mark.parametrize("name", ["mrw_pda", "large"])
def test_frozen_packets_full_size(mcrt, oracle_mod, torch_cuda, name):
    """FP64 path with MRW on the full grid under a frozen temperature field:
    the same events packet by packet as the oracle for >= 99.9 % of a
    sample of packets taken from the middle of a 1e6-packet run."""
    torch = torch_cuda
    d, o = W.config(name)
    Tf = _power_law_T(d)
    n, off = 3000, 400000
    ctx = mcrt.Context(d, mrw=True, gamma=o.gamma, n_int_min=o.n_int_min, n_T=o.n_T)
    recs = ctx.trace(n, o.seed, n_total=1000000, offset=off,
                     frozen_T=torch.from_numpy(Tf).cuda(), n_recs=n)
    torch.cuda.synchronize()
    g = mcrt.Context.records_numpy(recs)
    ora = oracle_mod.Oracle(d, n_T=o.n_T)
    ref = ora.run(n, o.seed, n_total=1000000, offset=off, frozen_T=Tf, n_recs=n, mrw=True,
                  gamma=o.gamma, n_int_min=o.n_int_min)["recs"]
    same = np.ones(n, bool)
    for f in ("fate", "k", "n_cross", "n_scat", "n_abs", "n_mrw", "n_draws"):
        same &= g[f] == ref[f]
    assert same.mean() >= 0.999, same.mean()
    assert ref["n_mrw"].sum() > 0


def test_bench_step_invariants(mcrt, torch_cuda):
    """The benchmark's timed step (1e-2 Msun disk, 1e6 packets, FP32, MRW,
    T update, PDA on < 100 visits): energy conserved to 1e-6, integer tallies
    sum to the event counters, every packet ends, the PDA converges."""
    torch = torch_cuda
    d, o = W.config("mrw_pda")
    ctx = mcrt.Context(d, precision="fp32", mrw=True, gamma=o.gamma, n_int_min=o.n_int_min,
                       pda_visits=o.pda_visits, n_T=o.n_T)
    ctx.reset()
    ctx.trace(o.n_packets, o.seed)
    ctx.update_T()
    st = ctx.pda_solve()
    torch.cuda.synchronize()
    c = ctx.counters()
    assert c["launch"] == o.n_packets and c["escaped"] + c["star"] == o.n_packets
    assert c["capped"] == 0
    assert 0 < c["handed"] <= 8192   # long walks go to the whole-wavefront launch
    assert _energy(ctx, mcrt) == pytest.approx(1.0, abs=1e-6)
    na = ctx.get(mcrt.GET_N_ABS).cpu().numpy().view(np.uint32).astype(np.int64)
    nm = ctx.get(mcrt.GET_N_MRW).cpu().numpy().view(np.uint32).astype(np.int64)
    assert na.sum() == c["abs"] and nm.sum() == c["mrw"] and c["mrw"] > 0
    reg = ctx.get(mcrt.GET_REGION).cpu().numpy()
    vis = ctx.get(mcrt.GET_VISITS).cpu().numpy().view(np.uint32)
    dusty = d.rho > 0
    assert np.array_equal(reg == 1, dusty & (vis < o.pda_visits) & (reg != 2))
    assert st["converged"] == 1
    T = ctx.get(mcrt.GET_T).cpu().numpy()
    assert np.all(np.isfinite(T)) and np.all(T[reg == 1] > 0)


def test_batched_64_disks_invariants(mcrt, torch_cuda):
    """The 64-disk batched workload at 1 % of its drawn packets, one
    graph-captured pass: every disk conserves energy and traces all its
    packets.  At 1 % of the packets the low-visit region covers most of some
    grids; where its Picard sweeps do not settle (the oracle's do not
    either on such regions) the batch reports MCRT_E_NOT_CONVERGED, and the
    solution still obeys the maximum principle."""
    torch = torch_cuda
    draws = W.batch_draws()
    ctxs = [mcrt.Context(W.batch_disk(b), precision="fp32", mrw=True, gamma=3.0, n_int_min=20,
                         pda_visits=100) for b in draws]
    npk = [max(1000, int(round(b["n_packets"] * 0.01))) for b in draws]
    stats, rc = mcrt.batch_run_rc(ctxs, npk, [b["seed"] for b in draws], n_iter=1,
                                  use_graph=True)
    torch.cuda.synchronize()
    assert rc == (mcrt.OK if all(s["converged"] for s in stats) else mcrt.E_NOT_CONVERGED)
    assert sum(s["converged"] for s in stats) >= 60
    for ctx, n, st in zip(ctxs, npk, stats):
        c = ctx.counters()
        assert c["launch"] == n and c["escaped"] + c["star"] == n
        assert _energy(ctx, mcrt) == pytest.approx(1.0, abs=1e-6)
        T = ctx.get(mcrt.GET_T).cpu().numpy()
        assert np.all(np.isfinite(T))
        reg = ctx.get(mcrt.GET_REGION).cpu().numpy()
        if st["n_region"] > 0:
            # maximum principle: region temperatures within the Monte Carlo range
            T_pda = T.copy()
            ctx.update_T()
            T_mc = ctx.get(mcrt.GET_T).cpu().numpy()
            bc = (reg != 1) & (T_mc > 0)
            assert T_pda[reg == 1].min() >= T_mc[bc].min() * (1 - 1e-6)
            assert T_pda[reg == 1].max() <= T_mc[bc].max() * (1 + 1e-6)
