"""GPU (HIP, through the C-ABI) against the CPU oracle on the same seeded inputs.

Deterministic parity: tables, cell location (bit-exact), temperature
inversion, frozen-temperature transport packet by packet, and the PDA solve
on an identical region.  Statistical parity: immediate-reemission runs (the
GPU's concurrency orders absorptions differently), with the tolerances of the
method's photon noise.
"""
import math
import os

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


def _frozen_field(d, T1=300.0):
    rc = 0.5 * (d.r_edges[:-1] + d.r_edges[1:]) / W.AU
    T = T1 * rc[:, None] ** -0.5 * (1 + 0.3 * d.mu_edges[None, 1:])
    return np.ascontiguousarray(T.reshape(-1))


def test_tables_match_oracle(mcrt, oracle_mod):
    """Planck bin integrals (series vs quadrature), the emission CDF and the
    diffusion means (closed form vs the eta iteration) agree."""
    d = W.make_disk("t", M_dust_msun=1e-3, n_r=8, n_mu=6, n_lambda=40,
                    species=((1.0, 0.3), (0.3, 0.5), (0.1, 0.7)))
    ctx = mcrt.Context(d, n_T=96)
    ora = oracle_mod.Oracle(d, n_T=96)
    t = ctx.tables()
    assert np.array_equal(t["T"], ora.T_nodes) or np.allclose(t["T"], ora.T_nodes, rtol=1e-15)
    nz = ora.cdf > 1e-300
    assert np.allclose(t["cdf"][nz], ora.cdf[nz], rtol=1e-9)
    assert np.allclose(t["Drho"], ora.Drho, rtol=1e-9, atol=0)
    assert np.allclose(t["kbar"], ora.kbar, rtol=1e-9)
    assert np.allclose(t["star_cdf"], ora.star_cdf, rtol=1e-10)
    assert t["L_star"] == pytest.approx(ora.L_star, rel=1e-14)


def test_locate_bit_exact(mcrt, oracle_mod, torch_cuda):
    torch = torch_cuda
    d = W.small_disk(n_r=23, n_mu=17)
    ctx = mcrt.Context(d)
    ora = oracle_mod.Oracle(d)
    rng = np.random.default_rng(5)
    n = 20000
    r = np.exp(rng.uniform(np.log(d.r_edges[0] * 0.7), np.log(d.r_edges[-1] * 1.3), n))
    mu = rng.uniform(-1, 1, n)
    ph = rng.uniform(0, 2 * np.pi, n)
    st = np.sqrt(1 - mu * mu)
    pts = [np.stack([r * st * np.cos(ph), r * st * np.sin(ph), r * mu], 1)]
    # points on the faces: spheres along the axes, cones in the x-z plane
    for e in range(d.n_r + 1):
        re_ = d.r_edges[e]
        pts.append(np.array([[re_, 0, 0], [0, re_, 0], [0, 0, re_], [0, 0, -re_]]))
        for m in d.mu_edges:
            pts.append(np.array([[re_ * math.sqrt(1 - m * m), 0, re_ * m],
                                 [re_ * math.sqrt(1 - m * m), 0, -re_ * m]]))
    xyz = np.ascontiguousarray(np.concatenate(pts))
    got = ctx.locate(torch.from_numpy(xyz).cuda()).cpu().numpy()
    want = ora.locate(xyz)
    assert np.array_equal(got, want)


def test_update_T_matches_oracle(mcrt, oracle_mod, torch_cuda):
    torch = torch_cuda
    d, _ = W.config("plain")
    ctx = mcrt.Context(d)
    ora = oracle_mod.Oracle(d)
    ctx.trace(20000, 3)
    torch.cuda.synchronize()
    E = ctx.get(mcrt.GET_E_ABS).cpu().numpy()
    T_gpu = ctx.update_T().cpu().numpy()
    T_ora = ora.update_T(E)
    assert np.allclose(T_gpu, T_ora, rtol=1e-12, atol=0)


@pytest.mark.parametrize("mrw", [False, True])
def test_frozen_T_packet_parity(mcrt, oracle_mod, torch_cuda, mrw):
    """With re-emission from a fixed temperature field no packet depends on
    another, so the GPU FP64 path and the oracle follow the same events packet
    by packet (same Philox draws)."""
    torch = torch_cuda
    d = W.small_disk(M_dust_msun=3e-3, n_r=14, n_mu=10, n_lambda=24)
    Tf = _frozen_field(d)
    n = 4000
    kw = dict(mrw=mrw, gamma=2.0, n_int_min=5)
    ctx = mcrt.Context(d, **kw)
    recs = ctx.trace(n, 17, frozen_T=torch.from_numpy(Tf).cuda(), n_recs=n)
    torch.cuda.synchronize()
    g = mcrt.Context.records_numpy(recs)
    ora = oracle_mod.Oracle(d)
    o = ora.run(n, 17, frozen_T=Tf, n_recs=n, mrw=mrw, gamma=2.0, n_int_min=5)["recs"]
    same = ((g["fate"] == o["fate"]) & (g["k"] == o["k"]) & (g["n_cross"] == o["n_cross"]) &
            (g["n_scat"] == o["n_scat"]) & (g["n_abs"] == o["n_abs"]) &
            (g["n_mrw"] == o["n_mrw"]) & (g["n_draws"] == o["n_draws"]))
    assert same.mean() >= 0.999, same.mean()
    pos = np.stack([g["x"], g["y"], g["z"]], 1)
    opos = np.stack([o["x"], o["y"], o["z"]], 1)
    scale = np.linalg.norm(opos, axis=1)
    err = np.linalg.norm(pos - opos, axis=1) / scale
    assert np.mean(err[same] < 1e-9) >= 0.999
    if mrw:
        assert o["n_mrw"].sum() > 100
    # tallies of the frozen run agree too
    c = ctx.counters()
    assert c["launch"] == n and c["escaped"] + c["star"] + c["capped"] == n


def test_energy_conservation_gpu(mcrt, torch_cuda):
    torch = torch_cuda
    d, _ = W.config("plain")
    ctx = mcrt.Context(d)
    ctx.trace(200000, 0)
    torch.cuda.synchronize()
    sed = ctx.sed().cpu().numpy()
    E_star = ctx.get(mcrt.GET_E_STAR).cpu().numpy()[0]
    L = ctx.tables()["L_star"]
    assert (sed.sum() + E_star) / L == pytest.approx(1.0, abs=1e-6)
    c = ctx.counters()
    assert c["escaped"] + c["star"] == 200000 and c["capped"] == 0


def _ensemble(run_fn, seeds):
    Ts, seds = [], []
    for s in seeds:
        T, sed = run_fn(s)
        Ts.append(T)
        seds.append(sed)
    return np.array(Ts), np.array(seds)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_plain_run_statistical_parity(mcrt, oracle_mod, torch_cuda, precision):
    """The plain workload (1e-4 Msun, 40 x 30 cells, 50 bins, 1e5 packets,
    immediate reemission, no MRW/PDA).  Packets absorbed repeatedly in one
    cell make the per-cell photon noise correlated (larger than
    1/(4 sqrt(N_abs))), so both sides run an ensemble of seeds and the
    ensemble means are compared with their empirical standard errors: cell
    temperatures agree to within 4 standard errors and 1 % (mass-weighted
    mean), the SED within 2 % in bins with >= 1e4 packets."""
    torch = torch_cuda
    d, o = W.config("plain")
    K = 6
    ctx = mcrt.Context(d, precision=precision)
    ora = oracle_mod.Oracle(d)
    vis = None

    def gpu(seed):
        nonlocal vis
        ctx.reset()
        ctx.trace(o.n_packets, seed)
        T = ctx.update_T().cpu().numpy()
        vis = ctx.get(mcrt.GET_VISITS).cpu().numpy()
        return T, ctx.sed().cpu().numpy()

    def cpu(seed):
        st = ora.run(o.n_packets, seed)
        return ora.update_T(st["E_abs"]), st["sed"]

    Tg, Sg = _ensemble(gpu, range(100, 100 + K))
    To, So = _ensemble(cpu, range(200, 200 + K))
    mg, mo = Tg.mean(0), To.mean(0)
    se = np.sqrt(Tg.var(0, ddof=1) / K + To.var(0, ddof=1) / K)
    ok = (vis >= 100) & (Tg.min(0) > 0) & (To.min(0) > 0)
    assert ok.sum() > 50
    z = (mg[ok] - mo[ok]) / se[ok]
    assert np.mean(np.abs(z) < 4) > 0.97, np.sort(np.abs(z))[-10:]
    assert abs(np.mean(z)) < 1.0          # no global bias
    # 1 % where the ensembles resolve it, else 4 standard errors
    rel = np.abs(mg[ok] / mo[ok] - 1)
    se_rel = se[ok] / mo[ok]
    assert np.mean(rel < np.maximum(0.01, 4 * se_rel)) > 0.97
    w = ora.mass[ok]
    assert np.sum(w * rel) / w.sum() < max(0.01, 2 * np.sum(w * se_rel) / w.sum())
    # SED: escaped luminosity per wavelength bin and per inclination bin,
    # ensemble totals; bins holding >= 1e4 packets on both sides within 2 %
    eps = ora.L_star / o.n_packets
    for axis in (2, 1):
        sg, so = Sg.sum(0).sum(axis - 1) / eps, So.sum(0).sum(axis - 1) / eps
        big = (sg >= 1e4) & (so >= 1e4)
        assert big.sum() >= 5
        tol = np.maximum(0.02, 4 * np.sqrt(1 / sg[big] + 1 / so[big]))
        assert np.all(np.abs(sg[big] / so[big] - 1) < tol)
    assert Sg.sum(axis=(1, 2)).mean() == pytest.approx(So.sum(axis=(1, 2)).mean(), rel=2e-3)


@pytest.mark.parametrize("solver", [1, 2])
def test_pda_matches_oracle_cholesky(mcrt, oracle_mod, torch_cuda, solver):
    """Same region and Dirichlet temperatures: the GPU Jacobi-PCG with Picard
    sweeps reproduces the oracle's banded-Cholesky Picard solution."""
    torch = torch_cuda
    d = W.make_disk("p", M_dust_msun=1e-2, n_r=40, n_mu=30, n_lambda=30)
    rng = np.random.default_rng(4)
    rc = 0.5 * (d.r_edges[:-1] + d.r_edges[1:]) / W.AU
    T_mc = (400 * rc[:, None] ** -0.5 * (1 + rng.uniform(0, 0.2, (d.n_r, d.n_mu)))).reshape(-1)
    mask = np.zeros((d.n_r, d.n_mu), np.uint8)
    mask[5:35, 0:12] = 1
    mask[20:24, 12:16] = 1
    ctx = mcrt.Context(d, pda_solver=solver)
    ctx.set_T(torch.from_numpy(T_mc).cuda())
    st = ctx.pda_solve(torch.from_numpy(mask.reshape(-1)).cuda())
    T_g = ctx.get(mcrt.GET_T).cpu().numpy()
    reg_g = ctx.get(mcrt.GET_REGION).cpu().numpy()
    ora = oracle_mod.Oracle(d)
    T_o, reg_o, sweeps, ch = ora.pda(T_mc, mask.reshape(-1))
    assert np.array_equal(reg_g, reg_o)
    assert st["sweeps"] >= 2 and st["last_change"] < 1e-8
    assert np.allclose(T_g, T_o, rtol=1e-7)


def test_fp32_frozen_tallies_match_fp64(mcrt, torch_cuda):
    """FP32 cell-relative tracking against the FP64 path on a frozen
    temperature field with MRW: seed ensembles on both sides; absorbed energy
    per cell agrees within 4 empirical standard errors (97 % of cells with
    >= 400 absorptions), SED bins within max(2 %, 4 sigma), MRW step counts
    within 5 %, energy conserved in every run."""
    torch = torch_cuda
    d = W.small_disk(M_dust_msun=3e-3, n_r=14, n_mu=10, n_lambda=24)
    Tf = torch.from_numpy(_frozen_field(d)).cuda()
    K, n = 6, 100000
    res = {}
    for prec in ("fp64", "fp32"):
        ctx = mcrt.Context(d, precision=prec, mrw=True, gamma=2.0, n_int_min=5)
        L = ctx.tables()["L_star"]
        Es, Ns, Ss, mrw = [], [], [], 0
        for kseed in range(K):
            ctx.reset()
            ctx.trace(n, 500 + kseed + (0 if prec == "fp64" else 100), frozen_T=Tf)
            torch.cuda.synchronize()
            Es.append(ctx.get(mcrt.GET_E_ABS).cpu().numpy())
            Ns.append(ctx.get(mcrt.GET_N_ABS).cpu().numpy())
            sed = ctx.sed().cpu().numpy()
            Ss.append(sed)
            E_star = ctx.get(mcrt.GET_E_STAR).cpu().numpy()[0]
            assert (sed.sum() + E_star) / L == pytest.approx(1.0, abs=1e-6)
            mrw += ctx.counters()["mrw"]
        res[prec] = (np.array(Es), np.array(Ns), np.array(Ss), mrw)
    E64, N64, S64, m64 = res["fp64"]
    E32, N32, S32, m32 = res["fp32"]
    ok = (N64.mean(0) >= 400) & (N32.mean(0) >= 400)
    assert ok.sum() > 20
    se = np.sqrt(E64.var(0, ddof=1) / K + E32.var(0, ddof=1) / K)
    z = (E32.mean(0) - E64.mean(0))[ok] / se[ok]
    assert np.mean(np.abs(z) < 4) > 0.97, np.sort(np.abs(z))[-5:]
    eps = L / n
    s64, s32 = S64.sum(0).sum(1) / eps, S32.sum(0).sum(1) / eps
    big = (s64 >= 1e4) & (s32 >= 1e4)
    assert big.sum() >= 5
    tol = np.maximum(0.02, 4 * np.sqrt(1 / s64[big] + 1 / s32[big]))
    assert np.all(np.abs(s32[big] / s64[big] - 1) < tol)
    assert m32 > 0 and abs(m32 / m64 - 1) < 0.05


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_integer_tallies_exact(mcrt, torch_cuda, precision):
    """Integer tallies, however they are accumulated on the device (per-lane
    counts per cell stay, workgroup histograms in LDS): per-cell absorption
    and MRW counts sum to the event counters, and a frozen-temperature run
    (deterministic per packet) gives bit-identical visit, absorption and MRW
    counts when repeated; visits never exceed crossings."""
    torch = torch_cuda
    d = W.small_disk(M_dust_msun=3e-3, n_r=14, n_mu=10, n_lambda=24)
    Tf = torch.from_numpy(_frozen_field(d)).cuda()
    ctx = mcrt.Context(d, precision=precision, mrw=True, gamma=2.0, n_int_min=5)
    runs = []
    for _ in range(2):
        ctx.reset()
        ctx.trace(60000, 77, frozen_T=Tf)
        torch.cuda.synchronize()
        c = ctx.counters()
        v = ctx.get(mcrt.GET_VISITS).cpu().numpy().view(np.uint32).astype(np.int64)
        na = ctx.get(mcrt.GET_N_ABS).cpu().numpy().view(np.uint32).astype(np.int64)
        nm = ctx.get(mcrt.GET_N_MRW).cpu().numpy().view(np.uint32).astype(np.int64)
        assert na.sum() == c["abs"] and nm.sum() == c["mrw"]
        assert 0 < v.sum() <= c["cross"] + c["launch"]
        assert c["mrw"] > 0
        runs.append((v, na, nm))
    for a, b in zip(runs[0], runs[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("mrw", [False, True])
def test_wave_mode_same_events(mcrt, torch_cuda, mrw, precision):
    """The whole-wavefront mode (the last live packet of a wavefront traced by
    all 64 lanes) follows the same events as the per-lane mode: packets traced
    one per launch (so each runs in wave mode after its first event) against
    the same packets in one launch with the mode off, frozen temperature."""
    torch = torch_cuda
    d = W.small_disk(M_dust_msun=1e-1, n_r=14, n_mu=10, n_lambda=24)
    Tf = torch.from_numpy(_frozen_field(d)).cuda()
    n = 300
    kw = dict(precision=precision, mrw=mrw, gamma=2.0, n_int_min=5)
    lanes = mcrt.Context(d, wave_events=0, **kw)
    ref = mcrt.Context.records_numpy(lanes.trace(n, 31, n_total=n, frozen_T=Tf, n_recs=n))
    wave = mcrt.Context(d, wave_events=1, **kw)
    got = []
    for p in range(n):
        r = wave.trace(1, 31, n_total=n, offset=p, frozen_T=Tf, n_recs=1)
        got.append(mcrt.Context.records_numpy(r)[0])
    torch.cuda.synchronize()
    got = np.array(got, dtype=ref.dtype)
    same = np.ones(n, bool)
    for f in ("fate", "k", "n_cross", "n_scat", "n_abs", "n_mrw", "n_draws"):
        same &= got[f] == ref[f]
    assert same.mean() >= 0.99, same.mean()
    assert (ref["n_scat"] + ref["n_abs"]).sum() > 2 * n
    if mrw:
        assert ref["n_mrw"].sum() > 0
    pos = np.stack([got["x"], got["y"], got["z"]], 1)
    rpos = np.stack([ref["x"], ref["y"], ref["z"]], 1)
    err = np.linalg.norm(pos - rpos, axis=1) / np.linalg.norm(rpos, axis=1)
    assert np.mean(err[same] < 1e-5) >= 0.99


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_mrw_coefficients_from_current_T(mcrt, torch_cuda, precision):
    """mrw_coef_T = 1: a trace takes the MRW coefficients from the temperature
    the context holds when it starts (after mcrt_update_T, or as set by
    mcrt_set_T).  Packets traced one per launch are deterministic, so the
    same field gives the same events and another field other events."""
    torch = torch_cuda
    d = W.small_disk(M_dust_msun=1e-1, n_r=14, n_mu=10, n_lambda=24)
    kw = dict(precision=precision, mrw=True, gamma=2.0, n_int_min=5, mrw_coef_T=1,
              wave_events=0)
    n = 150

    def sequence(ctx):
        ctx.reset()
        out = []
        for p in range(n):
            r = ctx.trace(1, 77, n_total=n, offset=p, n_recs=1)
            out.append(mcrt.Context.records_numpy(r)[0])
        torch.cuda.synchronize()
        return np.array(out, dtype=out[0].dtype)

    def same(a, b):
        return all(np.array_equal(a[f], b[f]) for f in ("fate", "k", "n_cross", "n_scat",
                                                          "n_abs", "n_mrw", "n_draws"))

    # a pass, then its temperature
    a = mcrt.Context(d, **kw)
    a.reset()
    a.trace(20000, 5)
    a.update_T()
    T1 = a.get(mcrt.GET_T).clone()
    got_a = sequence(a)
    # the same field set by hand on a fresh context
    b = mcrt.Context(d, **kw)
    b.set_T(T1)
    got_b = sequence(b)
    assert same(got_a, got_b)
    assert got_a["n_mrw"].sum() > 0
    # after a pass, a field set by hand replaces the pass's
    c = mcrt.Context(d, **kw)
    c.reset()
    c.trace(20000, 5)
    c.update_T()
    c.set_T(3.0 * T1)
    got_c = sequence(c)
    e = mcrt.Context(d, **kw)
    e.set_T(3.0 * T1)
    assert same(got_c, sequence(e))
    assert not same(got_a, got_c)


@pytest.mark.parametrize("wave_events", [0, 1])
def test_zero_optical_depth_into_tiny_extinction(mcrt, torch_cuda, wave_events):
    """A packet launched with exactly zero optical depth (its draw rounds to
    1 in FP32) into cells whose FP32 extinction is denormal, so that its
    reciprocal overflows: the flight is 0, the packet interacts where it
    enters and leaves the disk with a finite position (per lane, and in the
    whole-wavefront launch after its first event)."""
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    from test_philox_np import TAU_ZERO_PID, TAU_ZERO_SEED
    torch = torch_cuda
    d = W.small_disk(n_r=12, n_mu=8, n_lambda=16)
    rho = np.full(d.rho.shape, 1e-44)
    ctx = mcrt.Context(d, rho=rho, precision="fp32", mrw=True, max_events=100000,
                       wave_events=wave_events)
    ctx.reset()
    recs = ctx.trace(1, TAU_ZERO_SEED, n_total=TAU_ZERO_PID + 1, offset=TAU_ZERO_PID, n_recs=1)
    torch.cuda.synchronize()
    r = mcrt.Context.records_numpy(recs)[0]
    assert r["fate"] in (1, 2), r
    assert np.all(np.isfinite([r["x"], r["y"], r["z"]]))
    assert r["n_scat"] + r["n_abs"] >= 1
    assert ctx.counters()["capped"] == 0
