"""Anisotropic (Henyey-Greenstein) scattering on the GPU against the oracle:
the diffusion tables with the isotropic-equivalent scattering opacity
(1 - g) sigma, frozen-temperature packets event by event (FP64), the same
events in the per-lane and whole-wavefront modes, and ensembles of running
immediate-reemission runs (FP32 and FP64) against the oracle's."""
import numpy as np
import pytest

from paper_0902_3092_amd import workloads as W

pytestmark = pytest.mark.gpu

G = 0.6


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
    return np.ascontiguousarray((T1 * rc[:, None] ** -0.5 * (1 + 0.3 * d.mu_edges[None, 1:])).reshape(-1))


def test_tables_match_oracle_with_g(mcrt, oracle_mod):
    d = W.make_disk("t", M_dust_msun=1e-3, n_r=8, n_mu=6, n_lambda=40,
                    species=((1.0, 0.3), (0.3, 0.5), (0.1, 0.7)))
    t = mcrt.Context(d, n_T=96, g_asym=G).tables()
    ora = oracle_mod.Oracle(d, n_T=96, g_asym=G)
    assert np.allclose(t["Drho"], ora.Drho, rtol=1e-9, atol=0)
    assert np.allclose(t["kbar"], ora.kbar, rtol=1e-9)
    # the scattering opacity enters D: with g it is larger than without
    assert np.all(t["Drho"][1:] > mcrt.Context(d, n_T=96).tables()["Drho"][1:])


@pytest.mark.parametrize("mrw,gg", [(False, G), (True, G), (True, -0.4)])
def test_frozen_T_packet_parity_hg(mcrt, oracle_mod, torch_cuda, mrw, gg):
    torch = torch_cuda
    d = W.small_disk(M_dust_msun=3e-3, n_r=14, n_mu=10, n_lambda=24)
    Tf = _frozen_field(d)
    n = 4000
    ctx = mcrt.Context(d, mrw=mrw, gamma=2.0, n_int_min=5, g_asym=gg)
    g = mcrt.Context.records_numpy(ctx.trace(n, 17, frozen_T=torch.from_numpy(Tf).cuda(), n_recs=n))
    torch.cuda.synchronize()
    o = oracle_mod.Oracle(d, g_asym=gg).run(n, 17, frozen_T=Tf, n_recs=n, mrw=mrw, gamma=2.0,
                                            n_int_min=5)["recs"]
    same = np.ones(n, bool)
    for f in ("fate", "k", "n_cross", "n_scat", "n_abs", "n_mrw", "n_draws"):
        same &= g[f] == o[f]
    assert same.mean() >= 0.999, same.mean()
    assert o["n_scat"].sum() > n
    pos = np.stack([g["x"], g["y"], g["z"]], 1)
    opos = np.stack([o["x"], o["y"], o["z"]], 1)
    err = np.linalg.norm(pos - opos, axis=1) / np.linalg.norm(opos, axis=1)
    assert np.mean(err[same] < 1e-9) >= 0.999
    dirs = np.stack([g["u"], g["v"], g["w"]], 1)
    assert np.allclose(np.linalg.norm(dirs, axis=1), 1.0, atol=1e-12)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_wave_mode_same_events_hg(mcrt, torch_cuda, precision):
    torch = torch_cuda
    d = W.small_disk(M_dust_msun=1e-1, n_r=14, n_mu=10, n_lambda=24)
    Tf = torch.from_numpy(_frozen_field(d)).cuda()
    n = 200
    kw = dict(precision=precision, mrw=True, gamma=2.0, n_int_min=5, g_asym=G)
    ref = mcrt.Context.records_numpy(mcrt.Context(d, wave_events=0, **kw).trace(
        n, 31, n_total=n, frozen_T=Tf, n_recs=n))
    wave = mcrt.Context(d, wave_events=1, **kw)
    got = np.array([mcrt.Context.records_numpy(
        wave.trace(1, 31, n_total=n, offset=p, frozen_T=Tf, n_recs=1))[0] for p in range(n)],
        dtype=ref.dtype)
    torch.cuda.synchronize()
    same = np.ones(n, bool)
    for f in ("fate", "k", "n_cross", "n_scat", "n_abs", "n_mrw", "n_draws"):
        same &= got[f] == ref[f]
    assert same.mean() >= 0.99, same.mean()
    assert ref["n_scat"].sum() > n // 2


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_running_statistical_parity_hg(mcrt, oracle_mod, torch_cuda, precision):
    """Immediate reemission on the plain workload with g = 0.6: ensembles of
    seeds on both sides; cell temperatures within 4 standard errors (97 % of
    cells with >= 100 visits), no global bias, SED bins within 2 % or 4 sigma,
    energy conserved."""
    torch = torch_cuda
    d, o = W.config("plain")
    K, n = 4, 100000
    ctx = mcrt.Context(d, precision=precision, g_asym=G)
    ora = oracle_mod.Oracle(d, g_asym=G)
    Tg, Sg, To, So = [], [], [], []
    vis = None
    for s in range(K):
        ctx.reset()
        ctx.trace(n, 300 + s)
        Tg.append(ctx.update_T().cpu().numpy())
        Sg.append(ctx.sed().cpu().numpy())
        vis = ctx.get(mcrt.GET_VISITS).cpu().numpy()
        E_star = ctx.get(mcrt.GET_E_STAR).cpu().numpy()[0]
        assert (Sg[-1].sum() + E_star) / ora.L_star == pytest.approx(1.0, abs=1e-6)
        st = ora.run(n, 400 + s)
        To.append(ora.update_T(st["E_abs"]))
        So.append(st["sed"])
    Tg, To, Sg, So = map(np.array, (Tg, To, Sg, So))
    se = np.sqrt(Tg.var(0, ddof=1) / K + To.var(0, ddof=1) / K)
    ok = (vis >= 100) & (Tg.min(0) > 0) & (To.min(0) > 0) & (se > 0)
    assert ok.sum() > 50
    z = (Tg.mean(0)[ok] - To.mean(0)[ok]) / se[ok]
    assert np.mean(np.abs(z) < 4) > 0.97, np.sort(np.abs(z))[-10:]
    assert abs(np.mean(z)) < 1.0
    eps = ora.L_star / n
    sg, so = Sg.sum(0).sum(1) / eps, So.sum(0).sum(1) / eps
    big = (sg >= 1e4) & (so >= 1e4)
    assert big.sum() >= 5
    assert np.all(np.abs(sg[big] / so[big] - 1) < np.maximum(0.02, 4 * np.sqrt(1 / sg[big] + 1 / so[big])))


def test_batch_rejects_anisotropic_contexts(mcrt):
    d = W.small_disk(M_dust_msun=1e-3, n_r=8, n_mu=6, n_lambda=16)
    ctx = mcrt.Context(d, precision="fp32", g_asym=0.5)
    with pytest.raises(mcrt.McrtError):
        mcrt.batch_run([ctx], [1000], [1], n_iter=1)


def test_g_out_of_range_is_refused(mcrt):
    d = W.small_disk(M_dust_msun=1e-3, n_r=8, n_mu=6, n_lambda=16)
    with pytest.raises(mcrt.McrtError):
        mcrt.Context(d, g_asym=1.0)
