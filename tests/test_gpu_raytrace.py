"""Observables by integration of the source function on the device (Sect.
2.3, Sect. 3.3) against the oracle:

* the path-length tallies and the mean intensity they give, on frozen-T
  runs of the 1e-2 Msun workload that both sides trace packet for packet
  (MRW on, so the walk's path and its spectrum weights are covered);
* the ray-traced SED from the same temperature and mean intensity, at three
  inclinations, ray for ray the same quadrature;
* the optically thin isothermal shell against its closed form;
* the ray-traced image (the intensity of every ray) of the same disk and of
  the 1e-2 Msun workload's grid, ray for ray against the oracle, and summed
  with the rays' areas against the ray-traced SED;
* visibility amplitudes of an image (the oracle's, on both sides) at several
  baselines, position angles and inclinations against the oracle's, and the
  argument checks of the entry point.
"""
import math
import os
import sys

import numpy as np
import pytest

from paper_0902_3092_amd import workloads as W

sys.path.insert(0, os.path.dirname(__file__))
from frozen_runs import agreeing_runs  # noqa: E402

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


def _field(d):
    rc = 0.5 * (d.r_edges[:-1] + d.r_edges[1:]) / W.AU
    mc = 0.5 * (d.mu_edges[:-1] + d.mu_edges[1:])
    return np.ascontiguousarray((400.0 * rc[:, None] ** -0.5 * (1 + 0.5 * mc[None, :])).reshape(-1))


def test_mean_intensity_matches_oracle(mcrt, oracle_mod, torch_cuda):
    """FP64 tracking flies the oracle's lengths up to rounding: positions
    agree to ~1e-11 relative, and a face distance taken just after a crossing
    loses digits to cancellation, so a few cells' sums differ at ~1e-8."""
    torch = torch_cuda
    precision, rtol = "fp64", 1e-7
    d, o = W.config("mrw_pda")
    Tf = _field(d)
    kw = dict(mrw=True, gamma=o.gamma, n_int_min=o.n_int_min)
    make = lambda: mcrt.Context(d, precision=precision, j_tally=1, **kw)
    ora = oracle_mod.Oracle(d)
    ctx, st, agree = agreeing_runs(mcrt, make, ora, 20000, 71, Tf, torch, paths=True, **kw)
    assert agree >= 0.999
    assert st["mrw_path"].sum() > 0
    # the tallies themselves, then the mean intensity they give
    Pg = ctx.get(mcrt.GET_PATH).cpu().numpy().reshape(st["path"].shape)
    Mg = ctx.get(mcrt.GET_MRW_PATH).cpu().numpy()
    for name, g, w in (("path", Pg, st["path"]), ("mrw_path", Mg, st["mrw_path"])):
        bad = ~np.isclose(g, w, rtol=rtol, atol=1e-12 * w.max())
        if bad.any():
            idx = np.argsort(-np.abs(g - w).reshape(-1) / (np.abs(w).reshape(-1) + 1e-300))[:5]
            print(name, "differs at", [(int(i), float(g.reshape(-1)[i]), float(w.reshape(-1)[i]))
                                       for i in idx])
        assert not bad.any(), name
    Jg = ctx.mean_intensity(torch.from_numpy(Tf).cuda()).cpu().numpy()
    Jo = ora.mean_intensity(Tf, st)
    bad = ~np.isclose(Jg, Jo, rtol=rtol, atol=1e-12 * Jo.max())
    if bad.any():
        i = np.argwhere(bad)[:5]
        print("J differs at (cell, bin, gpu, oracle, mrw path):",
              [(int(c), int(k), float(Jg[c, k]), float(Jo[c, k]), float(Mg[c])) for c, k in i])
    assert not bad.any()
    # the MRW cells' share is there on both sides
    m = st["n_mrw"] > 0
    assert m.sum() > 50 and Jo[m].sum() > 0


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_tallies_against_their_definitions(mcrt, oracle_mod, torch_cuda, precision):
    """Frozen temperatures at table nodes, MRW on, FP32 and FP64 tracking
    (which follow the oracle packet for packet only in FP64), against what
    the tallies are by definition:
    * the split tally is the absorbed energy of the odd-numbered packets
      traced alone (one per launch; frozen T keeps the packets apart);
    * every MRW deposit is rho kappa-bar times the walk's path (kappa-bar at
      a node is exact), so the MRW path tally carries the deposits;
    * the flights' path-length estimate of the absorbed energy,
      sum_k rho kappa_k P_k, agrees with the count estimate eps N_abs within
      the photon noise."""
    torch = torch_cuda
    d, o = W.config("mrw_pda")
    tb = mcrt.Context(d).tables()
    nodes = tb["T"]
    rng = np.random.default_rng(8)
    Tf = np.ascontiguousarray(nodes[rng.integers(len(nodes) // 3, 2 * len(nodes) // 3,
                                                 d.n_cells)])
    Tg = torch.from_numpy(Tf).cuda()
    kw = dict(precision=precision, mrw=True, gamma=o.gamma, n_int_min=o.n_int_min)
    n, seed = 10000, 41
    full = mcrt.Context(d, conv_split=1, j_tally=1, **kw)
    full.reset()
    full.trace(n, seed, frozen_T=Tg)
    odd = mcrt.Context(d, **kw)
    odd.reset()
    for p in range(1, n, 2):
        odd.trace(1, seed, n_total=n, offset=p, frozen_T=Tg)
    torch.cuda.synchronize()
    E_half = full.get(mcrt.GET_E_HALF).cpu().numpy()
    assert np.allclose(E_half, odd.get(mcrt.GET_E_ABS).cpu().numpy(), rtol=1e-12, atol=0)
    eps = tb["L_star"] / n
    E = full.get(mcrt.GET_E_ABS).cpu().numpy()
    n_abs = full.get(mcrt.GET_N_ABS).cpu().numpy().view(np.uint32).astype(np.float64)
    mrw = full.get(mcrt.GET_MRW_PATH).cpu().numpy()
    path = full.get(mcrt.GET_PATH).cpu().numpy().reshape(d.n_cells, d.n_lambda)
    kbar = np.interp(Tf, nodes, tb["kbar"])
    m = mrw > 0
    assert m.sum() >= 5
    assert np.allclose(E[m] - eps * n_abs[m], d.rho[m] * kbar[m] * mrw[m], rtol=1e-9, atol=0)
    kabs = d.kappa_abs[0]
    by_path = (d.rho[:, None] * kabs[None, :] * path).sum()
    by_count = eps * n_abs.sum()
    print(precision, "absorbed energy from the paths / from the counts: %.4f"
          % (by_path / by_count))
    assert by_path / by_count == pytest.approx(1.0, abs=0.03)


def test_raytrace_sed_matches_oracle(mcrt, oracle_mod, torch_cuda):
    """A 30 x 20 disk of 1e-3 Msun, 30 bins: the temperature field of the
    frozen runs and a scattering source J = 0.3 B(T); the same rays on both
    sides (2 rings per radial cell, 8 azimuths)."""
    torch = torch_cuda
    d = W.make_disk("ray", M_dust_msun=1e-3, n_r=30, n_mu=20, n_lambda=30)
    T = _field(d)
    ora = oracle_mod.Oracle(d)
    ctx = mcrt.Context(d)
    # J = 0.3 B(T) per cell, from the oracle's tables: B_k = (cdf_k - cdf_k-1) / kappa_abs,k
    # at the nearest lower node is enough for a test input
    nodes = ora.T_nodes
    idx = np.clip(np.searchsorted(nodes, T) - 1, 0, len(nodes) - 1)
    cdf = ora.cdf
    kB = np.diff(np.concatenate([np.zeros((len(nodes), 1)), cdf], axis=1), axis=1)
    J = np.ascontiguousarray(0.3 * kB[idx] / d.kappa_abs[0][None, :])
    ci = [0.05, 0.5, 0.95]
    Lo = ora.raytrace_sed(T, J=J, cos_i=ci, n_sub=2, n_phi=8)
    Lg = ctx.raytrace_sed(torch.from_numpy(T).cuda(), torch.from_numpy(J).cuda(), cos_i=ci,
                          n_sub=2, n_phi=8).cpu().numpy()
    big = Lo > 1e-12 * Lo.max()
    assert big.sum() > 60
    assert np.allclose(Lg[big], Lo[big], rtol=1e-8, atol=0), np.max(np.abs(Lg[big] / Lo[big] - 1))
    # the edge-on view is dimmer in the optical than the pole-on one
    assert Lo[0, 5] < Lo[2, 5]


def test_raytrace_thin_shell_closed_form(mcrt, oracle_mod, torch_cuda):
    torch = torch_cuda
    d = W.uniform_shell(1e-19, n_r=10, n_mu=6, n_lambda=12, gray=False, albedo=0.3,
                        R_in_au=1.0, R_out_au=10.0)
    ora = oracle_mod.Oracle(d, n_T=64)
    ctx = mcrt.Context(d, n_T=64)
    T = np.full(ora.n_cells, 150.0)
    L = ctx.raytrace_sed(torch.from_numpy(T).cuda(), cos_i=[0.05, 0.5, 0.95], n_sub=16,
                         n_phi=16).cpu().numpy()
    from test_oracle_raytrace import planck_bins
    Bb = planck_bins(d.lambda_edges, 150.0)
    tau = 1e-19 * (d.kappa_abs[0] + d.kappa_sca[0]) * (d.r_edges[-1] - d.r_edges[0])
    star = ctx.tables()["L_star"] * np.diff(np.concatenate([[0.0], ctx.tables()["star_cdf"]])) \
        * np.exp(-tau)
    dust = 4 * math.pi * ora.mass.sum() * d.kappa_abs[0] * Bb
    big = dust > 1e-8 * star
    for q in range(3):
        got = L[q] - star
        assert np.allclose(got[big], dust[big], rtol=2e-3, atol=0)


def _ray_inputs(ora, d):
    T = _field(d)
    nodes = ora.T_nodes
    idx = np.clip(np.searchsorted(nodes, T) - 1, 0, len(nodes) - 1)
    kB = np.diff(np.concatenate([np.zeros((len(nodes), 1)), ora.cdf], axis=1), axis=1)
    J = np.ascontiguousarray(0.3 * kB[idx] / d.kappa_abs[0][None, :])
    return T, J


def test_raytrace_image_matches_oracle(mcrt, oracle_mod, torch_cuda):
    """The disk, temperature and scattering source of the SED test: every ray's
    intensity at three inclinations against the oracle's, and the image summed
    over its rays (4 pi I times the area each ray carries) plus the dimmed star
    against the ray-traced SED of the same rays."""
    torch = torch_cuda
    d = W.make_disk("ray", M_dust_msun=1e-3, n_r=30, n_mu=20, n_lambda=30)
    ora = oracle_mod.Oracle(d)
    ctx = mcrt.Context(d)
    T, J = _ray_inputs(ora, d)
    ci = [0.05, 0.5, 0.95]
    n_sub, n_phi = 2, 8
    Io = ora.raytrace_image(T, J=J, cos_i=ci, n_sub=n_sub, n_phi=n_phi)
    Tg, Jg = torch.from_numpy(T).cuda(), torch.from_numpy(J).cuda()
    Ig = ctx.raytrace_image(Tg, Jg, cos_i=ci, n_sub=n_sub, n_phi=n_phi).cpu().numpy()
    assert Ig.shape == Io.shape == (3, (d.n_r + 1) * n_sub, n_phi, d.n_lambda)
    scale = np.abs(Io).max()
    big = Io > 1e-12 * scale
    assert big.mean() > 0.3
    assert np.allclose(Ig[big], Io[big], rtol=1e-8, atol=0), np.max(np.abs(Ig[big] / Io[big] - 1))
    assert np.all(np.abs(Ig[~big]) <= 1e-10 * scale)
    # summed with the rays' areas: the SED without the star, which is at
    # most the star's own luminosity per bin
    from test_oracle_raytrace_image import ring_radii
    _, area = ring_radii(d.r_edges, n_sub)
    dust = 4 * math.pi * np.einsum("qrpk,r->qk", Ig, area / n_phi)
    L = ctx.raytrace_sed(Tg, Jg, cos_i=ci, n_sub=n_sub, n_phi=n_phi).cpu().numpy()
    share = np.diff(np.concatenate([[0.0], ctx.tables()["star_cdf"]]))
    star = L - dust
    assert np.all(star >= -1e-9 * L)
    assert np.all(star <= ctx.tables()["L_star"] * share * (1 + 1e-9))


def test_raytrace_image_full_grid(mcrt, oracle_mod, torch_cuda):
    """The 1e-2 Msun workload's grid (100 x 60 cells, 100 bins) seen at 45
    degrees, no scattering source: the image ray for ray against the oracle."""
    torch = torch_cuda
    d, _ = W.config("mrw_pda")
    ora = oracle_mod.Oracle(d)
    ctx = mcrt.Context(d)
    T = _field(d)
    ci, n_sub, n_phi = [0.7071067811865476], 2, 12
    Io = ora.raytrace_image(T, cos_i=ci, n_sub=n_sub, n_phi=n_phi)
    Ig = ctx.raytrace_image(torch.from_numpy(T).cuda(), cos_i=ci, n_sub=n_sub,
                            n_phi=n_phi).cpu().numpy()
    scale = np.abs(Io).max()
    big = Io > 1e-12 * scale
    assert big.mean() > 0.3
    assert np.allclose(Ig[big], Io[big], rtol=1e-8, atol=0), np.max(np.abs(Ig[big] / Io[big] - 1))
    assert np.all(np.abs(Ig[~big]) <= 1e-10 * scale)


def test_visibility_matches_oracle(mcrt, oracle_mod, torch_cuda):
    """The 30 x 20 disk's image at three inclinations (the oracle's, given to
    both sides), 150 pc away, baselines of 0, 100 and 500 m at three position
    angles: every amplitude against the oracle's."""
    torch = torch_cuda
    d = W.make_disk("ray", M_dust_msun=1e-3, n_r=30, n_mu=20, n_lambda=30)
    ora = oracle_mod.Oracle(d)
    ctx = mcrt.Context(d)
    T, J = _ray_inputs(ora, d)
    ci, n_sub, n_phi = [0.05, 0.5, 0.95], 2, 8
    img = ora.raytrace_image(T, J=J, cos_i=ci, n_sub=n_sub, n_phi=n_phi)
    base = [[0.0, 0.0], [1e4, 0.0], [1e4, 1.0], [5e4, 2.0]]
    dist = 150 * 3.0857e18
    Vo = ora.visibility(img, ci, n_sub, n_phi, base, dist)
    Vg = ctx.visibility(torch.from_numpy(img).cuda(), ci, n_sub, n_phi, base, dist).cpu().numpy()
    assert Vg.shape == Vo.shape == (3, 4, d.n_lambda)
    assert np.allclose(Vg, Vo, rtol=1e-10, atol=1e-13), np.max(np.abs(Vg - Vo))
    assert np.allclose(Vo[:, 0, :], 1.0, atol=1e-13)        # zero baseline
    assert Vo[:, 3, :].min() < 0.9                           # resolved somewhere
    with pytest.raises(mcrt.McrtError):
        ctx.visibility(torch.from_numpy(img).cuda(), ci, n_sub, n_phi, [[-1.0, 0.0]], dist)
    with pytest.raises(mcrt.McrtError):
        ctx.visibility(torch.from_numpy(img).cuda(), ci, n_sub, n_phi, base, 0.0)
    # more (inclination, baseline) pairs than a third of the cells: the
    # partial sums would not fit the context's buffer, so the call refuses
    many = [0.5] * 64
    big_img = torch.zeros((64, (d.n_r + 1) * n_sub, n_phi, d.n_lambda), dtype=torch.float64,
                          device="cuda")
    assert 64 * 4 > ctx.n_cells // 3
    with pytest.raises(mcrt.McrtError):
        ctx.visibility(big_img, many, n_sub, n_phi, base, dist)


def test_visibility_of_the_workload_image(mcrt, oracle_mod, torch_cuda):
    """The 1e-2 Msun workload's grid seen at 45 degrees from 150 pc with a
    100 m baseline (the setting of the paper's visibility curves): the image
    traced on the device and its amplitudes against the oracle's, both from
    the oracle's temperature field."""
    torch = torch_cuda
    d, _ = W.config("mrw_pda")
    ora = oracle_mod.Oracle(d)
    ctx = mcrt.Context(d)
    T = _field(d)
    ci, n_sub, n_phi = [0.7071067811865476], 2, 16
    base, dist = [[1e4, 0.0], [1e4, 1.5707963267948966]], 150 * 3.0857e18
    Ig = ctx.raytrace_image(torch.from_numpy(T).cuda(), cos_i=ci, n_sub=n_sub, n_phi=n_phi)
    Vg = ctx.visibility(Ig, ci, n_sub, n_phi, base, dist).cpu().numpy()
    Io = ora.raytrace_image(T, cos_i=ci, n_sub=n_sub, n_phi=n_phi)
    Vo = ora.visibility(Io, ci, n_sub, n_phi, base, dist)
    assert np.allclose(Vg, Vo, rtol=1e-8, atol=1e-12), np.max(np.abs(Vg - Vo))
    assert np.all((Vo >= 0.0) & (Vo <= 1.0 + 1e-12))

