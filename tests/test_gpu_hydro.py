"""Vertical hydrostatic equilibrium on the GPU (mcrt_hydrostatic) against the
oracle: the density for a given temperature field, the cell masses the next
temperature inversion uses, and iterations of trace -> T -> PDA ->
hydrostatic keeping every shell's mass."""
import dataclasses

import numpy as np
import pytest

from paper_0902_3092_amd import workloads as W

pytestmark = pytest.mark.gpu

M_STAR = 2.5 * W.M_SUN


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


def _T_field(d, seed=3):
    rc = 0.5 * (d.r_edges[:-1] + d.r_edges[1:]) / W.AU
    base = 300.0 * rc[:, None] ** -0.5 * (1 + 2.0 * d.mu_edges[None, 1:])
    noise = np.random.default_rng(seed).uniform(0.9, 1.1, base.shape)
    return np.ascontiguousarray((base * noise).reshape(-1))


def test_hydrostatic_matches_oracle(mcrt, oracle_mod, torch_cuda):
    torch = torch_cuda
    d = W.make_disk("h", M_dust_msun=1e-3, n_r=30, n_mu=24, n_lambda=20)
    T = _T_field(d)
    ctx = mcrt.Context(d, n_T=64)
    ctx.set_T(torch.from_numpy(T).cuda())
    rho = ctx.hydrostatic(M_STAR).cpu().numpy()
    ora = oracle_mod.Oracle(d, n_T=64)
    want = ora.hydrostatic(T, M_STAR, 2.3, 1.0)
    nz = want > 1e-300
    assert np.array_equal(rho > 0, want > 0) or np.all(rho[~nz] < 1e-280)
    assert np.allclose(rho[nz], want[nz], rtol=1e-10, atol=0)
    m_old = (d.rho * ora.volumes).reshape(d.n_r, -1).sum(1)
    m_new = (rho * ora.volumes).reshape(d.n_r, -1).sum(1)
    assert np.allclose(m_new, m_old, rtol=1e-12, atol=0)


def test_hydrostatic_updates_cell_masses(mcrt, oracle_mod, torch_cuda):
    """After the new density, the temperature inversion of a tally uses the
    new cell masses: the same T as the oracle built on that density."""
    torch = torch_cuda
    d = W.small_disk(M_dust_msun=3e-3, n_r=14, n_mu=10, n_lambda=24)
    ctx = mcrt.Context(d)
    ctx.set_T(torch.from_numpy(_T_field(d)).cuda())
    rho = ctx.hydrostatic(M_STAR).cpu().numpy()
    ctx.reset()
    ctx.trace(20000, 5)
    T = ctx.update_T().cpu().numpy()
    E = ctx.get(mcrt.GET_E_ABS).cpu().numpy()
    ora = oracle_mod.Oracle(dataclasses.replace(d, rho=rho))
    assert np.allclose(T, ora.update_T(E), rtol=1e-12, atol=1e-12)
    c = ctx.counters()
    assert c["escaped"] + c["star"] == 20000


def test_vertical_structure_iterations(mcrt, oracle_mod, torch_cuda):
    """Three passes of trace, T, PDA and hydrostatic equilibrium on one disk:
    each shell keeps its mass, the density stays finite and positive where it
    was, and the temperature inversion stays consistent."""
    torch = torch_cuda
    d = W.small_disk(M_dust_msun=3e-3, n_r=14, n_mu=10, n_lambda=24)
    ctx = mcrt.Context(d, precision="fp32", mrw=True, pda_visits=30)
    V = oracle_mod.Oracle(d).volumes
    m0 = (d.rho * V).reshape(d.n_r, -1).sum(1)
    for it in range(3):
        ctx.reset()
        ctx.trace(100000, 40 + it)
        ctx.update_T()
        ctx.pda_solve()
        rho = ctx.hydrostatic(M_STAR).cpu().numpy()
        torch.cuda.synchronize()
        assert np.all(np.isfinite(rho)) and np.all(rho >= 0) and not np.any((rho > 0) & (d.rho <= 0))
        mid = rho.reshape(d.n_r, -1)[:, 0]
        assert np.all(mid[m0 > 0] > 0)
        assert np.allclose((rho * V).reshape(d.n_r, -1).sum(1), m0, rtol=1e-12, atol=0)


def test_no_gravity_keeps_rho_T(mcrt, torch_cuda):
    """M_star = 0: pressure balance alone, rho T constant along each shell."""
    torch = torch_cuda
    d = W.make_disk("h", M_dust_msun=1e-3, n_r=20, n_mu=16, n_lambda=20)
    T = _T_field(d, seed=9)
    ctx = mcrt.Context(d, n_T=64)
    ctx.set_T(torch.from_numpy(T).cuda())
    rho = ctx.hydrostatic(0.0).cpu().numpy()
    pT = (rho * T).reshape(d.n_r, -1)
    live = pT[:, 0] > 0
    assert live.sum() > 5
    assert np.allclose(pT[live], pT[live, :1], rtol=1e-12, atol=0)


def test_hydrostatic_arguments(mcrt):
    d = W.small_disk(M_dust_msun=1e-3, n_r=8, n_mu=6, n_lambda=16)
    ctx = mcrt.Context(d)
    with pytest.raises(mcrt.McrtError):
        ctx.hydrostatic(-1.0)
    with pytest.raises(mcrt.McrtError):
        ctx.hydrostatic(M_STAR, mu_mol=0.0)


def test_batched_passes_with_hydrostatic_step(mcrt, oracle_mod, torch_cuda):
    """mcrt_batch_run with the hydrostatic step on one of two disks (captured
    graph, two passes): the final density of that disk is the oracle's
    equilibrium for the final temperature (the shell masses being those of
    the initial disk), and the other disk's density is untouched."""
    torch = torch_cuda
    d1 = W.small_disk(M_dust_msun=3e-3, n_r=14, n_mu=10, n_lambda=24)
    d2 = W.small_disk(M_dust_msun=1e-3, n_r=10, n_mu=8, n_lambda=24)
    kw = dict(precision="fp32", mrw=True, gamma=3.0, n_int_min=20, pda_visits=30)
    c1 = mcrt.Context(d1, hydro_M_star=M_STAR, **kw)
    c2 = mcrt.Context(d2, **kw)
    mcrt.batch_run([c1, c2], [100000, 50000], [5, 6], n_iter=2, use_graph=True)
    torch.cuda.synchronize()
    T = c1.get(mcrt.GET_T).cpu().numpy()
    rho = c1.get(mcrt.GET_RHO).cpu().numpy()
    ora = oracle_mod.Oracle(d1)
    want, cold_o = ora.hydrostatic(T, M_STAR, 2.3, 1.0, return_cold=True)
    cold_g = int(c1.get(mcrt.GET_HYDRO_COLD).cpu().numpy()[0])
    # each shell is in equilibrium for the final T, unless one side held it
    # as it was: a shell holding a dusty cell without a temperature is held
    # when that cell is opaque at the density of the moment (the GPU's after
    # the first pass, the oracle's initial one here)
    n_r = d1.n_r
    Rg, Wo = rho.reshape(n_r, -1), want.reshape(n_r, -1)
    ok = np.array([np.allclose(Rg[i][Wo[i] > 1e-250], Wo[i][Wo[i] > 1e-250], rtol=1e-9, atol=0)
                   and np.all(Rg[i][Wo[i] <= 1e-250] < 1e-240) for i in range(n_r)])
    has_cold = np.any((T <= 0.0).reshape(n_r, -1) & (d1.rho > 0.0).reshape(n_r, -1), axis=1)
    print("shells in equilibrium: %d of %d; held: GPU %d, oracle %d"
          % (ok.sum(), n_r, cold_g, cold_o))
    assert np.all(has_cold[~ok])
    assert (~ok).sum() <= cold_g + cold_o
    assert ok.sum() >= n_r - 3
    assert (Wo[ok] > 1e-250).sum() > n_r * 3
    V = ora.volumes
    m0 = (d1.rho * V).reshape(d1.n_r, -1).sum(1)
    assert np.allclose((rho * V).reshape(d1.n_r, -1).sum(1), m0, rtol=1e-12, atol=0)
    assert not np.allclose(rho, d1.rho, rtol=1e-3, atol=0)
    assert np.array_equal(c2.get(mcrt.GET_RHO).cpu().numpy(), d2.rho)
    c = c1.counters()
    assert c["escaped"] + c["star"] == 100000
