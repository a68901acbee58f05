"""The differentiable PDA (linear solve with D frozen at T_D, eq. T diffusion
of Sect. 2.2.1) and its adjoint on the GPU, through the C-ABI, against the
oracle: the forward field against banded Cholesky, the adjoint gradient
against the oracle's direct (tangent-linear) gradient, which is itself pinned
to finite differences on the CPU, and the torch.autograd front end against
finite differences of the GPU forward solve."""
import numpy as np
import pytest

from paper_0902_3092_amd import workloads as W
from pda_cases import grad_problem

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


def _dev(torch, a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _grad_workload(oracle_mod):
    d, _ = W.config("pda_grad")
    ora = oracle_mod.Oracle(d)
    chi = lambda T: np.interp(T, ora.T_nodes, 1.0 / (3.0 * ora.Drho))
    return d, ora, W.pda_grad_inputs(d, chi)


@pytest.mark.parametrize("solver", [1, 2])
def test_pda_linear_matches_oracle_small(mcrt, oracle_mod, torch_cuda, solver):
    torch = torch_cuda
    d, T_D, T_bc, mask, ks, w = grad_problem()
    rho = d.rho * np.random.default_rng(7).uniform(0.7, 1.3, d.n_cells)
    ctx = mcrt.Context(d, pda_solver=solver)
    T_g, st = ctx.pda_linear(_dev(torch, mask, np.uint8), _dev(torch, T_D), _dev(torch, T_bc),
                             rho=_dev(torch, rho), kscale=_dev(torch, ks))
    T_o = oracle_mod.Oracle(d, rho=rho).pda_linear(T_D, T_bc, mask, kscale=ks)
    T_g = T_g.cpu().numpy()
    assert st["n_region"] > 0
    assert np.array_equal(T_g[mask == 0], T_bc[mask == 0])
    assert np.allclose(T_g, T_o, rtol=1e-8, atol=0)


@pytest.mark.parametrize("solver", [1, 2])
def test_pda_adjoint_matches_direct_small(mcrt, oracle_mod, torch_cuda, solver):
    """Every cell of a 14 x 10 grid: dJ/dlog rho and dJ/ds from one adjoint
    solve against one direct solve per parameter."""
    torch = torch_cuda
    d, T_D, T_bc, mask, ks, w = grad_problem()
    ctx = mcrt.Context(d, pda_solver=solver)
    ctx.pda_linear(_dev(torch, mask, np.uint8), _dev(torch, T_D), _dev(torch, T_bc),
                   kscale=_dev(torch, ks))
    g_r, g_s = ctx.pda_adjoint(_dev(torch, w))
    g_r, g_s = g_r.cpu().numpy(), g_s.cpu().numpy()
    cells = np.arange(d.n_cells)
    o_r, o_s = oracle_mod.Oracle(d).pda_grad_direct(T_D, T_bc, mask, w, cells, kscale=ks)
    for g, o in ((g_r, o_r), (g_s, o_s)):
        scale = np.abs(o).max()
        assert scale > 0
        assert np.allclose(g, o, rtol=1e-6, atol=1e-8 * scale)
    # no dependence outside the region and its face neighbours
    far = np.ones((d.n_r, d.n_mu), bool)
    m2 = mask.reshape(d.n_r, d.n_mu).astype(bool)
    far &= ~m2
    far[1:] &= ~m2[:-1]
    far[:-1] &= ~m2[1:]
    far[:, 1:] &= ~m2[:, :-1]
    far[:, :-1] &= ~m2[:, 1:]
    assert np.all(g_r[far.reshape(-1)] == 0) and np.all(g_s[far.reshape(-1)] == 0)


def test_pda_adjoint_full_workload(mcrt, oracle_mod, torch_cuda):
    """200 x 120 cells, 1e-1 Msun, region tau_R > 10: the forward field on
    every cell and the gradient of the mass-weighted midplane temperature on
    a sample of 48 cells (region, its rim and the midplane row) against the
    oracle."""
    torch = torch_cuda
    d, ora, (T_D, T_bc, mask, ks, w) = _grad_workload(oracle_mod)
    assert 1000 < mask.sum() < d.n_cells
    ctx = mcrt.Context(d)
    T_g, st = ctx.pda_linear(_dev(torch, mask, np.uint8), _dev(torch, T_D), _dev(torch, T_bc),
                             kscale=_dev(torch, ks))
    T_o = ora.pda_linear(T_D, T_bc, mask, kscale=ks)
    assert np.allclose(T_g.cpu().numpy(), T_o, rtol=1e-8, atol=0)
    g_r, g_s = ctx.pda_adjoint(_dev(torch, w))
    g_r, g_s = g_r.cpu().numpy(), g_s.cpu().numpy()
    rng = np.random.default_rng(11)
    m2 = mask.reshape(d.n_r, d.n_mu)
    rim = np.nonzero((m2[:, :-1] == 1) & (m2[:, 1:] == 0))
    rim_cells = rim[0] * d.n_mu + rim[1] + 1
    cells = np.unique(np.concatenate([
        rng.choice(np.nonzero(mask)[0], 16, replace=False),
        rng.choice(rim_cells, 16, replace=False),
        rng.choice(np.nonzero(m2[:, 0])[0], 16, replace=False) * d.n_mu]))
    o_r, o_s = ora.pda_grad_direct(T_D, T_bc, mask, w, cells, kscale=ks)
    for g, o in ((g_r[cells], o_r), (g_s[cells], o_s)):
        scale = np.abs(o).max()
        assert scale > 0
        assert np.allclose(g, o, rtol=1e-5, atol=1e-7 * scale)


def test_autograd_mass_weighted_midplane(mcrt, oracle_mod, torch_cuda):
    """J = sum_c w_c(rho) T_c with mass weights built in torch from log rho:
    autograd adds the explicit weight term to the adjoint term; checked
    against central differences (step 1e-6) of the GPU forward solve and
    against the oracle's direct gradient plus the explicit term."""
    torch = torch_cuda
    from paper_0902_3092_amd.autograd import pda_temperature
    d, T_D, T_bc, mask, ks, _ = grad_problem(seed=3)
    ctx = mcrt.Context(d, cg_tol=1e-15)
    vol = _dev(torch, W.cell_volumes(d))
    mid = torch.zeros(d.n_cells, dtype=torch.float64, device="cuda")
    mid[0::d.n_mu] = 1.0
    m_t, T_D_t, T_bc_t = _dev(torch, mask, np.uint8), _dev(torch, T_D), _dev(torch, T_bc)

    def objective(log_rho, kscale):
        T = pda_temperature(ctx, log_rho, kscale, m_t, T_D_t, T_bc_t)
        m = torch.exp(log_rho) * vol * mid
        return (m * T).sum() / m.sum(), T

    with np.errstate(divide="ignore"):   # dust-free cells: log rho = -inf, weight 0
        log_rho = _dev(torch, np.log(d.rho)).requires_grad_(True)
    kscale = _dev(torch, ks).requires_grad_(True)
    J, T = objective(log_rho, kscale)
    J.backward()
    gl, gk = log_rho.grad.cpu().numpy(), kscale.grad.cpu().numpy()

    # oracle: implicit term by the direct method, explicit term written out
    T_o = oracle_mod.Oracle(d).pda_linear(T_D, T_bc, mask, kscale=ks)
    midn = np.zeros(d.n_cells)
    midn[0::d.n_mu] = 1.0
    m = d.rho * W.cell_volumes(d) * midn
    w = m / m.sum()
    J_o = float(np.dot(w, T_o))
    cells = np.arange(d.n_cells)
    o_r, o_s = oracle_mod.Oracle(d).pda_grad_direct(T_D, T_bc, mask, w, cells, kscale=ks)
    o_r = o_r + w * (T_o - J_o)
    assert J.item() == pytest.approx(J_o, rel=1e-10)
    for g, o in ((gl, o_r), (gk, o_s)):
        assert np.allclose(g, o, rtol=1e-6, atol=1e-8 * np.abs(o).max())

    # finite differences of the GPU forward at step 1e-6 on a few cells
    h = 1e-6
    with torch.no_grad():
        for c in (2 * d.n_mu, 5 * d.n_mu + 1, 7 * d.n_mu + 3, 9 * d.n_mu + 5):
            for which, g in ((0, gl), (1, gk)):
                vals = []
                for sgn in (1.0, -1.0):
                    lr, k2 = log_rho.detach().clone(), kscale.detach().clone()
                    (lr if which == 0 else k2)[c] += sgn * h
                    vals.append(float(objective(lr, k2)[0]))
                fd = (vals[0] - vals[1]) / (2 * h)
                assert abs(g[c] - fd) <= 1e-4 * np.abs(g).max() + 1e-3 * abs(fd), (c, which, g[c], fd)
