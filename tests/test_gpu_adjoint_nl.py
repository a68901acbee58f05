"""The nonlinear differentiable PDA on the GPU (Picard to the fixed point of
eq. T diffusion, Sect. 2.2.1, with the diffusion coefficient of the
temperature itself, Sect. 2.2.3) and its adjoint on the non-symmetric
Jacobian, through the C-ABI, against the oracle: the forward field against
the oracle's Picard forward, the gradient against the oracle's direct method
on its Jacobian (pinned to finite differences on the CPU), on every cell of
a small grid at two Dirichlet contrasts and on sampled cells of the
200 x 120 differentiation workload; the torch.autograd front end against the
adjoint."""
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


def _problem(contrast):
    d, T_D, T_bc, mask, ks, w = grad_problem()
    if contrast:
        T_bc = T_D * np.random.default_rng(7).uniform(1.0 / 3.0, 3.0, d.n_cells)
    return d, T_bc, mask, ks, w


TIGHT = dict(pda_tol=1e-13, cg_tol=1e-14, pda_max_sweeps=200)


@pytest.mark.parametrize("contrast", [False, True])
def test_nonlinear_forward_and_gradient_match_oracle_small(mcrt, oracle_mod, torch_cuda,
                                                           contrast):
    torch = torch_cuda
    d, T_bc, mask, ks, w = _problem(contrast)
    ctx = mcrt.Context(d, **TIGHT)
    T_g, st = ctx.pda_nonlinear(_dev(torch, mask, np.uint8), _dev(torch, T_bc),
                                kscale=_dev(torch, ks))
    assert st["converged"] == 1 and st["sweeps"] > 2 and st["n_region"] > 0
    ora = oracle_mod.Oracle(d)
    cells = np.arange(d.n_cells)
    T_o, o_r, o_s = ora.pda_nl_grad_direct(T_bc, mask, w, cells, kscale=ks)
    T_g = T_g.cpu().numpy()
    assert np.array_equal(T_g[mask == 0], T_bc[mask == 0])
    assert np.allclose(T_g, T_o, rtol=1e-10, atol=0)
    g_r, g_s, ast = ctx.pda_nonlinear_adjoint(_dev(torch, w), stats=True)
    assert ast["converged"] == 1
    g_r, g_s = g_r.cpu().numpy(), g_s.cpu().numpy()
    for g, o in ((g_r, o_r), (g_s, o_s)):
        scale = np.abs(o).max()
        assert scale > 0
        assert np.allclose(g, o, rtol=1e-6, atol=1e-8 * scale)
    # the linear adjoint of the same temperature misses the D(T) terms
    ctx2 = mcrt.Context(d, **TIGHT)
    ctx2.pda_linear(_dev(torch, mask, np.uint8), _dev(torch, T_o), _dev(torch, T_bc),
                    kscale=_dev(torch, ks))
    l_r, _ = ctx2.pda_adjoint(_dev(torch, w))
    l_r = l_r.cpu().numpy()
    big = np.abs(o_r) > 1e-3 * np.abs(o_r).max()
    assert np.max(np.abs(l_r[big] / o_r[big] - 1)) > (1e-2 if contrast else 1e-5)


def test_nonlinear_adjoint_is_repeatable_and_guarded(mcrt, oracle_mod, torch_cuda):
    torch = torch_cuda
    d, T_bc, mask, ks, w = _problem(True)
    ctx = mcrt.Context(d, **TIGHT)
    with pytest.raises(mcrt.McrtError):
        ctx.pda_nonlinear_adjoint(_dev(torch, w))          # no forward yet
    ctx.pda_nonlinear(_dev(torch, mask, np.uint8), _dev(torch, T_bc), kscale=_dev(torch, ks))
    a1 = ctx.pda_nonlinear_adjoint(_dev(torch, w))[0].cpu().numpy()
    a2 = ctx.pda_nonlinear_adjoint(_dev(torch, w))[0].cpu().numpy()
    assert np.array_equal(a1, a2)
    # a linear solve in between replaces the kept state
    ctx.pda_linear(_dev(torch, mask, np.uint8), _dev(torch, T_bc), _dev(torch, T_bc))
    with pytest.raises(mcrt.McrtError):
        ctx.pda_nonlinear_adjoint(_dev(torch, w))


def test_nonlinear_full_workload(mcrt, oracle_mod, torch_cuda):
    """200 x 120 cells, 1e-1 Msun, region tau_R > 10, the Dirichlet field of
    the differentiation workload: the forward field on every cell and the
    gradient of the mass-weighted midplane temperature on 48 sampled cells
    (region, its rim and the midplane row) against the oracle."""
    torch = torch_cuda
    d, _ = W.config("pda_grad")
    ora = oracle_mod.Oracle(d)
    chi = lambda T: np.interp(T, ora.T_nodes, 1.0 / (3.0 * ora.Drho))
    T_D, T_bc, mask, ks, w = W.pda_grad_inputs(d, chi)
    assert 1000 < mask.sum() < d.n_cells
    ctx = mcrt.Context(d, **TIGHT)
    T_g, st = ctx.pda_nonlinear(_dev(torch, mask, np.uint8), _dev(torch, T_bc),
                                kscale=_dev(torch, ks))
    assert st["converged"] == 1
    rng = np.random.default_rng(11)
    m2 = mask.reshape(d.n_r, d.n_mu)
    rim = np.nonzero((m2[:, :-1] == 1) & (m2[:, 1:] == 0))
    rim_cells = rim[0] * d.n_mu + rim[1] + 1
    cells = np.unique(np.concatenate([
        rng.choice(np.nonzero(mask)[0], 16, replace=False),
        rng.choice(rim_cells, 16, replace=False),
        rng.choice(np.nonzero(m2[:, 0])[0], 16, replace=False) * d.n_mu]))
    T_o, o_r, o_s = ora.pda_nl_grad_direct(T_bc, mask, w, cells, kscale=ks)
    assert np.allclose(T_g.cpu().numpy(), T_o, rtol=1e-9, atol=0)
    g_r, g_s, ast = ctx.pda_nonlinear_adjoint(_dev(torch, w), stats=True)
    assert ast["converged"] == 1
    g_r, g_s = g_r.cpu().numpy(), g_s.cpu().numpy()
    for g, o in ((g_r[cells], o_r), (g_s[cells], o_s)):
        scale = np.abs(o).max()
        assert scale > 0
        assert np.allclose(g, o, rtol=1e-5, atol=1e-7 * scale)


def test_autograd_nonlinear(mcrt, oracle_mod, torch_cuda):
    """J = sum_c w_c T_c through pda_temperature_nonlinear: the gradient that
    autograd returns is the oracle's direct gradient, and a second forward on
    the context makes the first one's backward refuse."""
    torch = torch_cuda
    from paper_0902_3092_amd.autograd import pda_temperature_nonlinear
    d, T_bc, mask, ks, w = _problem(True)
    ctx = mcrt.Context(d, **TIGHT)
    m_t, T_bc_t, w_t = _dev(torch, mask, np.uint8), _dev(torch, T_bc), _dev(torch, w)
    with np.errstate(divide="ignore"):
        log_rho = _dev(torch, np.log(d.rho)).requires_grad_(True)
    kscale = _dev(torch, ks).requires_grad_(True)
    T = pda_temperature_nonlinear(ctx, log_rho, kscale, m_t, T_bc_t)
    (w_t * T).sum().backward()
    gl, gk = log_rho.grad.cpu().numpy(), kscale.grad.cpu().numpy()
    cells = np.arange(d.n_cells)
    _, o_r, o_s = oracle_mod.Oracle(d).pda_nl_grad_direct(T_bc, mask, w, cells, kscale=ks)
    for g, o in ((gl, o_r), (gk, o_s)):
        assert np.allclose(g, o, rtol=1e-6, atol=1e-8 * np.abs(o).max())
    T1 = pda_temperature_nonlinear(ctx, log_rho, kscale, m_t, T_bc_t)
    T2 = pda_temperature_nonlinear(ctx, log_rho, kscale, m_t, T_bc_t)
    T2.sum().backward()
    with pytest.raises(RuntimeError):
        T1.sum().backward()
