"""Pins of the oracle's nonlinear PDA for differentiation (Sect. 2.2.1, eq. T
diffusion with the temperature-dependent diffusion coefficient of Sect.
2.2.3) and of its gradient by the direct method on the non-symmetric
Jacobian:

* the gradient against central finite differences of the oracle's own
  Picard forward (a different route: repeated nonlinear solves);
* the forward is a fixed point: one more linear solve with D frozen at it
  returns it;
* gray dust, where D does not depend on T: the forward is the linear solve
  and the gradient the linear (symmetric) one, already pinned;
* on non-gray dust the dependence of D on T changes the gradient: the linear
  gradient at the same temperature differs from it.
"""
import numpy as np
import pytest

from paper_0902_3092_amd import workloads as W
from pda_cases import grad_problem


def _problem(contrast):
    """grad_problem, with the Dirichlet field spread by a factor up to 3 either
    way when `contrast` (steep temperature differences between neighbours,
    where the dependence of D on T weighs most)."""
    d, T_D, T_bc, mask, ks, w = grad_problem()
    if contrast:
        T_bc = T_D * np.random.default_rng(7).uniform(1.0 / 3.0, 3.0, d.n_cells)
    return d, T_bc, mask, ks, w


def _cells(d, mask, seed=1):
    rng = np.random.default_rng(seed)
    cand = np.nonzero(mask)[0]
    return np.concatenate([rng.choice(cand, 10, replace=False), [2 * d.n_mu + 7, 1 * d.n_mu]])


@pytest.mark.parametrize("contrast", [False, True])
@pytest.mark.parametrize("param", ["logrho", "kscale"])
def test_nonlinear_gradient_matches_finite_differences(oracle_mod, param, contrast):
    d, T_bc, mask, ks, w = _problem(contrast)
    ora = oracle_mod.Oracle(d)
    cells = _cells(d, mask)
    T, g_r, g_s = ora.pda_nl_grad_direct(T_bc, mask, w, cells, kscale=ks)
    g = g_r if param == "logrho" else g_s

    def J(c, step):
        rho = d.rho.copy()
        k2 = ks.copy()
        if param == "logrho":
            rho[c] *= np.exp(step)
        else:
            k2[c] += step
        Tn, sweeps, ch = oracle_mod.Oracle(d, rho=rho).pda_nonlinear(T_bc, mask, kscale=k2)
        assert ch < 1e-12
        return np.dot(w, Tn)

    h = 4e-3
    for q, c in enumerate(cells):
        fd1 = (J(c, h) - J(c, -h)) / (2 * h)
        fd2 = (J(c, h / 2) - J(c, -h / 2)) / h
        fd = (4 * fd2 - fd1) / 3
        scale = max(abs(fd), 1e-6 * np.abs(g).max())
        assert abs(g[q] - fd) <= 1e-6 * scale + 1e-9 * np.abs(g).max(), (c, g[q], fd)
    assert np.abs(g).max() > 0


def test_nonlinear_forward_is_a_fixed_point(oracle_mod):
    d, _, T_bc, mask, ks, _ = grad_problem(seed=2)
    ora = oracle_mod.Oracle(d)
    T, sweeps, ch = ora.pda_nonlinear(T_bc, mask, kscale=ks)
    assert sweeps > 2 and ch < 1e-12
    again = ora.pda_linear(T, T_bc, mask, kscale=ks)
    assert np.allclose(again, T, rtol=1e-11, atol=0)
    # and it moved: the linear solve with D at the Dirichlet field differs
    first = ora.pda_linear(T_bc, T_bc, mask, kscale=ks)
    reg = mask.astype(bool)
    assert np.max(np.abs(first[reg] / T[reg] - 1)) > 1e-5


def test_gray_dust_reduces_to_the_linear_solve(oracle_mod):
    d = W.uniform_shell(1e-12, n_r=12, n_mu=10, albedo=0.3, R_in_au=1.0, R_out_au=20.0)
    ora = oracle_mod.Oracle(d)
    rng = np.random.default_rng(4)
    T_bc = rng.uniform(200.0, 400.0, d.n_cells)
    mask = np.zeros((d.n_r, d.n_mu), np.uint8)
    mask[3:9, 0:6] = 1
    mask = mask.reshape(-1)
    ks = rng.uniform(0.8, 1.2, d.n_cells)
    w = rng.uniform(0.0, 1.0, d.n_cells)
    cells = _cells(d, mask, seed=5)
    T, g_r, g_s = ora.pda_nl_grad_direct(T_bc, mask, w, cells, kscale=ks)
    T_lin = ora.pda_linear(T_bc, T_bc, mask, kscale=ks)
    assert np.allclose(T, T_lin, rtol=1e-12, atol=0)
    l_r, l_s = ora.pda_grad_direct(T, T_bc, mask, w, cells, kscale=ks)
    assert np.allclose(g_r, l_r, rtol=1e-9, atol=1e-12 * np.abs(l_r).max())
    assert np.allclose(g_s, l_s, rtol=1e-9, atol=1e-12 * np.abs(l_s).max())


def test_temperature_dependence_of_D_changes_the_gradient(oracle_mod):
    d, T_bc, mask, ks, w = _problem(True)
    ora = oracle_mod.Oracle(d)
    cells = _cells(d, mask)
    T, g_r, _ = ora.pda_nl_grad_direct(T_bc, mask, w, cells, kscale=ks)
    l_r, _ = ora.pda_grad_direct(T, T_bc, mask, w, cells, kscale=ks)
    big = np.abs(g_r) > 1e-3 * np.abs(g_r).max()
    assert big.sum() >= 4
    assert np.max(np.abs(l_r[big] / g_r[big] - 1)) > 1e-2
