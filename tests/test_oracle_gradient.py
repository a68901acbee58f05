"""The oracle's PDA gradient (direct, tangent-linear method) against central
finite differences of the oracle's own banded-Cholesky forward solve: the
reference that the HIP adjoint is checked against is pinned here."""
import numpy as np
import pytest

from pda_cases import grad_problem


@pytest.mark.parametrize("param", ["logrho", "kscale"])
def test_direct_gradient_matches_finite_differences(oracle_mod, param):
    d, T_D, T_bc, mask, ks, w = grad_problem()
    ora = oracle_mod.Oracle(d)
    rng = np.random.default_rng(1)
    # cells next to and inside the region, where the gradient is not zero
    cand = np.nonzero(mask)[0]
    cells = np.concatenate([rng.choice(cand, 10, replace=False), [2 * d.n_mu + 7, 1 * d.n_mu]])
    g_r, g_s = ora.pda_grad_direct(T_D, T_bc, mask, w, cells, kscale=ks)
    g = g_r if param == "logrho" else g_s
    def J(c, step):
        rho = d.rho.copy()
        k2 = ks.copy()
        if param == "logrho":
            rho[c] *= np.exp(step)
        else:
            k2[c] += step
        return np.dot(w, oracle_mod.Oracle(d, rho=rho).pda_linear(T_D, T_bc, mask, kscale=k2))

    h = 4e-3
    for q, c in enumerate(cells):
        # central differences at h and h/2, Richardson-extrapolated (error O(h^4))
        fd1 = (J(c, h) - J(c, -h)) / (2 * h)
        fd2 = (J(c, h / 2) - J(c, -h / 2)) / h
        fd = (4 * fd2 - fd1) / 3
        scale = max(abs(fd), 1e-6 * np.abs(g).max())
        assert abs(g[q] - fd) <= 1e-6 * scale + 1e-9 * np.abs(g).max(), (c, g[q], fd)
    assert np.abs(g).max() > 0
