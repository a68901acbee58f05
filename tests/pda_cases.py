"""Seeded inputs of the linear PDA solve and its gradient, shared by the
oracle's pin and the GPU parity tests (inputs only, no arithmetic of the
method)."""
import numpy as np

from paper_0902_3092_amd import workloads as W


def grad_problem(seed=0, n_r=14, n_mu=10, M_dust_msun=1e-3, n_lambda=30):
    """Power-law frozen temperature T_D, a perturbed Dirichlet field T_bc, a
    rectangular region touching the midplane, random extinction scales and
    an objective J = sum_c w_c T_c weighted on the midplane row."""
    d = W.make_disk("g", M_dust_msun=M_dust_msun, n_r=n_r, n_mu=n_mu, n_lambda=n_lambda)
    rng = np.random.default_rng(seed)
    rc = 0.5 * (d.r_edges[:-1] + d.r_edges[1:]) / W.AU
    mu_c = 0.5 * (d.mu_edges[:-1] + d.mu_edges[1:])
    T_D = (300.0 * rc[:, None] ** -0.5 * (1 + 0.2 * mu_c[None, :])).reshape(-1)
    T_bc = T_D * rng.uniform(0.9, 1.1, d.n_cells)
    mask = np.zeros((n_r, n_mu), np.uint8)
    mask[2:n_r - 2, 0:n_mu // 2 + 1] = 1
    kscale = rng.uniform(0.8, 1.2, d.n_cells)
    w = np.zeros((n_r, n_mu))
    w[:, 0] = rng.uniform(0.5, 1.5, n_r)
    w /= w.sum()
    return d, T_D, T_bc, mask.reshape(-1), kscale, w.reshape(-1)
