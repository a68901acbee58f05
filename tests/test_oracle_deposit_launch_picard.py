"""Pins of three oracle steps that the transport invariants cannot see:

* the energy an MRW step deposits (Sect. 2.2.2, eqs. modified RW and
  probability RW, with D and kappa-bar of Sect. 2.2.3), against an explicit
  photon random walk to the same sphere edge, and end to end against the
  explicit walk in the cells where the MRW acts;
* the wavelength bin of a launched packet (the star's spectrum, Sect. 2.1),
  against Planck bin integrals done here by quadrature;
* the Picard iteration of the PDA on a temperature-dependent diffusion
  coefficient (Sect. 2.2.1, eq. T diffusion), against the exact solution of
  the spherical problem through the Kirchhoff transform.
"""
import math

import numpy as np
import pytest
from scipy import integrate, optimize, stats

from paper_0902_3092_amd import workloads as W

H, KB, CL = 6.62607015e-27, 1.380649e-16, 2.99792458e10
# Extrapolation length of the Milne problem for isotropic scattering
# (Chandrasekhar, Radiative Transfer, Sect. 4): a diffusing walk sees an
# absorbing sphere edge as if it lay this many mean free paths further out.
MILNE_Q = 0.7104


def _walk_absorptions(tau0, n, omega, seed):
    """Explicit photon walk from the centre of a homogeneous sphere of radius
    tau0 mean free paths: exponential flights, isotropic directions,
    absorption (counted, then immediate reemission) with chance 1 - omega at
    each interaction inside; ends when a flight reaches the edge.  Returns
    the absorptions of each walker."""
    rng = np.random.default_rng(seed)
    pos = np.zeros((n, 3))
    alive = np.ones(n, bool)
    nab = np.zeros(n)
    while alive.any():
        idx = np.nonzero(alive)[0]
        m = len(idx)
        s = -np.log(rng.random(m))
        w = 2 * rng.random(m) - 1
        ph = 2 * np.pi * rng.random(m)
        st = np.sqrt(1 - w * w)
        p = pos[idx] + s[:, None] * np.stack([st * np.cos(ph), st * np.sin(ph), w], 1)
        out = (p * p).sum(1) >= tau0 * tau0
        alive[idx[out]] = False
        inside = idx[~out]
        pos[inside] = p[~out]
        nab[inside] += rng.random(len(inside)) >= omega
    return nab


def _gray_model(oracle_mod, rho=1e-14, albedo=0.5):
    d = W.uniform_shell(rho, n_r=4, n_mu=4, n_lambda=20, albedo=albedo, R_in_au=1.0,
                        R_out_au=2.0)
    d.mu_edges = np.array([0.0, 0.25, 0.5, 0.75, 1.0])
    return d, oracle_mod.Oracle(d)


@pytest.mark.parametrize("tau0,n", [(10.0, 40000), (30.0, 16000), (100.0, 3000)])
def test_mrw_deposit_vs_explicit_walk(oracle_mod, tau0, n):
    """Mean energy of one MRW step, eps rho kappa-bar (s R0^2 / D) averaged
    over the escape law, equals the mean number of absorptions of an explicit
    walk from the sphere's centre to its edge (gray dust, albedo 0.5, so
    kappa-bar = kappa and D = 1/(3 rho chi)).  The diffusion law ignores the
    boundary layer, which the walk sees as an edge MILNE_Q mean free paths
    further out: (tau0 / (tau0 + MILNE_Q))^2 of the walk's count."""
    d, ora = _gray_model(oracle_mod)
    chi = d.kappa_abs[0, 0] + d.kappa_sca[0, 0]
    R0 = tau0 / (d.rho[0] * chi)
    P0 = (np.arange(4000) + 0.5) / 4000
    dep = np.mean([ora.mrw_deposit(0, 300.0, R0, oracle_mod.mrw_escape_s(p)) for p in P0])
    nab = _walk_absorptions(tau0, n, 0.5, int(tau0))
    want = nab.mean() * (tau0 / (tau0 + MILNE_Q)) ** 2
    se = nab.std(ddof=1) / math.sqrt(n) * (tau0 / (tau0 + MILNE_Q)) ** 2
    assert abs(dep - want) < 4 * se + 0.01 * want, (dep, want, se)
    # the diffusion limit itself: (1 - albedo) tau0^2 / 2 absorptions
    assert dep == pytest.approx(0.5 * tau0 ** 2 / 2, rel=2e-3)


def test_mrw_deposit_weights_nongray(oracle_mod):
    """With wavelength-dependent opacity the deposit per unit path is the
    table's kappa-bar and the path uses the table's D: one MRW step of
    escape variable s deposits rho kappa-bar s R0^2 / D, linear in s and R0^2,
    and independent of rho at fixed optical radius (rho R0 fixed)."""
    d = W.make_disk("ng", M_dust_msun=1e-3, n_r=6, n_mu=4, n_lambda=30)
    ora = oracle_mod.Oracle(d)
    c = int(np.argmax(d.rho))
    T = 250.0
    Drho, kbar = ora.table_interp("Drho", T), ora.table_interp("kbar", T)
    R0 = 3.0e11
    a = ora.mrw_deposit(c, T, R0, 0.2)
    # dimensionless: (rho R0)^2 s kappa-bar / (D rho)
    assert a == pytest.approx((d.rho[c] * R0) ** 2 * 0.2 * kbar / Drho, rel=1e-13)
    assert ora.mrw_deposit(c, T, R0, 0.4) == pytest.approx(2 * a, rel=1e-13)
    assert ora.mrw_deposit(c, T, 2 * R0, 0.2) == pytest.approx(4 * a, rel=1e-13)


def test_mrw_on_off_in_mrw_cells(oracle_mod):
    """End to end in the cells where the MRW acts: a thick gray shell
    (radial optical depth 40, albedo 0.5, cells several mean free paths
    across) traced with and without the MRW.  With the MRW 30-65 % of the
    absorbed energy there comes from MRW deposits; the absorbed energy per
    cell must still match the explicit walk within the photon noise plus 5 %
    for the MRW's own bias (the paper finds its temperature errors of a few
    percent, Sect. 3.2) -- a deposit off by a factor two would move it by
    30-65 %."""
    d, _ = _gray_model(oracle_mod, rho=1.0)
    chi = d.kappa_abs[0, 0] + d.kappa_sca[0, 0]
    d.rho = np.full(d.n_cells, 40.0 / (chi * (d.r_edges[-1] - d.r_edges[0])))
    ora = oracle_mod.Oracle(d)
    n = 1500
    Tf = np.full(d.n_cells, 300.0)
    Es = {}
    for mrw in (False, True):
        E, N = [], []
        for s in range(4):
            st = ora.run(n, 40 + s + (10 if mrw else 0), mrw=mrw, gamma=2.0, n_int_min=5,
                         frozen_T=Tf)
            E.append(st["E_abs"] / st["eps"])
            N.append(st["n_mrw"].copy())
        Es[mrw] = (np.array(E), np.array(N))
    Eoff, _ = Es[False]
    Eon, Nmrw = Es[True]
    assert Nmrw.sum() > 5000
    # share of the absorbed energy deposited by MRW steps in the MRW cells
    counts_on = Eon.mean(0)
    cells = Nmrw.mean(0) > 100
    assert cells.sum() >= 4
    m_off, m_on = Eoff.mean(0), Eon.mean(0)
    se = np.sqrt(Eoff.var(0, ddof=1) / 4 + Eon.var(0, ddof=1) / 4)
    rel = m_on[cells] / m_off[cells] - 1
    tol = 4 * se[cells] / m_off[cells] + 0.05
    assert np.all(np.abs(rel) < tol), (rel, tol)
    # the whole shell: total absorbed energy
    tot_off, tot_on = Eoff.sum(1), Eon.sum(1)
    se_t = math.sqrt(tot_off.var(ddof=1) / 4 + tot_on.var(ddof=1) / 4)
    assert abs(tot_on.mean() / tot_off.mean() - 1) < 4 * se_t / tot_off.mean() + 0.03
    assert counts_on.sum() > 0


def _planck_bin(nu_a, nu_b, T):
    f = lambda x: x ** 3 / math.expm1(x)   # B_nu in units of 2 (kT)^3/(h^2 c^2) dx
    xa, xb = H * nu_a / (KB * T), H * nu_b / (KB * T)
    return integrate.quad(f, xa, xb, epsabs=0, epsrel=1e-12, limit=200)[0]


def test_launch_spectrum_is_stellar(oracle_mod):
    """Packets leave the star with the bin drawn from its spectrum (Sect. 2.1):
    in an empty shell every packet escapes in the bin it was launched in, so
    the escaped counts per bin follow int_bin B_nu(T_star) dnu, normalised
    over the grid's bins, computed here by quadrature in x = h nu / k T
    (chi-square test, bins with >= 20 expected packets, the rest merged)."""
    d = W.uniform_shell(1e-30, n_r=3, n_mu=2, n_lambda=50)
    ora = oracle_mod.Oracle(d)
    n = 200000
    st = ora.run(n, 12)
    counts = st["sed"].sum(1) / st["eps"]
    assert counts.sum() == pytest.approx(n, abs=0.5)
    lam = d.lambda_edges
    p = np.array([_planck_bin(CL / lam[k + 1], CL / lam[k], d.T_star)
                  for k in range(len(lam) - 1)])
    p /= p.sum()
    e = n * p
    big = e >= 20
    obs = np.append(counts[big], counts[~big].sum())
    exp = np.append(e[big], e[~big].sum())
    chi2 = ((obs - exp) ** 2 / exp).sum()
    dof = len(obs) - 1
    assert stats.chi2.sf(chi2, dof) > 1e-4, (chi2, dof)


def _kirchhoff_shell(ora, T_in, T_out, r_in, r_out):
    """Exact radial solution of div(D(T) grad T^4) = 0 between two spheres:
    Phi(T) = int_0^T D(T') 4 T'^3 dT' satisfies Phi = A + B/r."""
    Tn = ora.T_nodes
    nodes = Tn[(Tn > 0) & (Tn < 2 * T_in)]

    def Phi(T):
        pts = np.concatenate([[1e-3], nodes[nodes < T], [T]])
        tot = 0.0
        for a, b in zip(pts[:-1], pts[1:]):
            tot += integrate.quad(lambda t: ora.table_interp("Drho", t) * 4 * t ** 3, a, b,
                                  epsabs=0, epsrel=1e-12)[0]
        return tot

    Pi, Po = Phi(T_in), Phi(T_out)
    B = (Pi - Po) / (1 / r_in - 1 / r_out)
    A = Pi - B / r_in

    def T_of_r(r):
        target = A + B / r
        return optimize.brentq(lambda t: Phi(t) - target, T_out * 0.9, T_in * 1.1, xtol=1e-12,
                               rtol=1e-14)
    return T_of_r


def test_pda_picard_on_temperature_dependent_D(oracle_mod):
    """A non-gray shell (kappa ~ 1/lambda beyond 1 micron, so D falls ~5x
    between 150 and 800 K) with Dirichlet temperatures on its first and last
    radial cells: the PDA's Picard sweeps must converge to the exact solution
    Phi(T) = A + B/r of the nonlinear equation (Kirchhoff transform), with the
    discretisation error falling ~4x per grid doubling (second order).  A
    diffusion coefficient frozen at the initial temperature fails this."""
    errs, sweeps_all = [], []
    for n_r in (24, 48, 96):
        d = W.uniform_shell(1e-13, n_r=n_r, n_mu=3, n_lambda=60, gray=False, albedo=0.5,
                            R_in_au=1.0, R_out_au=10.0)
        d.mu_edges = np.array([0.0, 0.3, 0.7, 1.0])
        ora = oracle_mod.Oracle(d)
        rc = 0.5 * (d.r_edges[:-1] + d.r_edges[1:])
        T_in, T_out = 800.0, 150.0
        T_of_r = _kirchhoff_shell(ora, T_in, T_out, rc[0], rc[-1])
        T_mc = np.full((n_r, d.n_mu), 300.0)
        T_mc[0, :], T_mc[-1, :] = T_in, T_out
        reg = np.zeros((n_r, d.n_mu), np.uint8)
        reg[1:-1, :] = 1
        T, ro, sweeps, ch = ora.pda(T_mc.reshape(-1), reg.reshape(-1))
        sweeps_all.append((sweeps, ch))
        T = T.reshape(n_r, d.n_mu)
        want = np.array([T_of_r(r) for r in rc[1:-1]])
        assert np.allclose(T[1:-1, :], T[1:-1, :1], rtol=1e-10)   # no theta dependence
        errs.append(np.abs(T[1:-1, 0] / want - 1).max())
        if n_r == 24:
            # the answer of one sweep (D from the initial field)
            T1, _, _, _ = ora.pda(T_mc.reshape(-1), reg.reshape(-1), max_sweeps=1)
            err1 = np.abs(T1.reshape(n_r, -1)[1:-1, 0] / want - 1).max()
    assert errs[1] < errs[0] / 3.3 and errs[2] < errs[1] / 3.5, errs
    assert errs[2] < 5e-4
    assert all(sw >= 3 and ch < 1e-8 for sw, ch in sweeps_all), sweeps_all
    assert err1 > 10 * errs[0]      # one sweep is far off: the Picard sweeps matter
