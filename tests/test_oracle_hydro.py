"""Pins of the oracle's vertical hydrostatic equilibrium (Sect. 2.5, eq.
balance): an isothermal shell against the closed form of the integral of
z / R^3 along it (with second-order convergence of the trapezoidal rule), a
shell without gravity (rho T constant), and the mass of every shell kept."""
import dataclasses
import math

import numpy as np
import pytest

from paper_0902_3092_amd import workloads as W

G, K_B, M_P = 6.67430e-8, 1.380649e-16, 1.67262192369e-24
M_STAR = 2.5 * W.M_SUN


def _disk(n_mu, mu_max=0.4):
    d = W.small_disk(M_dust_msun=1e-3, n_r=4, n_mu=8, n_lambda=16)
    mu = np.concatenate([np.linspace(0.0, mu_max, n_mu), [1.0]])
    rho = np.full(d.n_r * n_mu, 1e-12)
    return dataclasses.replace(d, mu_edges=mu, rho=rho)


def _profile(oracle_mod, n_mu, T0=150.0):
    d = _disk(n_mu)
    ora = oracle_mod.Oracle(d, n_T=16)
    T = np.full(ora.n_cells, T0)
    rho = ora.hydrostatic(T, M_STAR, 2.3).reshape(d.n_r, n_mu)
    r = 0.5 * (d.r_edges[:-1] + d.r_edges[1:])
    mc = 0.5 * (d.mu_edges[:-1] + d.mu_edges[1:])
    R = r[:, None] * np.sqrt(1 - mc[None, :] ** 2)
    A = 2.3 * M_P * G * M_STAR / (K_B * T0)
    want = np.exp(-A * (1 / R - 1 / R[:, :1]))       # integral of z / R^3 dz = 1 / R
    return rho[:, :-1] / rho[:, :1], want[:, :-1]


def test_isothermal_shell_closed_form(oracle_mod):
    errs = []
    for n in (41, 81, 161):
        got, want = _profile(oracle_mod, n)
        ok = want > 1e-6
        errs.append(np.max(np.abs(np.log(got[ok] / want[ok]))))
    assert errs[-1] < 2e-3
    # second order: halving the spacing cuts the error by about four
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_no_gravity_keeps_rho_T(oracle_mod):
    d = _disk(20)
    ora = oracle_mod.Oracle(d, n_T=16)
    T = np.random.default_rng(1).uniform(20.0, 500.0, ora.n_cells)
    rho = ora.hydrostatic(T, 0.0, 2.3)
    pT = (rho * T).reshape(d.n_r, -1)
    assert np.allclose(pT, pT[:, :1], rtol=1e-12, atol=0)


def test_shell_mass_kept(oracle_mod):
    d = W.small_disk(M_dust_msun=1e-3, n_r=12, n_mu=10, n_lambda=16)
    ora = oracle_mod.Oracle(d, n_T=16)
    T = np.random.default_rng(2).uniform(10.0, 800.0, ora.n_cells)
    rho = ora.hydrostatic(T, M_STAR, 2.3)
    m_old = (d.rho * ora.volumes).reshape(d.n_r, -1).sum(1)
    m_new = (rho * ora.volumes).reshape(d.n_r, -1).sum(1)
    assert np.allclose(m_new, m_old, rtol=1e-12, atol=0)
    # hotter columns are thicker: the density falls more slowly with z
    T2 = T * 4.0
    rho2 = ora.hydrostatic(T2, M_STAR, 2.3).reshape(d.n_r, -1)
    r1 = rho.reshape(d.n_r, -1)
    top = rho2[:, -1] / rho2[:, 0] >= r1[:, -1] / r1[:, 0]
    assert top.all()


def test_cold_shell_keeps_its_density(oracle_mod):
    """An optically thick dust cell with no temperature (T = 0: nothing was
    absorbed there) cannot be balanced: a zero temperature would collapse the
    scale height, which the paper avoids by filling such cells with the PDA
    first (Sect. 3.4, vertical-structure Case 3).  Its shell keeps the input
    density and is counted; the other shells are solved as usual.  A cold cell
    transparent at every wavelength (optical width < 1) holds next to no mass
    and is floored instead."""
    d = W.small_disk(M_dust_msun=1e-1, n_r=12, n_mu=10, n_lambda=16)
    ora = oracle_mod.Oracle(d, n_T=16)
    T = np.random.default_rng(3).uniform(20.0, 500.0, ora.n_cells).reshape(d.n_r, -1)
    T[4, 0] = 0.0          # a cold midplane cell (optical width ~66)
    T[7, 3] = 0.0          # optical width ~21
    T[2, 9] = 0.0          # transparent near the pole: floored, not counted
    rho, n_cold = ora.hydrostatic(T.reshape(-1), M_STAR, 2.3, return_cold=True)
    assert n_cold == 2
    rho = rho.reshape(d.n_r, -1)
    rho0 = d.rho.reshape(d.n_r, -1)
    assert np.array_equal(rho[4], rho0[4]) and np.array_equal(rho[7], rho0[7])
    warm = [i for i in range(d.n_r) if i not in (4, 7)]
    assert not np.allclose(rho[warm], rho0[warm], rtol=1e-3, atol=0)
    # the warm shells match a run where the cold shells are given temperatures
    T2 = T.copy()
    T2[4, 0], T2[7, 3] = 100.0, 100.0
    rho2 = ora.hydrostatic(T2.reshape(-1), M_STAR, 2.3).reshape(d.n_r, -1)
    assert np.array_equal(rho[warm], rho2[warm])


def _column_case(oracle_mod, n_r=100, n_mu=60, hr0=0.03):
    """The workload's grid with the exact solution of eq. balance on vertical
    columns: T depends on the cylindrical radius R only, with the scale height
    of the density law, so rho(R, z) = Sigma(R) / (sqrt(pi) h) exp(-(z/h)^2)
    is in equilibrium column by column (h^2 = 2 k T R^3 / (mu m_p G M)), with
    Sigma(R) fixed.  Cell-centre values."""
    d = W.make_disk("col", M_dust_msun=1e-2, n_r=n_r, n_mu=n_mu, n_lambda=16, hr0=hr0)
    p = d.params
    r = 0.5 * (d.r_edges[:-1] + d.r_edges[1:])
    mc = 0.5 * (d.mu_edges[:-1] + d.mu_edges[1:])
    R = r[:, None] * np.sqrt(1 - mc[None, :] ** 2)
    z = r[:, None] * mc[None, :]
    rho0 = W.density_law(R, z, d.M_dust, p["R_in_au"] * W.AU, p["R_out_au"] * W.AU, p["h1"],
                         p["p"])
    h = p["h1"] * (R / W.AU) ** p["p"]
    T = 2.3 * M_P * G * M_STAR * h ** 2 / (2 * K_B * R ** 3)
    d = dataclasses.replace(d, rho=np.ascontiguousarray(rho0.reshape(-1)))
    return d, T.reshape(-1), rho0, z / h


def test_shell_reading_departs_little_from_vertical_columns(oracle_mod):
    """The oracle balances eq. balance along each radial shell (z = r mu, R =
    r sqrt(1 - mu^2), the shell's mass kept) instead of along vertical columns
    at fixed R with Sigma(R) kept, as the paper states it.  Fed the exact
    column equilibrium, a column solver returns it unchanged; the shell
    reading's departure from it is measured here: where the mass is, it is a
    few tenths of a percent (the two readings' exponents differ by a term of
    order (z/h)^2 (h/r)^2), and it grows towards the surface layers."""
    d, T, rho0, zh = _column_case(oracle_mod)
    ora = oracle_mod.Oracle(d, n_T=16)
    rho1 = ora.hydrostatic(T, M_STAR, 2.3).reshape(d.n_r, d.n_mu)
    m = rho0 * ora.volumes.reshape(d.n_r, d.n_mu)
    ok = rho0 > 0
    dev = np.where(ok, rho1 / np.where(ok, rho0, 1) - 1, 0.0)
    w = m / m.sum()
    mean_abs = float((w * np.abs(dev)).sum())
    bands = {}
    for lo, hi in ((0, 1), (1, 2), (2, 3)):
        sel = ok & (zh >= lo) & (zh < hi)
        bands[(lo, hi)] = (float(np.abs(dev[sel]).max()), float(w[sel].sum()))
    print("shell vs column: mass-weighted mean |drho/rho| %.2e; by z/h band (max, mass "
          "fraction): %s" % (mean_abs, bands))
    assert mean_abs < 5e-3
    assert bands[(0, 1)][0] < 1e-2 and bands[(0, 1)][1] > 0.8
    assert bands[(1, 2)][0] < 6e-2 and bands[(2, 3)][1] < 1e-2
    # the departure falls as the disk gets thinner, as (h/r)^2
    d2, T2, rho02, _ = _column_case(oracle_mod, hr0=0.015)
    ora2 = oracle_mod.Oracle(d2, n_T=16)
    rho12 = ora2.hydrostatic(T2, M_STAR, 2.3).reshape(d2.n_r, d2.n_mu)
    m2 = rho02 * ora2.volumes.reshape(d2.n_r, d2.n_mu)
    ok2 = rho02 > 0
    dev2 = np.where(ok2, rho12 / np.where(ok2, rho02, 1) - 1, 0.0)
    mean2 = float((m2 / m2.sum() * np.abs(dev2)).sum())
    print("half the scale height: %.2e" % mean2)
    assert 3.0 < mean_abs / mean2 < 5.0
