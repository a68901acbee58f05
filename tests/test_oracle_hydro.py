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
