"""The synthetic disk inputs against the paper's density law (Sect. 2.4)."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from paper_0902_3092_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_disk_setup.json")


def _radial_tau_closed_form(M, R_in, R_out, h1, p, chi):
    return M * (R_in ** -p - R_out ** -p) * W.AU ** p / (
        2 * math.pi * math.sqrt(math.pi) * h1 * p * (R_out - R_in)) * chi


def test_density_law_reproduces_printed_radial_tau():
    """eq:density integrated through the midplane gives eq:radial tau; the two
    optical depths the paper prints for its two disk masses follow from one
    and the same extinction coefficient at 550 nm."""
    g = json.load(open(GOLD))
    R_in, R_out = g["R_in_au"] * W.AU, g["R_out_au"] * W.AU
    h1, p = g["h1_au"] * W.AU, g["p"]
    chis = []
    for M_msun, tau in zip(g["M_dust_msun"], g["tau_radial_550nm"]):
        M = M_msun * W.M_SUN
        col = integrate.quad(lambda R: W.density_law(np.array([R]), np.array([0.0]), M, R_in,
                                                     R_out, h1, p)[0], R_in, R_out,
                             limit=400, epsrel=1e-11)[0]
        closed = _radial_tau_closed_form(M, R_in, R_out, h1, p, 1.0)
        assert col == pytest.approx(closed, rel=1e-8)
        chis.append(tau / col)
    assert chis[0] == pytest.approx(chis[1], rel=0.01)
    assert 1e4 < chis[0] < 5e4       # sub-micron silicate at 550 nm: ~ 2.3e4 cm^2/g


def test_density_law_surface_density_and_mass():
    """Sigma(R) = M / (2 pi (R_out - R_in) R): the vertical integral of
    eq:density, and the disk holds M."""
    M, R_in, R_out, h1, p = 1e30, 0.1 * W.AU, 100 * W.AU, 0.03 * W.AU, 9 / 7
    for R in (0.3 * W.AU, 7 * W.AU, 60 * W.AU):
        h = h1 * (R / W.AU) ** p
        sig = integrate.quad(lambda z: W.density_law(np.array([R]), np.array([z]), M, R_in,
                                                     R_out, h1, p)[0], -12 * h, 12 * h,
                             epsrel=1e-12)[0]
        assert sig == pytest.approx(M / (2 * math.pi * (R_out - R_in) * R), rel=1e-9)


@pytest.mark.parametrize("name", ["plain", "mrw_pda"])
def test_grid_mass_and_midplane_column(name):
    d, o = W.config(name)
    V = W.cell_volumes(d)
    assert (d.rho * V).sum() == pytest.approx(d.M_dust, rel=0.01)
    rho = d.rho.reshape(d.n_r, d.n_mu)
    col = (rho[:, 0] * np.diff(d.r_edges)).sum()
    pr = d.params
    closed = _radial_tau_closed_form(d.M_dust, pr["R_in_au"] * W.AU, pr["R_out_au"] * W.AU,
                                     pr["h1"], pr["p"], 1.0)
    assert col == pytest.approx(closed, rel=0.03)
    chi = d.kappa_abs[0, 0] + d.kappa_sca[0, 0]
    if name == "mrw_pda":
        assert col * chi == pytest.approx(1e5, rel=0.03)


def test_batch_draws_ranges():
    draws = W.batch_draws()
    assert len(draws) == 64
    assert all(-5 <= math.log10(b["M_dust_msun"]) <= -1 for b in draws)
    assert all(0.02 <= b["hr0"] <= 0.05 for b in draws)
    assert all(50 <= b["n_r"] <= 200 and 40 <= b["n_mu"] <= 120 for b in draws)
    assert all(1e6 <= b["n_packets"] <= 1e7 for b in draws)
    assert W.batch_draws() == draws   # seeded
