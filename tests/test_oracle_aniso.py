"""Pins of the oracle's anisotropic scattering: the Henyey-Greenstein sampler
against its closed-form moments and distribution, the rotation into the
packet's frame, the isotropic limit, the similarity correction of the
diffusion tables (Sect. 2.2.3: sigma' = (1 - g) sigma) against its closed form
for gray dust, and an explicit random walk with that phase function against
the diffusion escape time the corrected tables predict."""
import dataclasses
import math

import numpy as np
import pytest

from paper_0902_3092_amd import workloads as W


def _hg_cdf(mu, g):
    """Cumulative Henyey-Greenstein distribution of the scattering cosine,
    integrated from p(mu) = (1 - g^2) / (2 (1 + g^2 - 2 g mu)^(3/2))."""
    return (1 - g * g) / (2 * g) * ((1 + g * g - 2 * g * mu) ** -0.5 - 1 / (1 + g))


def _unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1)[:, None]


@pytest.mark.parametrize("g", [0.3, 0.7, -0.5])
def test_hg_moments_and_distribution(oracle_mod, g):
    """<mu> = g and <mu^2> = (1 + 2 g^2) / 3 (the first two Legendre moments
    of the phase function are g and g^2); Kolmogorov-Smirnov against the CDF."""
    rng = np.random.default_rng(11)
    n = 200000
    din = _unit(rng, n)
    u = rng.uniform(size=(n, 2))
    dout = oracle_mod.scatter_dirs(g, u, din)
    mu = (din * dout).sum(1)
    assert np.allclose(np.linalg.norm(dout, axis=1), 1.0, atol=1e-12)
    assert mu.mean() == pytest.approx(g, abs=5 * mu.std() / math.sqrt(n))
    m2 = mu * mu
    assert m2.mean() == pytest.approx((1 + 2 * g * g) / 3, abs=5 * m2.std() / math.sqrt(n))
    x = np.sort(mu)
    F = _hg_cdf(x, g)
    D = max(np.max(np.arange(1, n + 1) / n - F), np.max(F - np.arange(n) / n))
    assert D < 1.63 / math.sqrt(n)     # 1 % level


@pytest.mark.parametrize("g", [0.6, -0.3])
def test_hg_rotation(oracle_mod, g):
    """The cosine between the old and new directions is the one the first
    draw selects (its CDF value is the draw), for directions near the poles
    too, and the azimuth about the old direction is uniform."""
    rng = np.random.default_rng(5)
    n = 20000
    din = _unit(rng, n)
    din[:50] = [0.0, 0.0, 1.0]
    din[50:100] = [0.0, 0.0, -1.0]
    din[100:150] = [1e-4, 0.0, math.sqrt(1 - 1e-8)]
    u = rng.uniform(size=(n, 2))
    dout = oracle_mod.scatter_dirs(g, u, din)
    mu = np.clip((din * dout).sum(1), -1, 1)
    assert np.allclose(_hg_cdf(mu, g), u[:, 0], atol=2e-6)
    # azimuth: the component of dout perpendicular to din averages to zero
    perp = dout - mu[:, None] * din
    assert np.abs(perp.mean(0)).max() < 5 * math.sqrt(1 / n)


def test_g_zero_is_isotropic(oracle_mod):
    """g = 0: the new direction does not depend on the old one, w = 2 u1 - 1."""
    rng = np.random.default_rng(2)
    n = 1000
    u = rng.uniform(size=(n, 2))
    a = oracle_mod.scatter_dirs(0.0, u, _unit(rng, n))
    b = oracle_mod.scatter_dirs(0.0, u, _unit(rng, n))
    assert np.array_equal(a, b)
    assert np.allclose(a[:, 2], 2 * u[:, 0] - 1, atol=1e-15)


def _gray(kabs, ksca):
    d = W.small_disk(M_dust_msun=1e-3, n_r=8, n_mu=6, n_lambda=20)
    nl = d.n_lambda
    return dataclasses.replace(d, kappa_abs=np.full((1, nl), kabs), kappa_sca=np.full((1, nl), ksca),
                               mass_frac=np.ones(1))


@pytest.mark.parametrize("g", [0.0, 0.5, 0.85])
def test_similarity_tables_gray(oracle_mod, g):
    """For gray dust the tables' D rho is 1 / (3 (kappa + (1 - g) sigma)) and
    the mean absorption opacity of an MRW step is kappa / (kappa + (1 - g)
    sigma) times that extinction (kappa-bar = kappa)."""
    kabs, ksca = 2.0, 3.0
    ora = oracle_mod.Oracle(_gray(kabs, ksca), n_T=32, g_asym=g)
    chi = kabs + (1 - g) * ksca
    assert np.allclose(ora.Drho[1:], 1 / (3 * chi), rtol=1e-10, atol=0)
    assert np.allclose(ora.kbar[1:], kabs, rtol=1e-10)


def test_similarity_tables_equal_scaled_scattering(oracle_mod):
    """Non-gray dust: the tables with (sigma, g) are those with ((1 - g)
    sigma, 0), while the transport keeps the real sigma."""
    d = W.small_disk(M_dust_msun=1e-3, n_r=8, n_mu=6, n_lambda=30)
    g = 0.6
    a = oracle_mod.Oracle(d, n_T=48, g_asym=g)
    b = oracle_mod.Oracle(dataclasses.replace(d, kappa_sca=np.asarray(d.kappa_sca) * (1 - g)),
                          n_T=48, g_asym=0.0)
    assert np.allclose(a.Drho, b.Drho, rtol=1e-12, atol=0)
    assert np.allclose(a.kbar, b.kbar, rtol=1e-12)
    assert np.array_equal(a.cdf, b.cdf)


def test_hg_walk_escape_matches_corrected_diffusion(oracle_mod):
    """Pure scattering with the Henyey-Greenstein phase function in a sphere
    of radius tau0 mean free paths, from the centre: the mean path to leave
    is R0^2 / (6 D) with the corrected D = lambda / (3 (1 - g)), i.e.
    tau0^2 lambda (1 - g) / 2, up to O(1 / (tau0 (1 - g))); the isotropic D
    would predict twice that at g = 0.5."""
    rng = np.random.default_rng(3)
    tau0, g, n = 30.0, 0.5, 4000
    pos = np.zeros((n, 3))
    d = _unit(rng, n)
    path = np.zeros(n)
    alive = np.ones(n, bool)
    while alive.any():
        idx = np.nonzero(alive)[0]
        m = len(idx)
        L = rng.exponential(1.0, m)
        p, dd = pos[idx], d[idx]
        b = (p * dd).sum(1)
        c = (p * p).sum(1) - tau0 ** 2
        s_exit = -b + np.sqrt(b * b - c)
        leave = L >= s_exit
        step = np.where(leave, s_exit, L)
        path[idx] += step
        pos[idx] = p + step[:, None] * dd
        alive[idx[leave]] = False
        stay = idx[~leave]
        if len(stay):
            d[stay] = oracle_mod.scatter_dirs(g, rng.uniform(size=(len(stay), 2)), d[stay])
    want = tau0 ** 2 * (1 - g) / 2
    excess = path.mean() / want - 1
    assert abs(excess) < 3.0 / (tau0 * (1 - g))
    assert path.mean() < 0.75 * tau0 ** 2 / 2


def test_aniso_transport_conserves_energy(oracle_mod):
    """Escaped plus star-absorbed energy is L_star with g = 0.7, MRW on."""
    d = W.small_disk(M_dust_msun=3e-3, n_r=14, n_mu=10, n_lambda=24)
    ora = oracle_mod.Oracle(d, g_asym=0.7)
    st = ora.run(4000, 8, mrw=True, gamma=2.0, n_int_min=5)
    c = ora.counters(st)
    assert c["escaped"] + c["star"] == 4000 and c["scat"] > 0
    assert (st["sed"].sum() + st["E_star"][0]) / ora.L_star == pytest.approx(1.0, abs=1e-12)
