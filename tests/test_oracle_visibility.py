"""Pins of the oracle's visibility amplitudes (Sect. 3.4 shows visibility
curves of the ray-traced disks: the Fourier transform of the image at a
baseline's spatial frequency, normalised by the total flux), on images made
by hand so that the transform has a closed form:

* a thin ring of radius b at uniform intensity: |J0(2 pi s b)|, s = B / (lambda D)
  (the azimuthal sum over the ring's rays and their mirror images is the
  trapezoid rule of the Bessel integral);
* the ring and the star, a point at the centre: |F_star + F_ring J0| / (F_star + F_ring);
* the star alone, or a zero baseline: 1;
* an axisymmetric image looks the same from every baseline position angle.

The azimuthal sums are exact for these closed forms only where the 2 n_phi
points of a ring resolve its fringes, 2 pi s b well below 2 n_phi: the pins
take the bins where 2 pi s b < n_phi."""
import math

import numpy as np
import pytest
from scipy.special import j0

from paper_0902_3092_amd import workloads as W


def _model(oracle_mod, rho):
    d = W.uniform_shell(rho, n_r=8, n_mu=4, n_lambda=24, gray=False, albedo=0.3,
                        R_in_au=1.0, R_out_au=10.0)
    return d, oracle_mod.Oracle(d, n_T=64)


def _ring_image(d, n_sub, n_phi, ring, value=1.0):
    img = np.zeros((1, (d.n_r + 1) * n_sub, n_phi, d.n_lambda))
    img[0, ring] = value
    return img


def _ring_mid(d, n_sub, ring):
    bounds = np.concatenate([[0.0], d.r_edges])
    c, p = divmod(ring, n_sub)
    lo, hi = bounds[c], bounds[c + 1]
    b_lo, b_hi = lo + (hi - lo) * p / n_sub, lo + (hi - lo) * (p + 1) / n_sub
    return 0.5 * (b_lo + b_hi), math.pi * (b_hi ** 2 - b_lo ** 2)


def _lam(d):
    return np.sqrt(d.lambda_edges[:-1] * d.lambda_edges[1:])


D = 150 * 3.0857e18          # 150 pc


def test_ring_is_a_bessel_function(oracle_mod):
    d, ora = _model(oracle_mod, 1e-10)       # the star hidden behind tau >> 1
    n_sub, n_phi, ring = 2, 64, 9
    img = _ring_image(d, n_sub, n_phi, ring)
    b, _ = _ring_mid(d, n_sub, ring)
    B = 1e4                                   # 100 m
    V = ora.visibility(img, [0.6], n_sub, n_phi, [[B, 0.3], [3 * B, 1.1]], D)[0]
    for j, Bj in enumerate((B, 3 * B)):
        z = 2 * math.pi * Bj / (_lam(d) * D) * b
        ok = z < n_phi
        assert z[ok].max() > 5.0 and ok.sum() >= 8   # past the first zeros
        assert np.allclose(V[j][ok], np.abs(j0(z[ok])), rtol=0, atol=1e-10), \
            np.max(np.abs(V[j][ok] - np.abs(j0(z[ok]))))


def test_ring_and_star(oracle_mod):
    d, ora = _model(oracle_mod, 1e-22)       # the star shines through
    n_sub, n_phi, ring = 2, 64, 11
    b, area = _ring_mid(d, n_sub, ring)
    Iv = 1e-3
    img = _ring_image(d, n_sub, n_phi, ring, Iv)
    share = np.diff(np.concatenate([[0.0], ora.star_cdf]))
    chi = d.kappa_abs[0] + d.kappa_sca[0]
    star = ora.L_star * share * np.exp(-1e-22 * chi * (d.r_edges[-1] - d.r_edges[0]))
    F_star, F_ring = star / (4 * math.pi), Iv * area
    B = 2e4
    V = ora.visibility(img, [1.0], n_sub, n_phi, [[B, 0.0]], D)[0, 0]
    z = 2 * math.pi * B / (_lam(d) * D) * b
    ok = z < n_phi
    assert ok.sum() >= 8
    want = np.abs(F_star + F_ring * j0(z)) / (F_star + F_ring)
    assert np.allclose(V[ok], want[ok], rtol=1e-9, atol=1e-12)
    # the star alone, and a zero baseline, are unresolved
    Vs = ora.visibility(np.zeros_like(img), [1.0], n_sub, n_phi, [[B, 0.4]], D)[0, 0]
    assert np.allclose(Vs, 1.0, rtol=0, atol=1e-14)
    V0 = ora.visibility(img, [1.0], n_sub, n_phi, [[0.0, 0.4]], D)[0, 0]
    assert np.allclose(V0, 1.0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("theta", [0.0, 0.7, 1.5707963267948966, 2.9])
def test_axisymmetric_image_ignores_position_angle(oracle_mod, theta):
    d, ora = _model(oracle_mod, 1e-10)
    n_sub, n_phi = 2, 48
    rng = np.random.default_rng(5)
    prof = rng.uniform(0.0, 1.0, ((d.n_r + 1) * n_sub, d.n_lambda))
    img = np.repeat(prof[None, :, None, :], n_phi, axis=2)
    B = 1e4
    V = ora.visibility(img, [0.3], n_sub, n_phi, [[B, theta], [B, 0.0]], D)[0]
    ok = 2 * math.pi * B / (_lam(d) * D) * d.r_edges[-1] < n_phi
    assert ok.sum() >= 8
    assert np.allclose(V[0][ok], V[1][ok], rtol=0, atol=1e-9)
    # and an image brighter on one side is not
    lop = img.copy()
    lop[:, :, : n_phi // 2, :] *= 3.0
    V2 = ora.visibility(lop, [0.3], n_sub, n_phi, [[3 * B, 0.0], [3 * B, 1.5707963267948966]],
                        D)[0]
    assert np.max(np.abs(V2[0] - V2[1])) > 1e-3
