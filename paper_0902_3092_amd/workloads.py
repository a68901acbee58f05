"""Seeded synthetic disk models (inputs only).

This module builds the *inputs* of the radiative-transfer problem: the (r, mu)
grid, the per-cell dust density, the wavelength bins with their opacities and
the star.  It holds none of the transport, temperature or diffusion arithmetic,
so the CPU oracle and the HIP path can both be fed from it without sharing any
of the method.

Disk model: the density law of Sect. 2.4 (eq:density) with a surface density
Sigma ~ R^-1 and a Gaussian vertical profile of scale height
h(R) = h1 (R/AU)^p.  The paper's own table of parameters uses p = 1.3,
h1 = 0.03 AU and astronomical silicate; the synthetic workloads here keep the
law and the shape, take p = 9/7 (H/r ~ r^(2/7)) and replace the silicate
opacities (not available) with a power law kappa ~ lambda^-1 beyond 1 micron.

Units are cgs throughout.
"""
from __future__ import annotations

import dataclasses
import json
import math
from typing import Dict, List, Optional

import numpy as np

AU = 1.495978707e13        # cm (IAU 2012)
R_SUN = 6.957e10           # cm (IAU 2015 nominal)
M_SUN = 1.98847e33         # g
MICRON = 1.0e-4            # cm

# Absorption opacity shortward of 1 micron.  Chosen so that the 1e-2 Msun disk
# on 0.1-100 AU has a midplane radial extinction optical depth of 1e5 at
# lambda <= 1 micron with albedo 0.5 (column 3.997e4 g/cm^2, chi = 2.502).
KAPPA0 = 1.251             # cm^2/g


@dataclasses.dataclass
class Disk:
    """One disk model: geometry, density, dust and star (all host numpy)."""
    name: str
    r_edges: np.ndarray        # [n_r+1] cm, increasing
    mu_edges: np.ndarray       # [n_mu+1] |cos theta|, mu_edges[0]=0 (midplane) ... 1 (pole)
    rho: np.ndarray            # [n_r*n_mu] g/cm^3, cell id = i_r*n_mu + j_mu
    lambda_edges: np.ndarray   # [n_lambda+1] cm, increasing
    kappa_abs: np.ndarray      # [n_species, n_lambda] cm^2/g
    kappa_sca: np.ndarray      # [n_species, n_lambda] cm^2/g
    mass_frac: np.ndarray      # [n_species], sums to 1 (same mixture in every cell)
    T_star: float              # K
    R_star: float              # cm
    M_dust: float              # g (the input mass; the grid holds ~this)
    params: dict = dataclasses.field(default_factory=dict)

    @property
    def n_r(self) -> int:
        return len(self.r_edges) - 1

    @property
    def n_mu(self) -> int:
        return len(self.mu_edges) - 1

    @property
    def n_lambda(self) -> int:
        return len(self.lambda_edges) - 1

    @property
    def n_cells(self) -> int:
        return self.n_r * self.n_mu

    @property
    def n_species(self) -> int:
        return self.kappa_abs.shape[0]


@dataclasses.dataclass
class RunOptions:
    """Run settings shared by every implementation of the method."""
    n_packets: int = 100000
    seed: int = 0
    mrw: bool = False
    gamma: float = 3.0          # MRW start criterion, d_min > gamma / (rho chi_R)
    n_int_min: int = 20         # interactions in the current cell before MRW may start
    pda_visits: int = 0         # PDA region = cells with fewer visits (0: PDA off)
    n_T: int = 256              # temperature-table nodes (node 0 is T = 0)
    T_lo: float = 1.0           # K, first non-zero node
    T_hi: float = 1.0e4         # K, last node
    n_inc: int = 10             # SED inclination bins in |cos i|
    max_events: int = 1 << 30   # per-packet event cap


# --------------------------------------------------------------------------
# grid, density, opacities
# --------------------------------------------------------------------------

def log_edges(lo: float, hi: float, n: int) -> np.ndarray:
    e = np.exp(np.linspace(math.log(lo), math.log(hi), n + 1))
    e[0], e[-1] = lo, hi
    return e


def mu_edges_for(n_mu: int, hr_min: float) -> np.ndarray:
    """mu_0 = 0, mu_1 = 0.05 * min(H/r), geometric from mu_1 up to mu_n = 1."""
    if n_mu == 1:  # one row: the whole polar range
        return np.array([0.0, 1.0])
    mu1 = 0.05 * hr_min
    e = np.empty(n_mu + 1)
    e[0] = 0.0
    e[1:] = mu1 * (1.0 / mu1) ** (np.arange(n_mu) / (n_mu - 1))
    e[-1] = 1.0
    return e


def density_law(R, z, M_dust, R_in, R_out, h1, p):
    """Eq. (eq:density): rho(R, z) for R_in <= R <= R_out, zero outside."""
    h = h1 * (R / AU) ** p
    norm = M_dust * AU ** p / (2.0 * math.pi * math.sqrt(math.pi) * h1 * (R_out - R_in))
    with np.errstate(over="ignore", divide="ignore", invalid="ignore"):
        rho = norm * R ** (-1.0 - p) * np.exp(-(z / h) ** 2)
    inside = (R >= R_in) & (R <= R_out)
    return np.where(inside, rho, 0.0)


def cell_density(r_edges, mu_edges, M_dust, R_in, R_out, h1, p, n_gauss=8):
    """Volume-averaged density per (r, mu) cell, n_gauss x n_gauss Gauss points
    in (r, mu) with the r^2 volume weight."""
    x, w = np.polynomial.legendre.leggauss(n_gauss)
    ra, rb = r_edges[:-1], r_edges[1:]
    ma, mb = mu_edges[:-1], mu_edges[1:]
    # points [n_r, g], [n_mu, g]
    rp = 0.5 * (rb - ra)[:, None] * x[None, :] + 0.5 * (rb + ra)[:, None]
    rw = 0.5 * (rb - ra)[:, None] * w[None, :] * rp ** 2
    mp = 0.5 * (mb - ma)[:, None] * x[None, :] + 0.5 * (mb + ma)[:, None]
    mw = 0.5 * (mb - ma)[:, None] * w[None, :]
    R = rp[:, None, :, None] * np.sqrt(1.0 - mp[None, :, None, :] ** 2)
    z = rp[:, None, :, None] * mp[None, :, None, :]
    rho = density_law(R, z, M_dust, R_in, R_out, h1, p)
    wt = rw[:, None, :, None] * mw[None, :, None, :]
    num = (rho * wt).sum(axis=(2, 3))
    den = wt.sum(axis=(2, 3))
    return (num / den).reshape(-1)


def powerlaw_opacity(lambda_edges, kappa0, albedo, scale=1.0):
    lc = np.sqrt(lambda_edges[:-1] * lambda_edges[1:])
    kabs = scale * kappa0 * np.where(lc <= MICRON, 1.0, (lc / MICRON) ** -1.0)
    ksca = kabs * albedo / (1.0 - albedo)
    return kabs, ksca


def make_disk(name: str, *, M_dust_msun: float, n_r: int, n_mu: int, n_lambda: int,
              R_in_au: float = 0.1, R_out_au: float = 100.0, hr0: float = 0.03,
              p: float = 9.0 / 7.0, species=((1.0, 0.5),), T_star: float = 1.0e4,
              R_star_rsun: float = 2.5, lambda_lo_um: float = 0.1,
              lambda_hi_um: float = 1000.0) -> Disk:
    """Build a disk model.  species = ((kappa scale, albedo), ...) in equal mass fractions."""
    R_in, R_out = R_in_au * AU, R_out_au * AU
    h1 = hr0 * AU
    M = M_dust_msun * M_SUN
    r_edges = log_edges(R_in, R_out, n_r)
    hr_min = hr0 * (R_in_au) ** (p - 1.0)
    mu_edges = mu_edges_for(n_mu, hr_min)
    rho = cell_density(r_edges, mu_edges, M, R_in, R_out, h1, p)
    lam = log_edges(lambda_lo_um * MICRON, lambda_hi_um * MICRON, n_lambda)
    ka, ks = [], []
    for scale, alb in species:
        a, s = powerlaw_opacity(lam, KAPPA0, alb, scale)
        ka.append(a)
        ks.append(s)
    ns = len(species)
    return Disk(name=name, r_edges=r_edges, mu_edges=mu_edges, rho=rho,
                lambda_edges=lam, kappa_abs=np.array(ka), kappa_sca=np.array(ks),
                mass_frac=np.full(ns, 1.0 / ns), T_star=T_star,
                R_star=R_star_rsun * R_SUN, M_dust=M,
                params=dict(M_dust_msun=M_dust_msun, R_in_au=R_in_au, R_out_au=R_out_au,
                            hr0=hr0, p=p, h1=h1, species=[list(s) for s in species]))


def cell_volumes(disk: Disk) -> np.ndarray:
    """Both mirror halves of each (r, |mu|) cell: (4 pi/3)(r2^3 - r1^3)(mu2 - mu1)."""
    dr3 = disk.r_edges[1:] ** 3 - disk.r_edges[:-1] ** 3
    dmu = disk.mu_edges[1:] - disk.mu_edges[:-1]
    return (4.0 * math.pi / 3.0 * dr3[:, None] * dmu[None, :]).reshape(-1)


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------

def config(name: str):
    """Return (Disk, RunOptions) for a named workload.

    plain      1e-4 Msun, 40 x 30 cells, 50 bins, 1e5 packets, no MRW/PDA, seed 0
    mrw_pda    1e-2 Msun, 100 x 60 cells, 100 bins, 1e6 packets, MRW gamma=3, PDA < 100 visits, seed 1
    pda_grad   1e-1 Msun, 200 x 120 cells, 100 bins (PDA-only differentiation workload)
    large      1e-1 Msun, 0.1-500 AU, 400 x 200 cells, 200 bins, 3 species, 1e8 packets, seed 4
    """
    if name == "plain":
        d = make_disk("plain", M_dust_msun=1e-4, n_r=40, n_mu=30, n_lambda=50)
        return d, RunOptions(n_packets=100000, seed=0, mrw=False, pda_visits=0)
    if name == "mrw_pda":
        d = make_disk("mrw_pda", M_dust_msun=1e-2, n_r=100, n_mu=60, n_lambda=100)
        return d, RunOptions(n_packets=1000000, seed=1, mrw=True, gamma=3.0, n_int_min=20,
                             pda_visits=100)
    if name == "pda_grad":
        d = make_disk("pda_grad", M_dust_msun=1e-1, n_r=200, n_mu=120, n_lambda=100)
        return d, RunOptions(n_packets=0, seed=2, mrw=False, pda_visits=0)
    if name == "large":
        d = make_disk("large", M_dust_msun=1e-1, n_r=400, n_mu=200, n_lambda=200,
                      R_out_au=500.0, species=((1.0, 0.3), (0.3, 0.5), (0.1, 0.7)))
        return d, RunOptions(n_packets=100000000, seed=4, mrw=True, gamma=3.0, n_int_min=20,
                             pda_visits=100, n_T=160)
    raise KeyError(name)


def pda_grad_inputs(disk: Disk, chi_R, tau_min: float = 10.0):
    """Inputs of the differentiation workload on ``disk``.

    T_D = T_bc = T_star (R_star / 2r)^(1/2) at the cell-centre radius (the
    optically thin gray temperature, a smooth field); region = cells whose
    vertical Rosseland optical depth from the pole to the cell centre exceeds
    ``tau_min``, the depth summed along theta at fixed r with
    ``chi_R(T)`` (cm^2/g, a callable the caller takes from a temperature
    table) evaluated at T_D; extinction scales 1; objective weights
    w_c = m_c / sum m over the midplane row (mass-weighted midplane T).
    Returns (T_D, T_bc, mask uint8, kscale, w), all [n_cells]."""
    rc = 0.5 * (disk.r_edges[:-1] + disk.r_edges[1:])
    T_D = np.repeat(disk.T_star * np.sqrt(disk.R_star / (2.0 * rc)), disk.n_mu)
    th = np.arccos(np.clip(disk.mu_edges, -1.0, 1.0))       # decreasing with mu
    dth = th[:-1] - th[1:]                                    # [n_mu] > 0
    dtau = (disk.rho * np.asarray(chi_R(T_D))).reshape(disk.n_r, disk.n_mu) \
        * rc[:, None] * dth[None, :]
    above = np.cumsum(dtau[:, ::-1], axis=1)[:, ::-1] - dtau  # cells nearer the pole
    tau_c = above + 0.5 * dtau
    mask = (tau_c > tau_min).astype(np.uint8).reshape(-1)
    m = (disk.rho * cell_volumes(disk)).reshape(disk.n_r, disk.n_mu)
    w = np.zeros((disk.n_r, disk.n_mu))
    w[:, 0] = m[:, 0] / m[:, 0].sum()
    return T_D, T_D.copy(), mask, np.ones(disk.n_cells), w.reshape(-1)


def batch_draws(n_disks: int = 64, seed: int = 3) -> List[dict]:
    """Draw the batched workload: per disk, in this order, log10 M ~ U(-5,-1),
    H/r0 ~ U(0.02, 0.05), n_r ~ U{50..200}, packets ~ logU(1e6, 1e7)."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n_disks):
        lm = rng.uniform(-5.0, -1.0)
        hr0 = rng.uniform(0.02, 0.05)
        n_r = int(rng.integers(50, 201))
        n_pk = int(round(10 ** rng.uniform(6.0, 7.0)))
        n_mu = int(round(40 + (n_r - 50) * 80 / 150))
        out.append(dict(index=b, M_dust_msun=10 ** lm, hr0=hr0, n_r=n_r, n_mu=n_mu,
                        n_packets=n_pk, seed=1000 + b))
    return out


def batch_disk(draw: dict, n_lambda: int = 100) -> Disk:
    return make_disk("batch%02d" % draw["index"], M_dust_msun=draw["M_dust_msun"],
                     n_r=draw["n_r"], n_mu=draw["n_mu"], n_lambda=n_lambda, hr0=draw["hr0"])


def small_disk(M_dust_msun=1e-4, n_r=12, n_mu=8, n_lambda=16, **kw) -> Disk:
    """A tiny disk for unit tests (the plain workload's physics, coarse grid)."""
    return make_disk("small", M_dust_msun=M_dust_msun, n_r=n_r, n_mu=n_mu,
                     n_lambda=n_lambda, **kw)


def gray_disk(M_dust_msun=1e-9, n_r=24, n_mu=10, n_lambda=40, albedo=0.0) -> Disk:
    """Optically thin gray dust: kappa flat over all bins."""
    d = make_disk("gray", M_dust_msun=M_dust_msun, n_r=n_r, n_mu=n_mu, n_lambda=n_lambda)
    ka = np.full((1, n_lambda), KAPPA0)
    d.kappa_abs = ka
    d.kappa_sca = ka * albedo / (1.0 - albedo) if albedo > 0 else np.zeros_like(ka)
    return d


def to_json(disk: Disk) -> str:
    return json.dumps({k: (v.tolist() if isinstance(v, np.ndarray) else v)
                       for k, v in dataclasses.asdict(disk).items()})


def uniform_shell(rho: float, n_r: int = 16, n_mu: int = 8, n_lambda: int = 40,
                  gray: bool = True, albedo: float = 0.0, R_in_au: float = 0.1,
                  R_out_au: float = 100.0) -> Disk:
    """Constant-density spherical shell (every cell the same rho) for geometry
    and optically-thin pins.  gray=True: one absorption opacity in every bin."""
    d = make_disk("shell", M_dust_msun=1e-6, n_r=n_r, n_mu=n_mu, n_lambda=n_lambda,
                  R_in_au=R_in_au, R_out_au=R_out_au)
    d.rho = np.full(d.n_cells, float(rho))
    if gray:
        ka = np.full((1, n_lambda), KAPPA0)
    else:
        ka = d.kappa_abs.copy()
    d.kappa_abs = ka
    d.kappa_sca = ka * albedo / (1.0 - albedo)
    d.M_dust = float(rho * cell_volumes(d).sum())
    return d
