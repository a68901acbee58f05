"""CPU oracle (plain single-threaded FP64) of MC radiative transfer with
immediate reemission, the modified random walk and the partial diffusion
approximation, after Min et al. (2009).

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library and does not import it.

The arithmetic lives in ``mcrt_oracle.c``; this module only marshals numpy
arrays through ctypes.  ``build()`` compiles the shared library with
``gcc -O2 -ffp-contract=off`` (no fused multiply-add, so results do not depend
on contraction choices).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mcrt_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_override = None

N_COUNTERS = 8
COUNTER_NAMES = ["escaped", "star", "capped", "cross", "scat", "abs", "mrw", "launch"]


def build(force: bool = True) -> str:
    """Compile liboracle.so in place."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Model(C.Structure):
    _fields_ = [("n_r", C.c_int), ("n_mu", C.c_int), ("n_lambda", C.c_int),
                ("r_edges", C.c_void_p), ("mu_edges", C.c_void_p), ("rho", C.c_void_p),
                ("lambda_edges", C.c_void_p), ("kappa_abs", C.c_void_p),
                ("kappa_sca", C.c_void_p), ("T_star", C.c_double), ("R_star", C.c_double),
                ("g_asym", C.c_double)]


class _Tables(C.Structure):
    _fields_ = [("n_T", C.c_int), ("T_lo", C.c_double), ("T_hi", C.c_double),
                ("T", C.c_void_p), ("cdf", C.c_void_p), ("Drho", C.c_void_p),
                ("kbar", C.c_void_p), ("star_cdf", C.c_void_p), ("L_star", C.c_double),
                ("eta_iters_max", C.c_int)]


class _Opts(C.Structure):
    _fields_ = [("mrw", C.c_int), ("gamma", C.c_double), ("n_int_min", C.c_int),
                ("n_inc", C.c_int), ("max_events", C.c_longlong), ("frozen_T", C.c_void_p),
                ("coef_T", C.c_void_p)]


REC_DTYPE = np.dtype([("fate", np.int32), ("k", np.int32), ("n_cross", np.int64),
                      ("n_scat", np.int64), ("n_abs", np.int64), ("n_mrw", np.int64),
                      ("n_draws", np.int64), ("x", np.float64), ("y", np.float64),
                      ("z", np.float64), ("u", np.float64), ("v", np.float64),
                      ("w", np.float64)])


def use_library(path=None):
    """Bind the module to another build of the oracle (``path``), e.g. one
    compiled by a test from a deliberately altered source; None: the default
    liboracle.so."""
    global _lib, _override
    _override = path
    _lib = None


def build_variant(src_text: str, path: str) -> str:
    """Compile ``src_text`` (a version of mcrt_oracle.c) into ``path`` with
    the flags of build(); the header is taken from this package."""
    src = os.path.splitext(path)[0] + ".c"
    with open(src, "w") as fh:
        fh.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                           "-I" + _HERE, "-o", path, src, "-lm"])
    return path


def lib():
    global _lib
    if _lib is None:
        path = _override or _LIB_PATH
        if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(path)
        vp, i64, u64, dbl = C.c_void_p, C.c_int64, C.c_uint64, C.c_double
        L.ora_philox4x32_10.argtypes = [vp, vp]
        L.ora_scatter_dirs.argtypes = [dbl, vp, vp, vp, C.c_int]
        L.ora_hydrostatic.argtypes = [vp, vp, dbl, dbl, dbl, vp]
        L.ora_hydrostatic.restype = C.c_int
        L.ora_pda_region.argtypes = [vp, vp, vp, vp, C.c_int, dbl, vp]
        L.ora_pda_region.restype = None
        L.ora_mrw_deposit.argtypes = [vp, vp, i64, dbl, dbl, dbl]
        L.ora_mrw_deposit.restype = dbl
        L.ora_scatter_dirs.restype = None
        L.ora_uniforms.argtypes = [u64, u64, u64, i64, vp]
        L.ora_planck_bins.argtypes = [vp, C.c_int, dbl, vp, vp]
        L.ora_build_tables.argtypes = [vp, vp]
        L.ora_locate.argtypes = [vp, dbl, dbl, dbl]
        L.ora_locate.restype = i64
        L.ora_T_of_E.argtypes = [vp, vp, dbl, dbl]
        L.ora_T_of_E.restype = dbl
        L.ora_reemit_sample.argtypes = [vp, vp, dbl, dbl, dbl]
        L.ora_reemit_sample.restype = C.c_int
        L.ora_table_interp.argtypes = [vp, C.c_int, dbl]
        L.ora_table_interp.restype = dbl
        L.ora_mrw_escape_s.argtypes = [dbl]
        L.ora_mrw_escape_s.restype = dbl
        L.ora_mrw_survival.argtypes = [dbl]
        L.ora_mrw_survival.restype = dbl
        L.ora_run.argtypes = [vp, vp, vp, u64, u64, u64, u64, vp, vp, vp, vp, vp, vp, vp, vp, i64,
                              vp, vp, vp]
        L.ora_mean_intensity.argtypes = [vp, vp, vp, vp, vp]
        L.ora_mean_intensity.restype = None
        L.ora_raytrace_sed.argtypes = [vp, vp, vp, vp, C.c_int, vp, C.c_int, C.c_int, vp]
        L.ora_raytrace_sed.restype = None
        L.ora_raytrace_image.argtypes = [vp, vp, vp, vp, C.c_int, vp, C.c_int, C.c_int, vp]
        L.ora_raytrace_image.restype = None
        L.ora_visibility.argtypes = [vp, vp, vp, C.c_int, vp, C.c_int, C.c_int, C.c_int, vp,
                                     C.c_double, vp]
        L.ora_visibility.restype = None
        L.ora_conv_stat.argtypes = [vp, vp, vp, vp, vp, C.c_int, vp, vp, vp]
        L.ora_conv_stat.restype = None
        L.ora_cell_volumes.argtypes = [vp, vp]
        L.ora_update_T.argtypes = [vp, vp, vp, vp]
        L.ora_pda.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int, dbl, vp, vp, vp]
        L.ora_pda_linear.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.ora_pda_grad_direct.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, C.c_int, vp, vp]
        L.ora_pda_nl.argtypes = [vp, vp, vp, vp, vp, C.c_int, C.c_double, vp, vp, vp]
        L.ora_pda_nl_grad_direct.argtypes = [vp, vp, vp, vp, vp, C.c_int, C.c_double, vp, vp,
                                             C.c_int, vp, vp, vp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32).copy()
    k = np.ascontiguousarray(key, dtype=np.uint32)
    lib().ora_philox4x32_10(_p(c), _p(k))
    return c


def uniforms(seed: int, pid: int, d0: int, n: int) -> np.ndarray:
    out = np.empty(n)
    lib().ora_uniforms(seed, pid, d0, n, _p(out))
    return out


def scatter_dirs(g: float, u, din) -> np.ndarray:
    """Directions after one scattering each with asymmetry parameter g, from
    the draw pairs u [n, 2] and incoming directions din [n, 3]."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    din = np.ascontiguousarray(din, dtype=np.float64)
    out = np.empty_like(din)
    lib().ora_scatter_dirs(float(g), _p(u), _p(din), _p(out), int(len(din)))
    return out


def planck_bins(lambda_edges, T):
    le = np.ascontiguousarray(lambda_edges, dtype=np.float64)
    nl = len(le) - 1
    B, dB = np.empty(nl), np.empty(nl)
    lib().ora_planck_bins(_p(le), nl, float(T), _p(B), _p(dB))
    return B, dB


def mrw_survival(s: float) -> float:
    return lib().ora_mrw_survival(float(s))


def mrw_escape_s(P0: float) -> float:
    return lib().ora_mrw_escape_s(float(P0))


class Oracle:
    """The oracle bound to one disk model (any object with the Disk fields)."""

    def __init__(self, disk, n_T: int = 256, T_lo: float = 1.0, T_hi: float = 1.0e4,
                 rho=None, g_asym: float = 0.0):
        self.disk = disk
        f = np.asarray(disk.mass_frac, dtype=np.float64)
        self.kabs = np.ascontiguousarray((f[:, None] * np.asarray(disk.kappa_abs)).sum(0))
        self.ksca = np.ascontiguousarray((f[:, None] * np.asarray(disk.kappa_sca)).sum(0))
        self.r_edges = np.ascontiguousarray(disk.r_edges, dtype=np.float64)
        self.mu_edges = np.ascontiguousarray(disk.mu_edges, dtype=np.float64)
        self.rho = np.ascontiguousarray(disk.rho if rho is None else rho, dtype=np.float64)
        self.lam = np.ascontiguousarray(disk.lambda_edges, dtype=np.float64)
        self.n_r, self.n_mu, self.n_lambda = len(self.r_edges) - 1, len(self.mu_edges) - 1, len(self.lam) - 1
        self.n_cells = self.n_r * self.n_mu
        self.model = _Model(self.n_r, self.n_mu, self.n_lambda, _p(self.r_edges),
                            _p(self.mu_edges), _p(self.rho), _p(self.lam), _p(self.kabs),
                            _p(self.ksca), float(disk.T_star), float(disk.R_star),
                            float(g_asym))
        self.g_asym = float(g_asym)
        nl = self.n_lambda
        self.T_nodes = np.zeros(n_T)
        self.cdf = np.zeros((n_T, nl))
        self.Drho = np.zeros(n_T)
        self.kbar = np.zeros(n_T)
        self.star_cdf = np.zeros(nl)
        self.tables = _Tables(n_T, T_lo, T_hi, _p(self.T_nodes), _p(self.cdf), _p(self.Drho),
                              _p(self.kbar), _p(self.star_cdf), 0.0, 0)
        rc = lib().ora_build_tables(C.byref(self.model), C.byref(self.tables))
        if rc != 0:
            raise RuntimeError("oracle table build failed")
        self.L_star = self.tables.L_star
        self.volumes = np.empty(self.n_cells)
        lib().ora_cell_volumes(C.byref(self.model), _p(self.volumes))
        self.mass = self.rho * self.volumes

    # -- geometry ---------------------------------------------------------
    def locate(self, xyz) -> np.ndarray:
        xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
        L = lib()
        return np.array([L.ora_locate(C.byref(self.model), *map(float, q)) for q in xyz],
                        dtype=np.int64)

    def T_of_E(self, E, mass) -> float:
        return lib().ora_T_of_E(C.byref(self.model), C.byref(self.tables), float(E), float(mass))

    def reemit_sample(self, T_old, T_new, xi) -> int:
        return lib().ora_reemit_sample(C.byref(self.model), C.byref(self.tables), float(T_old),
                                       float(T_new), float(xi))

    def table_interp(self, which: str, T: float) -> float:
        return lib().ora_table_interp(C.byref(self.tables), {"Drho": 0, "kbar": 1}[which],
                                      float(T))

    # -- transport --------------------------------------------------------
    def run(self, n_packets: int, seed: int, *, n_total: int = None, offset: int = 0,
            mrw: bool = False, gamma: float = 3.0, n_int_min: int = 20, n_inc: int = 10,
            max_events: int = 1 << 30, frozen_T=None, n_recs: int = 0, state=None,
            coef_T=None, paths: bool = False):
        """Trace packets [offset, offset+n_packets) of a run of n_total packets.
        `state` (a previous result) accumulates tallies across calls.  coef_T:
        temperatures for the MRW's coefficients and criterion (a previous
        pass's) instead of the running cell temperature."""
        n_total = n_packets if n_total is None else n_total
        nc, nl = self.n_cells, self.n_lambda
        if state is None:
            state = dict(E_abs=np.zeros(nc), visits=np.zeros(nc, np.uint32),
                         n_abs=np.zeros(nc, np.uint32), n_mrw=np.zeros(nc, np.uint32),
                         sed=np.zeros((nl, n_inc)),
                         E_star=np.zeros(1), counters=np.zeros(N_COUNTERS, np.int64),
                         E_half=np.zeros(nc))
        if paths and "path" not in state:
            state["path"] = np.zeros((nc, nl))
            state["mrw_path"] = np.zeros(nc)
        fz = None
        if frozen_T is not None:
            fz = np.ascontiguousarray(frozen_T, dtype=np.float64)
        ct = None
        if coef_T is not None:
            ct = np.ascontiguousarray(coef_T, dtype=np.float64)
        opts = _Opts(int(mrw), float(gamma), int(n_int_min), int(n_inc), int(max_events),
                     _p(fz) if fz is not None else None, _p(ct) if ct is not None else None)
        recs = np.zeros(max(n_recs, 1), REC_DTYPE)
        lib().ora_run(C.byref(self.model), C.byref(self.tables), C.byref(opts), n_packets,
                      n_total, seed, offset, _p(state["E_abs"]), _p(state["visits"]),
                      _p(state["n_abs"]), _p(state["n_mrw"]), _p(state["sed"]), _p(state["E_star"]),
                      _p(state["counters"]), _p(recs), n_recs, _p(state["E_half"]),
                      _p(state["path"]) if "path" in state else None,
                      _p(state["mrw_path"]) if "path" in state else None)
        state["recs"] = recs[:n_recs]
        state["eps"] = self.L_star / n_total
        return state

    def mean_intensity(self, T, state) -> np.ndarray:
        """J [n_cells, n_lambda] from a run's path tallies (run with paths=True)."""
        T = np.ascontiguousarray(T, dtype=np.float64)
        J = np.empty((self.n_cells, self.n_lambda))
        lib().ora_mean_intensity(C.byref(self.model), _p(T), _p(state["path"]),
                                 _p(state["mrw_path"]), _p(J))
        return J

    def raytrace_sed(self, T, J=None, cos_i=(0.7071067811865476,), n_sub: int = 4,
                     n_phi: int = 16) -> np.ndarray:
        """Ray-traced isotropic-equivalent luminosity per bin [n_inc, n_lambda]."""
        T = np.ascontiguousarray(T, dtype=np.float64)
        ci = np.ascontiguousarray(cos_i, dtype=np.float64)
        Jc = None if J is None else np.ascontiguousarray(J, dtype=np.float64)
        out = np.empty((len(ci), self.n_lambda))
        lib().ora_raytrace_sed(C.byref(self.model), C.byref(self.tables), _p(T),
                               _p(Jc) if Jc is not None else None, len(ci), _p(ci), int(n_sub),
                               int(n_phi), _p(out))
        return out

    def raytrace_image(self, T, J=None, cos_i=(0.7071067811865476,), n_sub: int = 4,
                       n_phi: int = 16) -> np.ndarray:
        """Intensity per ray and bin [n_inc, (n_r + 1) n_sub, n_phi, n_lambda]
        of the ray set of raytrace_sed, without the star."""
        T = np.ascontiguousarray(T, dtype=np.float64)
        ci = np.ascontiguousarray(cos_i, dtype=np.float64)
        Jc = None if J is None else np.ascontiguousarray(J, dtype=np.float64)
        out = np.empty((len(ci), (self.n_r + 1) * n_sub, n_phi, self.n_lambda))
        lib().ora_raytrace_image(C.byref(self.model), C.byref(self.tables), _p(T),
                                 _p(Jc) if Jc is not None else None, len(ci), _p(ci),
                                 int(n_sub), int(n_phi), _p(out))
        return out

    def visibility(self, img, cos_i, n_sub: int, n_phi: int, baselines, distance: float):
        """Visibility amplitudes [n_inc, n_base, n_lambda] of an image from
        raytrace_image (same cos_i, n_sub, n_phi) with the dimmed star;
        baselines [n_base, 2]: length (cm), position angle (rad)."""
        img = np.ascontiguousarray(img, dtype=np.float64)
        ci = np.ascontiguousarray(cos_i, dtype=np.float64)
        bl = np.ascontiguousarray(baselines, dtype=np.float64).reshape(-1, 2)
        assert img.shape == (len(ci), (self.n_r + 1) * n_sub, n_phi, self.n_lambda)
        out = np.empty((len(ci), len(bl), self.n_lambda))
        lib().ora_visibility(C.byref(self.model), C.byref(self.tables), _p(img), len(ci), _p(ci),
                             int(n_sub), int(n_phi), len(bl), _p(bl), float(distance), _p(out))
        return out

    def conv_stat(self, state, T_prev, s2_prev, n_min: int = 100):
        """Convergence statistic of a pass (its tallies in `state`) against
        the previous pass's T_prev and s2_prev, which are updated in place
        (start with zeros and -1 for the first pass).  Returns (R, rms
        relative change, rms noise, cells)."""
        out = np.zeros(4)
        assert T_prev.dtype == np.float64 and s2_prev.dtype == np.float64
        lib().ora_conv_stat(C.byref(self.model), C.byref(self.tables), _p(state["E_abs"]),
                            _p(state["E_half"]), _p(np.ascontiguousarray(state["visits"],
                                                                         dtype=np.uint32)),
                            int(n_min), _p(T_prev), _p(s2_prev), _p(out))
        return float(out[0]), float(out[1]), float(out[2]), int(out[3])

    def counters(self, state) -> dict:
        return dict(zip(COUNTER_NAMES, (int(v) for v in state["counters"])))

    def hydrostatic(self, T, M_star: float, mu_mol: float = 2.3, T_floor: float = 1.0,
                    return_cold: bool = False):
        """Density in vertical hydrostatic equilibrium for the temperatures T,
        each radial shell keeping the mass of the model's density; shells with
        a dusty cell at T <= 0 keep their density (their count is returned
        with return_cold)."""
        T = np.ascontiguousarray(T, dtype=np.float64)
        out = np.empty(self.n_cells)
        n_cold = lib().ora_hydrostatic(C.byref(self.model), _p(T), float(M_star), float(mu_mol),
                                       float(T_floor), _p(out))
        return (out, n_cold) if return_cold else out

    def pda_region(self, visits, n_abs, n_mrw, visits_min: int = 100, sigma_max: float = 0.0):
        """PDA region of a run: dusty cells with fewer than visits_min entries,
        or (sigma_max > 0) with photon noise 1/(4 sqrt(N_abs + N_mrw)) above
        sigma_max."""
        v = np.ascontiguousarray(visits, dtype=np.uint32)
        a = np.ascontiguousarray(n_abs, dtype=np.uint32)
        m = np.ascontiguousarray(n_mrw, dtype=np.uint32)
        out = np.empty(self.n_cells, np.uint8)
        lib().ora_pda_region(C.byref(self.model), _p(v), _p(a), _p(m), int(visits_min),
                             float(sigma_max), _p(out))
        return out

    def mrw_deposit(self, cell: int, Tc: float, R0: float, s: float) -> float:
        """Energy per unit packet energy that one MRW step (escape variable s,
        sphere radius R0) deposits in `cell` at the temperature Tc."""
        return lib().ora_mrw_deposit(C.byref(self.model), C.byref(self.tables), int(cell),
                                     float(Tc), float(R0), float(s))

    def update_T(self, E_abs) -> np.ndarray:
        E = np.ascontiguousarray(E_abs, dtype=np.float64)
        T = np.empty(self.n_cells)
        lib().ora_update_T(C.byref(self.model), C.byref(self.tables), _p(E), _p(T))
        return T

    # -- PDA --------------------------------------------------------------
    def pda(self, T_mc, region, max_sweeps: int = 50, tol: float = 1e-8):
        T_mc = np.ascontiguousarray(T_mc, dtype=np.float64)
        reg = np.ascontiguousarray(region, dtype=np.uint8)
        T_out = np.empty(self.n_cells)
        reg_out = np.empty(self.n_cells, np.uint8)
        sweeps = C.c_int(0)
        change = C.c_double(0.0)
        conv = C.c_int(0)
        rc = lib().ora_pda(C.byref(self.model), C.byref(self.tables), _p(T_mc), _p(reg),
                           _p(T_out), _p(reg_out), max_sweeps, tol, C.byref(sweeps),
                           C.byref(change), C.byref(conv))
        if rc != 0:
            raise RuntimeError("oracle PDA: matrix not positive definite")
        self.last_pda_converged = bool(conv.value)
        return T_out, reg_out, sweeps.value, change.value

    def pda_linear(self, T_D, T_bc, region, kscale=None):
        T_D = np.ascontiguousarray(T_D, dtype=np.float64)
        T_bc = np.ascontiguousarray(T_bc, dtype=np.float64)
        reg = np.ascontiguousarray(region, dtype=np.uint8)
        ks = None if kscale is None else np.ascontiguousarray(kscale, dtype=np.float64)
        T_out = np.empty(self.n_cells)
        rc = lib().ora_pda_linear(C.byref(self.model), C.byref(self.tables), _p(T_D), _p(T_bc),
                                  _p(ks) if ks is not None else None, _p(reg), _p(T_out))
        if rc != 0:
            raise RuntimeError("oracle PDA: matrix not positive definite")
        return T_out


def _pda_grad_direct(self, T_D, T_bc, region, dJdT, cells, kscale=None):
    """dJ/dlog rho and dJ/ds of the linear PDA (D frozen at T_D) for the
    listed cells, by the direct method (one solve per parameter)."""
    T_D = np.ascontiguousarray(T_D, dtype=np.float64)
    T_bc = np.ascontiguousarray(T_bc, dtype=np.float64)
    reg = np.ascontiguousarray(region, dtype=np.uint8)
    g = np.ascontiguousarray(dJdT, dtype=np.float64)
    cl = np.ascontiguousarray(cells, dtype=np.int32)
    ks = None if kscale is None else np.ascontiguousarray(kscale, dtype=np.float64)
    gr = np.empty(len(cl))
    gs = np.empty(len(cl))
    rc = lib().ora_pda_grad_direct(C.byref(self.model), C.byref(self.tables), _p(T_D), _p(T_bc),
                                   _p(ks) if ks is not None else None, _p(reg), _p(g), _p(cl),
                                   len(cl), _p(gr), _p(gs))
    if rc != 0:
        raise RuntimeError("oracle PDA: matrix not positive definite")
    return gr, gs


Oracle.pda_grad_direct = _pda_grad_direct


def _pda_nonlinear(self, T_bc, region, kscale=None, max_sweeps: int = 200, tol: float = 1e-13):
    """Nonlinear PDA for differentiation: Picard to the fixed point from T_bc
    (D from the current T), Dirichlet T_bc outside the region.  Returns
    (T, sweeps, last relative change)."""
    T_bc = np.ascontiguousarray(T_bc, dtype=np.float64)
    reg = np.ascontiguousarray(region, dtype=np.uint8)
    ks = None if kscale is None else np.ascontiguousarray(kscale, dtype=np.float64)
    T_out = np.empty(self.n_cells)
    sweeps = C.c_int(0)
    change = C.c_double(0.0)
    rc = lib().ora_pda_nl(C.byref(self.model), C.byref(self.tables), _p(T_bc),
                          _p(ks) if ks is not None else None, _p(reg), max_sweeps, tol,
                          _p(T_out), C.byref(sweeps), C.byref(change))
    if rc != 0:
        raise RuntimeError("oracle PDA: matrix not positive definite")
    return T_out, sweeps.value, change.value


def _pda_nl_grad_direct(self, T_bc, region, dJdT, cells, kscale=None, max_sweeps: int = 200,
                        tol: float = 1e-13):
    """dJ/dlog rho and dJ/ds of the nonlinear PDA for the listed cells, by the
    direct method on its Jacobian.  Returns (T, g_logrho, g_kscale)."""
    T_bc = np.ascontiguousarray(T_bc, dtype=np.float64)
    reg = np.ascontiguousarray(region, dtype=np.uint8)
    g = np.ascontiguousarray(dJdT, dtype=np.float64)
    cl = np.ascontiguousarray(cells, dtype=np.int32)
    ks = None if kscale is None else np.ascontiguousarray(kscale, dtype=np.float64)
    T_out = np.empty(self.n_cells)
    gr = np.empty(len(cl))
    gs = np.empty(len(cl))
    rc = lib().ora_pda_nl_grad_direct(C.byref(self.model), C.byref(self.tables), _p(T_bc),
                                      _p(ks) if ks is not None else None, _p(reg), max_sweeps,
                                      tol, _p(g), _p(cl), len(cl), _p(T_out), _p(gr), _p(gs))
    if rc != 0:
        raise RuntimeError("oracle nonlinear PDA: solve failed")
    return T_out, gr, gs


Oracle.pda_nonlinear = _pda_nonlinear
Oracle.pda_nl_grad_direct = _pda_nl_grad_direct
