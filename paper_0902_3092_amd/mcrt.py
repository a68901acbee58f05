"""Python binding of the mcrt C-ABI (include/mcrt.h): argument marshalling only.

Every step of the method runs in the HIP library ``libmcrt.so``; this module
passes device pointers of torch tensors and the current HIP stream through
ctypes, with the same names as the C entry points.  If the library is missing
it raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcrt.so")
_lib = None

OK, E_ARG, E_OOM, E_HIP, E_NOT_CONVERGED, E_STUCK, E_SINGULAR_REGION = 0, -1, -2, -3, -4, -5, -6
TAIL_CAP = 8192   # packets the hand-off buffer holds (MCRT_TAIL_CAP)
FP64, FP32 = 0, 1
GET_E_ABS, GET_VISITS, GET_N_ABS, GET_N_MRW, GET_T, GET_REGION, GET_COUNTERS, GET_E_STAR, \
    GET_TABLES, GET_RHO, GET_HYDRO_COLD, GET_E_HALF, GET_PATH, GET_MRW_PATH = range(14)
COUNTER_NAMES = ["escaped", "star", "capped", "cross", "scat", "abs", "mrw", "launch", "handed",
                 "in_runs"]

EXPORTS = ["mcrt_default_options", "mcrt_setup", "mcrt_destroy", "mcrt_reset", "mcrt_trace",
           "mcrt_update_T", "mcrt_pda_solve", "mcrt_sed", "mcrt_locate", "mcrt_get",
           "mcrt_get_size", "mcrt_set_T", "mcrt_hydrostatic", "mcrt_strerror", "mcrt_last_error",
           "mcrt_batch_run", "mcrt_pda_linear", "mcrt_pda_adjoint", "mcrt_pda_solve_noalloc",
           "mcrt_batch_pda", "mcrt_convergence", "mcrt_batch_converge", "mcrt_mean_intensity",
           "mcrt_raytrace_sed", "mcrt_region_mask", "mcrt_pda_nonlinear",
           "mcrt_pda_nonlinear_adjoint", "mcrt_raytrace_image", "mcrt_visibility"]


class McrtError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        L = lib()
        msg = "%s: %s (%s)" % (where, L.mcrt_strerror(code).decode(), L.mcrt_last_error().decode())
        super().__init__(msg)


class Grid(C.Structure):
    _fields_ = [("n_r", C.c_int32), ("n_mu", C.c_int32), ("r_edges", C.c_void_p),
                ("mu_edges", C.c_void_p)]


class Star(C.Structure):
    _fields_ = [("T_star", C.c_double), ("R_star", C.c_double)]


class Dust(C.Structure):
    _fields_ = [("n_lambda", C.c_int32), ("n_species", C.c_int32), ("lambda_edges", C.c_void_p),
                ("kappa_abs", C.c_void_p), ("kappa_sca", C.c_void_p), ("mass_frac", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("mrw", C.c_int32), ("gamma", C.c_double),
                ("n_int_min", C.c_int32), ("n_T", C.c_int32), ("T_lo", C.c_double),
                ("T_hi", C.c_double), ("n_inc", C.c_int32), ("max_events", C.c_int64),
                ("pda_visits", C.c_int32), ("pda_max_sweeps", C.c_int32),
                ("pda_tol", C.c_double), ("cg_max_iter", C.c_int32), ("cg_tol", C.c_double),
                ("mrw_coef_T", C.c_int32), ("block_size", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("pda_solver", C.c_int32),
                ("pda_precond", C.c_int32), ("wave_events", C.c_int64),
                ("g_asym", C.c_double), ("hydro_M_star", C.c_double), ("hydro_mu", C.c_double),
                ("pda_sigma", C.c_double), ("conv_split", C.c_int32), ("j_tally", C.c_int32),
                ("wave_runahead", C.c_int32), ("handoff_live", C.c_int32)]


class ConvStats(C.Structure):
    _fields_ = [("passes", C.c_int32), ("converged_pass", C.c_int32), ("R_last", C.c_double),
                ("dT_rms", C.c_double), ("noise_rms", C.c_double), ("cells", C.c_int32)]


class PdaStats(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("cg_iters_total", C.c_int32),
                ("cg_iters_last", C.c_int32), ("n_region", C.c_int32),
                ("n_isolated", C.c_int32), ("last_change", C.c_double),
                ("last_residual", C.c_double), ("converged", C.c_int32)]


REC_DTYPE = np.dtype([("fate", np.int32), ("k", np.int32), ("n_cross", np.int64),
                      ("n_scat", np.int64), ("n_abs", np.int64), ("n_mrw", np.int64),
                      ("n_draws", np.int64), ("x", np.float64), ("y", np.float64),
                      ("z", np.float64), ("u", np.float64), ("v", np.float64),
                      ("w", np.float64)])


def lib():
    """Load libmcrt.so (built by build.py).  Raises if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmcrt.so is not built (run paper_0902_3092_amd/build.py or "
                               "__graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
        L.mcrt_default_options.argtypes = [vp]
        L.mcrt_default_options.restype = None
        L.mcrt_setup.argtypes = [vp, vp, vp, vp, vp, vp]
        L.mcrt_destroy.argtypes = [vp]
        L.mcrt_destroy.restype = None
        L.mcrt_reset.argtypes = [vp, vp]
        L.mcrt_trace.argtypes = [vp, u64, u64, u64, u64, vp, vp, i64, vp]
        L.mcrt_update_T.argtypes = [vp, vp, vp]
        L.mcrt_pda_solve.argtypes = [vp, vp, vp, vp]
        L.mcrt_sed.argtypes = [vp, vp, vp]
        L.mcrt_locate.argtypes = [vp, vp, i64, vp, vp]
        L.mcrt_get.argtypes = [vp, C.c_int, vp, vp]
        L.mcrt_get_size.argtypes = [vp, C.c_int]
        L.mcrt_get_size.restype = i64
        L.mcrt_set_T.argtypes = [vp, vp, vp]
        L.mcrt_hydrostatic.argtypes = [vp, C.c_double, C.c_double, vp, vp]
        L.mcrt_strerror.argtypes = [C.c_int]
        L.mcrt_strerror.restype = C.c_char_p
        L.mcrt_last_error.argtypes = []
        L.mcrt_last_error.restype = C.c_char_p
        L.mcrt_batch_run.argtypes = [vp, C.c_int, vp, vp, C.c_int, C.c_int, vp, vp]
        L.mcrt_pda_linear.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.mcrt_pda_adjoint.argtypes = [vp, vp, vp, vp, vp]
        L.mcrt_pda_nonlinear.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.mcrt_pda_nonlinear_adjoint.argtypes = [vp, vp, vp, vp, vp, vp]
        L.mcrt_pda_solve_noalloc.argtypes = [vp, vp, vp, vp]
        L.mcrt_batch_pda.argtypes = [vp, C.c_int, vp, vp]
        L.mcrt_convergence.argtypes = [vp, i32, i32, vp, vp]
        L.mcrt_mean_intensity.argtypes = [vp, vp, vp, vp]
        L.mcrt_region_mask.argtypes = [vp, i32, C.c_double, vp, vp]
        L.mcrt_raytrace_sed.argtypes = [vp, vp, vp, i32, vp, i32, i32, vp, vp]
        L.mcrt_raytrace_image.argtypes = [vp, vp, vp, i32, vp, i32, i32, vp, vp]
        L.mcrt_visibility.argtypes = [vp, vp, i32, vp, i32, i32, i32, vp, C.c_double, vp, vp]
        L.mcrt_batch_converge.argtypes = [vp, C.c_int, vp, vp, C.c_int, i32, C.c_double, C.c_int,
                                          vp, vp, vp, vp]
        _lib = L
    return _lib


def default_options() -> Options:
    o = Options()
    lib().mcrt_default_options(C.byref(o))
    return o


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _check(rc, where, allow=()):
    if rc != OK and rc not in allow:
        raise McrtError(rc, where)
    return rc


class Context:
    """mcrt_setup on one disk model (any object with the workload Disk fields)."""

    def __init__(self, disk, *, precision: str = "fp64", mrw: bool = False, gamma: float = 3.0,
                 n_int_min: int = 20, n_T: int = 256, T_lo: float = 1.0, T_hi: float = 1.0e4,
                 n_inc: int = 10, max_events: int = 1 << 30, pda_visits: int = 100,
                 pda_max_sweeps: int = 50, pda_tol: float = 1e-8, cg_max_iter: int = 20000,
                 cg_tol: float = 1e-12, mrw_coef_T: int = 0, block_size: int = 0,
                 blocks_per_cu: int = 0, pda_solver: int = 0, pda_precond: int = 1, wave_events: int = 2048, rho=None,
                 g_asym: float = 0.0, hydro_M_star: float = 0.0, hydro_mu: float = 2.3,
                 pda_sigma: float = 0.0, conv_split: int = 0, j_tally: int = 0,
                 wave_runahead: int = 0, handoff_live: int = 0):
        import torch  # noqa: F401  (the device context)
        L = lib()
        o = default_options()
        o.precision = FP32 if precision == "fp32" else FP64
        o.mrw = int(mrw)
        o.gamma, o.n_int_min, o.n_T, o.T_lo, o.T_hi = gamma, n_int_min, n_T, T_lo, T_hi
        o.n_inc, o.max_events, o.pda_visits = n_inc, max_events, pda_visits
        o.pda_max_sweeps, o.pda_tol, o.cg_max_iter, o.cg_tol = pda_max_sweeps, pda_tol, \
            cg_max_iter, cg_tol
        o.mrw_coef_T, o.block_size, o.blocks_per_cu = mrw_coef_T, block_size, blocks_per_cu
        o.pda_solver = pda_solver
        o.pda_precond = pda_precond
        o.wave_events = wave_events
        o.g_asym = g_asym
        o.hydro_M_star, o.hydro_mu = hydro_M_star, hydro_mu
        o.pda_sigma = pda_sigma
        o.conv_split = int(conv_split)
        o.j_tally = int(j_tally)
        o.wave_runahead = int(wave_runahead)
        o.handoff_live = int(handoff_live)
        self.options = o
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        self._keep = [f64(disk.r_edges), f64(disk.mu_edges), f64(disk.lambda_edges),
                      f64(disk.kappa_abs), f64(disk.kappa_sca), f64(disk.mass_frac),
                      f64(disk.rho if rho is None else rho)]
        re, me, le, ka, ks, mf, rh = self._keep
        g = Grid(len(re) - 1, len(me) - 1, re.ctypes.data, me.ctypes.data)
        s = Star(float(disk.T_star), float(disk.R_star))
        d = Dust(len(le) - 1, ka.shape[0], le.ctypes.data, ka.ctypes.data, ks.ctypes.data,
                 mf.ctypes.data)
        h = C.c_void_p()
        _check(L.mcrt_setup(C.byref(h), C.byref(g), C.byref(s), C.byref(d), rh.ctypes.data,
                            C.byref(o)), "mcrt_setup")
        self.handle = h
        self.n_r, self.n_mu, self.n_lambda = g.n_r, g.n_mu, d.n_lambda
        self.n_cells = self.n_r * self.n_mu
        self.n_inc = n_inc
        # count of calls that replace what mcrt_pda_adjoint differentiates:
        # each mcrt_pda_linear starts a new generation, and any other call
        # that reuses the PDA scratch or the density ends it
        self._lin_gen = 0

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.mcrt_destroy(h)
            self.handle = None

    # -- entry points -------------------------------------------------------
    def reset(self, stream=None):
        _check(lib().mcrt_reset(self.handle, _stream(stream)), "mcrt_reset")

    def trace(self, n_packets: int, seed: int, *, n_total: Optional[int] = None, offset: int = 0,
              frozen_T=None, n_recs: int = 0, stream=None):
        """mcrt_trace; returns the packet records (torch uint8 buffer viewed as REC_DTYPE by
        records_numpy) when n_recs > 0."""
        import torch
        n_total = n_packets if n_total is None else n_total
        recs = None
        if n_recs > 0:
            recs = torch.zeros(n_recs * REC_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        if frozen_T is not None:
            assert frozen_T.dtype == torch.float64 and frozen_T.is_cuda
            assert frozen_T.numel() == self.n_cells
        rc = lib().mcrt_trace(self.handle, n_packets, n_total, seed, offset, _ptr(frozen_T),
                              _ptr(recs), n_recs, _stream(stream))
        _check(rc, "mcrt_trace", allow=(E_STUCK,))
        return recs

    @staticmethod
    def records_numpy(recs):
        return np.frombuffer(recs.cpu().numpy().tobytes(), dtype=REC_DTYPE)

    def update_T(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.n_cells, dtype=torch.float64, device="cuda")
        _check(lib().mcrt_update_T(self.handle, _ptr(out), _stream(stream)), "mcrt_update_T")
        return out

    def pda_solve(self, mask=None, stream=None) -> dict:
        self._lin_gen += 1
        st = PdaStats()
        rc = lib().mcrt_pda_solve(self.handle, _ptr(mask), C.byref(st), _stream(stream))
        _check(rc, "mcrt_pda_solve", allow=(E_SINGULAR_REGION,))
        out = {f: getattr(st, f) for f, _ in PdaStats._fields_}
        out["rc"] = rc
        return out

    def pda_solve_noalloc(self, mask=None, stream=None) -> dict:
        """mcrt_pda_solve_noalloc: the one-workgroup PDA solve with the
        library's fixed scratch (no device allocation)."""
        st = PdaStats()
        rc = lib().mcrt_pda_solve_noalloc(self.handle, _ptr(mask), C.byref(st), _stream(stream))
        _check(rc, "mcrt_pda_solve_noalloc", allow=(E_SINGULAR_REGION,))
        out = {f: getattr(st, f) for f, _ in PdaStats._fields_}
        out["rc"] = rc
        return out

    def sed(self, stream=None):
        import torch
        out = torch.empty((self.n_lambda, self.n_inc), dtype=torch.float64, device="cuda")
        _check(lib().mcrt_sed(self.handle, _ptr(out), _stream(stream)), "mcrt_sed")
        return out

    def locate(self, xyz, stream=None):
        import torch
        assert xyz.dtype == torch.float64 and xyz.is_cuda and xyz.is_contiguous()
        n = xyz.numel() // 3
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        _check(lib().mcrt_locate(self.handle, _ptr(xyz), n, _ptr(out), _stream(stream)),
               "mcrt_locate")
        return out

    def get(self, what: int, stream=None):
        import torch
        nbytes = lib().mcrt_get_size(self.handle, what)
        if nbytes < 0:
            raise McrtError(E_ARG, "mcrt_get_size")
        buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        _check(lib().mcrt_get(self.handle, what, _ptr(buf), _stream(stream)), "mcrt_get")
        dt = {GET_E_ABS: torch.float64, GET_VISITS: torch.int32, GET_N_ABS: torch.int32,
              GET_N_MRW: torch.int32, GET_T: torch.float64, GET_REGION: torch.uint8,
              GET_COUNTERS: torch.int64, GET_E_STAR: torch.float64,
              GET_TABLES: torch.float64, GET_RHO: torch.float64,
              GET_HYDRO_COLD: torch.int32, GET_E_HALF: torch.float64, GET_PATH: torch.float64,
              GET_MRW_PATH: torch.float64}[what]
        return buf.view(dt)

    def counters(self) -> dict:
        v = self.get(GET_COUNTERS).cpu().numpy()
        return dict(zip(COUNTER_NAMES, (int(x) for x in v)))

    def tables(self) -> dict:
        v = self.get(GET_TABLES).cpu().numpy()
        nT, nl = self.options.n_T, self.n_lambda
        out, q = {}, 0
        for name, n in (("T", nT), ("cdf", nT * nl), ("Drho", nT), ("kbar", nT),
                        ("star_cdf", nl), ("L_star", 1)):
            out[name] = v[q:q + n]
            q += n
        out["cdf"] = out["cdf"].reshape(nT, nl)
        out["L_star"] = float(out["L_star"][0])
        return out

    def convergence(self, n_min: int = 100, first: bool = False, stream=None):
        """mcrt_convergence on the current tallies: (R, rms change, rms noise,
        cells)."""
        out = (C.c_double * 4)()
        _check(lib().mcrt_convergence(self.handle, int(n_min), int(first), out, _stream(stream)),
               "mcrt_convergence")
        return float(out[0]), float(out[1]), float(out[2]), int(out[3])

    def region_mask(self, visits_min: int = 100, sigma_max: float = 0.0, stream=None):
        """mcrt_region_mask: the PDA region rule with these parameters on the
        current tallies, as a uint8 mask [n_cells]."""
        import torch
        m = torch.empty(self.n_cells, dtype=torch.uint8, device="cuda")
        _check(lib().mcrt_region_mask(self.handle, int(visits_min), float(sigma_max), _ptr(m),
                                      _stream(stream)), "mcrt_region_mask")
        return m

    def mean_intensity(self, T=None, stream=None):
        """mcrt_mean_intensity: J [n_cells, n_lambda] from the path tallies."""
        import torch
        J = torch.empty((self.n_cells, self.n_lambda), dtype=torch.float64, device="cuda")
        _check(lib().mcrt_mean_intensity(self.handle, _ptr(T), _ptr(J), _stream(stream)),
               "mcrt_mean_intensity")
        return J

    def raytrace_sed(self, T=None, J=None, cos_i=(0.7071067811865476,), n_sub: int = 4,
                     n_phi: int = 16, stream=None):
        """mcrt_raytrace_sed: isotropic-equivalent luminosity per bin
        [n_inc, n_lambda] at the inclinations cos_i."""
        import torch
        ci = (C.c_double * len(cos_i))(*[float(x) for x in cos_i])
        L = torch.empty((len(cos_i), self.n_lambda), dtype=torch.float64, device="cuda")
        _check(lib().mcrt_raytrace_sed(self.handle, _ptr(T), _ptr(J), len(cos_i), ci, int(n_sub),
                                       int(n_phi), _ptr(L), _stream(stream)), "mcrt_raytrace_sed")
        return L

    def raytrace_image(self, T=None, J=None, cos_i=(0.7071067811865476,), n_sub: int = 4,
                       n_phi: int = 16, stream=None):
        """mcrt_raytrace_image: the intensity per ray and bin
        [n_inc, (n_r + 1) n_sub, n_phi, n_lambda] of raytrace_sed's rays,
        without the star."""
        import torch
        ci = (C.c_double * len(cos_i))(*[float(x) for x in cos_i])
        img = torch.empty((len(cos_i), (self.n_r + 1) * int(n_sub), int(n_phi), self.n_lambda),
                          dtype=torch.float64, device="cuda")
        _check(lib().mcrt_raytrace_image(self.handle, _ptr(T), _ptr(J), len(cos_i), ci,
                                         int(n_sub), int(n_phi), _ptr(img), _stream(stream)),
               "mcrt_raytrace_image")
        return img

    def visibility(self, image, cos_i, n_sub: int, n_phi: int, baselines, distance: float,
                   stream=None):
        """mcrt_visibility: amplitudes [n_inc, n_base, n_lambda] of an image
        from raytrace_image (the same cos_i, n_sub, n_phi) with the dimmed
        star; baselines [n_base, 2]: length (cm), position angle (rad)."""
        import torch
        shape = (len(cos_i), (self.n_r + 1) * int(n_sub), int(n_phi), self.n_lambda)
        if tuple(image.shape) != shape or image.dtype != torch.float64 or \
                not image.is_contiguous():
            raise ValueError("image must be a contiguous float64 tensor of shape %s" % (shape,))
        ci = (C.c_double * len(cos_i))(*[float(x) for x in cos_i])
        bl = np.ascontiguousarray(baselines, dtype=np.float64).reshape(-1, 2)
        bh = (C.c_double * bl.size)(*bl.reshape(-1).tolist())
        V = torch.empty((len(cos_i), len(bl), self.n_lambda), dtype=torch.float64, device="cuda")
        _check(lib().mcrt_visibility(self.handle, _ptr(image), len(cos_i), ci, int(n_sub),
                                     int(n_phi), len(bl), bh, float(distance), _ptr(V),
                                     _stream(stream)), "mcrt_visibility")
        return V

    def set_T(self, T, stream=None):
        _check(lib().mcrt_set_T(self.handle, _ptr(T), _stream(stream)), "mcrt_set_T")

    def hydrostatic(self, M_star: float, mu_mol: float = 2.3, stream=None):
        """mcrt_hydrostatic: density in vertical hydrostatic equilibrium for the
        current T (replaces the context's); returns a copy [n_cells]."""
        import torch
        rho = torch.empty(self.n_cells, dtype=torch.float64, device="cuda")
        self._lin_gen += 1
        _check(lib().mcrt_hydrostatic(self.handle, float(M_star), float(mu_mol), _ptr(rho),
                                      _stream(stream)), "mcrt_hydrostatic")
        return rho

    def pda_linear(self, mask, T_D, T_bc, rho=None, kscale=None, stream=None):
        """mcrt_pda_linear: one PDA solve with D frozen at T_D; returns (T, stats)."""
        import torch
        T_out = torch.empty(self.n_cells, dtype=torch.float64, device="cuda")
        st = PdaStats()
        self._lin_gen += 1
        rc = lib().mcrt_pda_linear(self.handle, _ptr(mask), _ptr(rho), _ptr(kscale), _ptr(T_D),
                                   _ptr(T_bc), _ptr(T_out), C.byref(st), _stream(stream))
        _check(rc, "mcrt_pda_linear")
        return T_out, {f: getattr(st, f) for f, _ in PdaStats._fields_}

    def pda_adjoint(self, dJdT, stream=None):
        """mcrt_pda_adjoint of the last pda_linear: (dJ/dlog rho, dJ/ds)."""
        import torch
        g_r = torch.empty(self.n_cells, dtype=torch.float64, device="cuda")
        g_s = torch.empty(self.n_cells, dtype=torch.float64, device="cuda")
        rc = lib().mcrt_pda_adjoint(self.handle, _ptr(dJdT.contiguous()), _ptr(g_r), _ptr(g_s),
                                    _stream(stream))
        _check(rc, "mcrt_pda_adjoint")
        return g_r, g_s


    def pda_nonlinear(self, mask, T_bc, rho=None, kscale=None, stream=None):
        """mcrt_pda_nonlinear: Picard to the fixed point with D = D(T), from
        T_bc; returns (T, stats)."""
        import torch
        T_out = torch.empty(self.n_cells, dtype=torch.float64, device="cuda")
        st = PdaStats()
        self._lin_gen += 1
        rc = lib().mcrt_pda_nonlinear(self.handle, _ptr(mask), _ptr(rho), _ptr(kscale),
                                      _ptr(T_bc), _ptr(T_out), C.byref(st), _stream(stream))
        _check(rc, "mcrt_pda_nonlinear")
        return T_out, {f: getattr(st, f) for f, _ in PdaStats._fields_}

    def pda_nonlinear_adjoint(self, dJdT, stream=None, stats=False):
        """mcrt_pda_nonlinear_adjoint of the last pda_nonlinear: (dJ/dlog rho,
        dJ/ds), and its statistics with stats=True."""
        import torch
        g_r = torch.empty(self.n_cells, dtype=torch.float64, device="cuda")
        g_s = torch.empty(self.n_cells, dtype=torch.float64, device="cuda")
        st = PdaStats()
        rc = lib().mcrt_pda_nonlinear_adjoint(self.handle, _ptr(dJdT.contiguous()), _ptr(g_r),
                                              _ptr(g_s), C.byref(st), _stream(stream))
        _check(rc, "mcrt_pda_nonlinear_adjoint")
        if stats:
            return g_r, g_s, {f: getattr(st, f) for f, _ in PdaStats._fields_}
        return g_r, g_s


def batch_run_rc(contexts, n_packets, seeds, n_iter: int = 5, use_graph: bool = True,
                 stream=None, allow=(E_NOT_CONVERGED, E_STUCK)):
    """mcrt_batch_run over Context objects; returns (the per-disk PDA statistics
    of the last pass, the return code).  Codes outside `allow` raise."""
    n = len(contexts)
    handles = (C.c_void_p * n)(*[c.handle.value for c in contexts])
    npk = (C.c_uint64 * n)(*[int(x) for x in n_packets])
    sd = (C.c_uint64 * n)(*[int(x) for x in seeds])
    stats = (PdaStats * n)()
    for c in contexts:
        c._lin_gen += 1      # the batch overwrites what a linear PDA solve kept
    rc = lib().mcrt_batch_run(handles, n, npk, sd, n_iter, int(use_graph), stats,
                              _stream(stream))
    _check(rc, "mcrt_batch_run", allow=allow)
    return [{f: getattr(s, f) for f, _ in PdaStats._fields_} for s in stats], rc


def batch_run(contexts, n_packets, seeds, n_iter: int = 5, use_graph: bool = True,
              stream=None):
    """mcrt_batch_run over Context objects; returns the per-disk PDA statistics
    of the last pass.  Raises on any code but MCRT_OK."""
    return batch_run_rc(contexts, n_packets, seeds, n_iter, use_graph, stream, allow=())[0]


def batch_converge(contexts, n_packets, seeds, max_iter: int = 10, n_min: int = 100,
                   threshold: float = 3.0, use_graph: bool = True, stream=None,
                   allow=(E_NOT_CONVERGED,)):
    """mcrt_batch_converge over Context objects: passes until every disk's
    convergence statistic is below `threshold`.  Returns (PDA statistics of
    the last pass, per-disk convergence records with the R of every pass, the
    return code).  Codes outside `allow` raise."""
    n = len(contexts)
    handles = (C.c_void_p * n)(*[c.handle.value for c in contexts])
    npk = (C.c_uint64 * n)(*[int(x) for x in n_packets])
    sd = (C.c_uint64 * n)(*[int(x) for x in seeds])
    stats = (PdaStats * n)()
    conv = (ConvStats * n)()
    hist = (C.c_double * (n * max_iter))()
    for c in contexts:
        c._lin_gen += 1
    rc = lib().mcrt_batch_converge(handles, n, npk, sd, int(max_iter), int(n_min),
                                   float(threshold), int(use_graph), stats, conv, hist,
                                   _stream(stream))
    _check(rc, "mcrt_batch_converge", allow=allow)
    recs = []
    for d in range(n):
        r = {f: getattr(conv[d], f) for f, _ in ConvStats._fields_}
        r["R"] = [hist[d * max_iter + k] for k in range(r["passes"])]
        recs.append(r)
    return [{f: getattr(s_, f) for f, _ in PdaStats._fields_} for s_ in stats], recs, rc


def batch_pda(contexts, stream=None, allow=(E_SINGULAR_REGION,)):
    """mcrt_batch_pda: the PDA of every context in one launch; returns (the
    per-disk statistics, the return code).  Codes outside `allow` raise."""
    n = len(contexts)
    handles = (C.c_void_p * n)(*[c.handle.value for c in contexts])
    stats = (PdaStats * n)()
    for c in contexts:
        c._lin_gen += 1
    rc = lib().mcrt_batch_pda(handles, n, stats, _stream(stream))
    _check(rc, "mcrt_batch_pda", allow=allow)
    return [{f: getattr(s, f) for f, _ in PdaStats._fields_} for s in stats], rc
