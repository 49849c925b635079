"""slhjb: MI355X semi-Lagrangian HJB solver (Reisinger & Rotaetxe Arto, arXiv:1605.04821).

Thin ctypes binding of ``libslhjb.so`` (C ABI in ``include/slhjb.h``).  This module only marshals
arguments: every step of the method runs in the library's HIP kernels.  Device arrays are torch
tensors on the GPU (contiguous, dtype as documented); PyTorch supplies memory and the stream.
There is no CPU fallback: if the library is missing the import fails.
"""
from __future__ import annotations

import ctypes
import math
import dataclasses
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libslhjb.so")

HJB_OK, HJB_EINVAL, HJB_EDEVICE, HJB_ENOMEM = 0, -1, -2, -3
HJB_ENOCONV_KRYLOV, HJB_ENOCONV_PI, HJB_ENONFINITE, HJB_EUNSUPPORTED = -4, -5, -6, -7
PREC_FP64, PREC_MIXED = 0, 1
COEF_CONST, COEF_XSCALED, COEF_FIELD = 0, 1, 2
PRECOND_NONE, PRECOND_JACOBI, PRECOND_VCYCLE, PRECOND_AMG = 0, 1, 2, 3
KRYLOV_FGMRES, KRYLOV_BICGSTAB = 0, 1
COARSE_REDISCRETIZED, COARSE_GALERKIN = 0, 1
FLAG_POSITIVITY, FLAG_NEAR_TIES = 1, 2

EXPORTED = ["hjb_amg_level", "hjb_coarse_operator", "hjb_desc_default", "hjb_setup", "hjb_set_stream", "hjb_set_options", "hjb_policy_sweep",
            "hjb_policy_sweep_noalloc", "hjb_apply",
            "hjb_linsolve", "hjb_step", "hjb_solve", "hjb_adjoint", "hjb_apply_transposed", "hjb_profile_enable",
            "hjb_profile_read", "hjb_profile_sample", "hjb_destroy", "hjb_last_error", "hjb_setup_batch", "hjb_batch_layout",
            "hjb_batch_set_stream", "hjb_batch_set_tile_widths", "hjb_batch_autotune", "hjb_solve_batch", "hjb_destroy_batch", "hjb_set_tile_width", "hjb_autotune"]
KERNEL_APPLY, KERNEL_SMOOTH, KERNEL_MG_RESID, KERNEL_DOT, KERNEL_AXPY, KERNEL_SWEEP = range(6)
KERNEL_NAMES = {KERNEL_APPLY: "apply", KERNEL_SMOOTH: "smooth", KERNEL_MG_RESID: "mg_residual",
                KERNEL_DOT: "multidot", KERNEL_AXPY: "multiaxpy", KERNEL_SWEEP: "sweep"}


class HJBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"slhjb error {code}: {msg}")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("lo", ctypes.c_double * 3),
                ("h", ctypes.c_double), ("K", ctypes.c_int32), ("P", ctypes.c_int32),
                ("coef_model", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("sigma", ctypes.c_void_p), ("drift", ctypes.c_void_p), ("c", ctypes.c_void_p),
                ("precision", ctypes.c_int32), ("precond", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("max_krylov", ctypes.c_int32), ("max_pi", ctypes.c_int32), ("nu1", ctypes.c_int32),
                ("nu2", ctypes.c_int32), ("coarse_sweeps", ctypes.c_int32), ("min_coarse", ctypes.c_int32),
                ("omega", ctypes.c_double), ("rtol_inf", ctypes.c_double), ("tau_rel", ctypes.c_double),
                ("pi_eta", ctypes.c_double), ("use_graphs", ctypes.c_int32), ("f_per_control", ctypes.c_int32),
                ("certified_skip", ctypes.c_int32), ("max_levels", ctypes.c_int32),
                ("nu_tight", ctypes.c_int32), ("coarse_sweeps_t", ctypes.c_int32),
                ("krylov", ctypes.c_int32), ("coarse_op", ctypes.c_int32), ("kcycle_levels", ctypes.c_int32),
                ("value_stride", ctypes.c_int32), ("amg_reuse", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


class StepStats(ctypes.Structure):
    _fields_ = [("pi_iters", ctypes.c_int32), ("krylov_total", ctypes.c_int32), ("krylov_max", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("res_inf", ctypes.c_double), ("cert_bound", ctypes.c_double),
                ("n_changed_first", ctypes.c_int64), ("n_near_ties", ctypes.c_int64)]


class SolveStats(ctypes.Structure):
    _fields_ = [("steps_done", ctypes.c_int32), ("flags", ctypes.c_int32), ("krylov_total", ctypes.c_int64),
                ("pi_total", ctypes.c_int64), ("max_cert_bound", ctypes.c_double),
                ("near_ties_total", ctypes.c_int64)]


class AdjointStats(ctypes.Structure):
    _fields_ = [("krylov_recompute", ctypes.c_int64), ("krylov_adjoint", ctypes.c_int64),
                ("max_res_adjoint", ctypes.c_double)]


def _load():
    # torch's HIP runtime must be loaded first: the library's libamdhip64 dependency then binds to it
    # (same soname) and both share one runtime and one set of streams
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libslhjb.so not built ({LIB_PATH}); run __graft_entry__.build() or "
                          f"python paper_1605_04821_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    vp, d, i32, i64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int64
    L.hjb_desc_default.argtypes = [ctypes.POINTER(Desc)]
    L.hjb_desc_default.restype = None
    L.hjb_setup.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(vp)]
    L.hjb_setup.restype = ctypes.c_int
    L.hjb_set_stream.argtypes = [vp, vp]
    L.hjb_set_options.argtypes = [vp, ctypes.POINTER(Desc)]
    L.hjb_policy_sweep.argtypes = [vp, vp, vp, vp, vp, d, d, d, d, vp, vp, vp, vp, vp,
                                   ctypes.POINTER(i64), ctypes.POINTER(d)]
    L.hjb_policy_sweep_noalloc.argtypes = [vp, vp, vp, vp, vp, d, d, d, d, vp, vp, vp, vp, vp,
                                           ctypes.POINTER(i64), ctypes.POINTER(d)]
    L.hjb_apply.argtypes = [vp, vp, vp, vp, d, d, d]
    L.hjb_coarse_operator.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i64), vp, vp]
    L.hjb_amg_level.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i32), vp, vp, vp]
    L.hjb_linsolve.argtypes = [vp, vp, vp, vp, vp, d, d, d, d, vp, ctypes.POINTER(StepStats)]
    L.hjb_step.argtypes = [vp, vp, vp, vp, vp, d, d, d, d, vp, vp, d, ctypes.POINTER(StepStats)]
    L.hjb_solve.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp, vp, d, vp, vp, vp, ctypes.POINTER(SolveStats)]
    L.hjb_adjoint.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, d, vp, vp, vp, vp, vp, vp, ctypes.POINTER(d),
                              ctypes.POINTER(AdjointStats)]
    L.hjb_apply_transposed.argtypes = [vp, vp, vp, vp, d, d, d]
    L.hjb_setup_batch.argtypes = [ctypes.POINTER(Desc), i32, ctypes.POINTER(vp)]
    L.hjb_batch_layout.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.hjb_batch_set_stream.argtypes = [vp, vp]
    L.hjb_batch_set_tile_widths.argtypes = [vp, ctypes.POINTER(i32)]
    L.hjb_batch_autotune.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(i32)]
    L.hjb_solve_batch.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, d, vp, vp, ctypes.POINTER(SolveStats)]
    L.hjb_destroy_batch.argtypes = [vp]
    L.hjb_destroy_batch.restype = None
    L.hjb_set_tile_width.argtypes = [vp, i32]
    L.hjb_autotune.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(i32), ctypes.POINTER(d)]
    L.hjb_profile_enable.argtypes = [vp, i32, i32]
    L.hjb_profile_read.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(d)]
    L.hjb_profile_sample.argtypes = [vp, i32]
    L.hjb_destroy.argtypes = [vp]
    L.hjb_destroy.restype = None
    L.hjb_last_error.argtypes = []
    L.hjb_last_error.restype = ctypes.c_char_p
    return L


_lib = _load()


def lib():
    return _lib


def _check(rc: int):
    if rc != HJB_OK:
        raise HJBError(rc, _lib.hjb_last_error().decode())


def _ptr(t) -> Optional[int]:
    """Device pointer of a contiguous CUDA tensor (None passes NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _setup_stream():
    """torch's current stream (initialising torch's device first), or NULL without a device: setup then
    reports HJB_EDEVICE itself."""
    import torch
    return _stream() if torch.cuda.is_available() else None


@dataclass
class Options:
    precision: int = PREC_FP64
    precond: int = PRECOND_VCYCLE
    restart: int = 10
    max_krylov: int = 600
    max_pi: int = 50
    nu1: int = 3
    nu2: int = 3
    coarse_sweeps: int = 4
    min_coarse: int = 17
    omega: float = 0.9
    rtol_inf: float = 1e-13
    tau_rel: float = 1e-13
    pi_eta: float = 0.35
    use_graphs: int = 1
    certified_skip: int = 1
    max_levels: int = 2
    nu_tight: int = 4
    coarse_sweeps_t: int = 2
    krylov: int = 0
    coarse_op: int = 0
    kcycle_levels: int = -1
    value_stride: int = 1
    amg_reuse: int = 0


class Solver:
    """A handle for one grid and control set (hjb_setup).

    dim, n, lo, h: the box grid; sigma (K,P,dim), drift (K,dim) or None, c (K,) or None: host arrays.
    """

    def __init__(self, dim, n, lo, h, sigma, drift=None, c=None, options: Optional[Options] = None,
                 coef_model: int = COEF_CONST, K: Optional[int] = None, f_per_control: bool = False):
        """sigma: (K, P, dim) per control (constant or x-scaled model) or (N, P, dim) per node (field model,
        K then taken from drift, c or the argument)."""
        self.options = options or Options()
        sigma = np.ascontiguousarray(sigma, dtype=np.float64)
        K0, P, dd = sigma.shape
        if dd != dim:
            raise ValueError("sigma must have shape (K or N, P, dim)")
        if coef_model == COEF_FIELD:
            K = K if K is not None else (len(drift) if drift is not None else len(c))
        else:
            K = K0
        self._sigma = sigma
        self._drift = None if drift is None else np.ascontiguousarray(drift, dtype=np.float64)
        self._c = None if c is None else np.ascontiguousarray(c, dtype=np.float64)
        self.dim, self.K, self.P = dim, K, P
        self.n = tuple(int(v) for v in n)
        self.N = int(np.prod(self.n))
        self.h = float(h)
        desc = Desc()
        _lib.hjb_desc_default(ctypes.byref(desc))
        desc.dim = dim
        for a in range(3):
            desc.n[a] = self.n[a] if a < dim else 1
            desc.lo[a] = float(lo[a]) if a < dim else 0.0
        desc.h = self.h
        desc.K, desc.P = K, P
        desc.coef_model = int(coef_model)
        desc.f_per_control = 1 if f_per_control else 0
        desc.sigma = self._sigma.ctypes.data
        desc.drift = None if self._drift is None else self._drift.ctypes.data
        desc.c = None if self._c is None else self._c.ctypes.data
        self._fill_options(desc, self.options)
        desc.stream = _setup_stream()   # torch initialises the device first; the library works on its stream
        self._desc = desc
        h_ = ctypes.c_void_p()
        _check(_lib.hjb_setup(ctypes.byref(desc), ctypes.byref(h_)))
        self._h = h_

    @staticmethod
    def _fill_options(desc, o: Options):
        desc.precision, desc.precond, desc.restart = o.precision, o.precond, o.restart
        desc.max_krylov, desc.max_pi, desc.nu1, desc.nu2 = o.max_krylov, o.max_pi, o.nu1, o.nu2
        desc.coarse_sweeps, desc.min_coarse, desc.omega = o.coarse_sweeps, o.min_coarse, o.omega
        desc.rtol_inf, desc.tau_rel, desc.pi_eta = o.rtol_inf, o.tau_rel, o.pi_eta
        desc.use_graphs = o.use_graphs
        desc.certified_skip = o.certified_skip
        desc.max_levels = o.max_levels
        desc.nu_tight = o.nu_tight
        desc.coarse_sweeps_t = o.coarse_sweeps_t
        desc.krylov = o.krylov
        desc.coarse_op = o.coarse_op
        desc.kcycle_levels = o.kcycle_levels
        desc.value_stride = o.value_stride
        desc.amg_reuse = o.amg_reuse

    @classmethod
    def from_instance(cls, inst, options: Optional[Options] = None):
        fpc = np.ndim(inst.f0) == 2
        if inst.sigma is None:
            return cls(inst.dim, inst.n, inst.lo, inst.h, inst.sigma_node, inst.drift, inst.c, options,
                       coef_model=COEF_FIELD, K=inst.K, f_per_control=fpc)
        cm = COEF_XSCALED if getattr(inst, "coef_model", "const") == "xscaled" else COEF_CONST
        return cls(inst.dim, inst.n, inst.lo, inst.h, inst.sigma, inst.drift, inst.c, options, coef_model=cm,
                   f_per_control=fpc)

    def set_options(self, options: Options):
        self._fill_options(self._desc, options)
        _check(_lib.hjb_set_options(self._h, ctypes.byref(self._desc)))
        self.options = options

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.hjb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        _check(_lib.hjb_set_stream(self._h, _stream()))

    # ---- entry points --------------------------------------------------------------------------
    def policy_sweep(self, X, U, f0, f1, t_prev, dt, theta, s, alpha_in, alpha_out,
                     gmin=None, margin=None, ties=None):
        """hjb_policy_sweep; returns (n_changed, tau)."""
        self._sync_stream()
        nch = ctypes.c_int64(0)
        tau = ctypes.c_double(0.0)
        _check(_lib.hjb_policy_sweep(self._h, _ptr(X), _ptr(U), _ptr(f0), _ptr(f1), float(t_prev), float(dt),
                                     float(theta), float(s), _ptr(alpha_in), _ptr(alpha_out), _ptr(gmin),
                                     _ptr(margin), _ptr(ties), ctypes.byref(nch), ctypes.byref(tau)))
        return int(nch.value), float(tau.value)

    def policy_sweep_noalloc(self, X, U, f0, f1, t_prev, dt, theta, s, alpha_in, alpha_out,
                             gmin=None, margin=None, ties=None, read_back=True):
        """hjb_policy_sweep_noalloc (scratch in the library's static device array); returns (n_changed, tau),
        or (None, None) without read-back."""
        self._sync_stream()
        nch = ctypes.c_int64(0)
        tau = ctypes.c_double(0.0)
        _check(_lib.hjb_policy_sweep_noalloc(self._h, _ptr(X), _ptr(U), _ptr(f0), _ptr(f1), float(t_prev), float(dt),
                                             float(theta), float(s), _ptr(alpha_in), _ptr(alpha_out), _ptr(gmin),
                                             _ptr(margin), _ptr(ties), ctypes.byref(nch) if read_back else None,
                                             ctypes.byref(tau) if read_back else None))
        return (int(nch.value), float(tau.value)) if read_back else (None, None)

    def apply(self, alpha, x, y, dt, theta, s=1.0):
        self._sync_stream()
        _check(_lib.hjb_apply(self._h, _ptr(alpha), _ptr(x), _ptr(y), float(dt), float(theta), float(s)))

    def linsolve(self, alpha, U, f0, f1, t_prev, dt, theta, s, X) -> StepStats:
        self._sync_stream()
        st = StepStats()
        _check(_lib.hjb_linsolve(self._h, _ptr(alpha), _ptr(U), _ptr(f0), _ptr(f1), float(t_prev), float(dt),
                                 float(theta), float(s), _ptr(X), ctypes.byref(st)))
        return st

    def step(self, Uprev, Unext, f0, f1, t_prev, dt, theta, s, alpha_io, Uprev2=None, dt_prev=0.0) -> StepStats:
        """hjb_step; Uprev2/dt_prev (optional) start policy iteration from the time extrapolation."""
        self._sync_stream()
        st = StepStats()
        _check(_lib.hjb_step(self._h, _ptr(Uprev), _ptr(Unext), _ptr(f0), _ptr(f1), float(t_prev), float(dt),
                             float(theta), float(s), _ptr(alpha_io), _ptr(Uprev2), float(dt_prev),
                             ctypes.byref(st)))
        return st

    def apply_transposed(self, alpha, x, y, dt, theta, s=1.0):
        self._sync_stream()
        _check(_lib.hjb_apply_transposed(self._h, _ptr(alpha), _ptr(x), _ptr(y), float(dt), float(theta), float(s)))

    def adjoint(self, g, psi, f0, f1, dts, thetas, s, policies, dJ_dUN, dJ_df0, dJ_dg, dJ_df1=None,
                want_ds=True, values=None):
        """hjb_adjoint at fixed policies; values: the forward values [n_steps+1][N] (None: recompute).
        Returns (dJ/ds or None, AdjointStats)."""
        self._sync_stream()
        dts = np.ascontiguousarray(dts, dtype=np.float64)
        thetas = np.ascontiguousarray(thetas, dtype=np.float64)
        st = AdjointStats()
        ds = ctypes.c_double(0.0)
        _check(_lib.hjb_adjoint(self._h, _ptr(g), _ptr(psi), _ptr(f0), _ptr(f1), int(len(dts)), dts.ctypes.data,
                                thetas.ctypes.data, float(s), _ptr(policies), _ptr(values), _ptr(dJ_dUN),
                                _ptr(dJ_df0),
                                _ptr(dJ_df1), _ptr(dJ_dg), ctypes.byref(ds) if want_ds else None,
                                ctypes.byref(st)))
        return (float(ds.value) if want_ds else None), st

    def coarse_operator(self, level: int):
        """hjb_coarse_operator: the Galerkin operator of one level as (cols, vals) device tensors of shape
        (width, nodes) (slot-major sliced ELL, column -1 for unused slots)."""
        import torch
        self._sync_stream()
        w, n = ctypes.c_int32(0), ctypes.c_int64(0)
        _check(_lib.hjb_coarse_operator(self._h, int(level), ctypes.byref(w), ctypes.byref(n), None, None))
        cols = torch.empty((w.value, n.value), dtype=torch.int32, device="cuda")
        vals = torch.empty((w.value, n.value), dtype=torch.float64, device="cuda")
        _check(_lib.hjb_coarse_operator(self._h, int(level), None, None, _ptr(cols), _ptr(vals)))
        return cols, vals

    def amg_level(self, level: int):
        """hjb_amg_level: one level of the aggregation hierarchy of the last solve as a dict with 'levels',
        'rows', 'width', 'agg' (level >= 1: int32 map from the finer level's rows, -1 outside every aggregate)
        and 'cols' / 'vals' (device tensors of shape (width, rows), slot-major sliced ELL, column -1 unused)."""
        import torch
        self._sync_stream()
        nl, n, w = ctypes.c_int32(0), ctypes.c_int64(0), ctypes.c_int32(0)
        _check(_lib.hjb_amg_level(self._h, int(level), ctypes.byref(nl), ctypes.byref(n), ctypes.byref(w),
                                  None, None, None))
        agg = None
        if level >= 1:
            nf = ctypes.c_int64(0)
            _check(_lib.hjb_amg_level(self._h, int(level) - 1, None, ctypes.byref(nf), None, None, None, None))
            agg = torch.empty(nf.value, dtype=torch.int32, device="cuda")
        cols = torch.empty((w.value, n.value), dtype=torch.int32, device="cuda")
        vals = torch.empty((w.value, n.value), dtype=torch.float64, device="cuda")
        _check(_lib.hjb_amg_level(self._h, int(level), None, None, None, _ptr(agg) if agg is not None else None,
                                  _ptr(cols), _ptr(vals)))
        return {"levels": nl.value, "rows": n.value, "width": w.value, "agg": agg, "cols": cols, "vals": vals}

    def set_tile_width(self, width: int):
        self._sync_stream()
        _check(_lib.hjb_set_tile_width(self._h, int(width)))

    def autotune(self, cache_path: Optional[str] = None):
        """hjb_autotune; returns (tile width, {width: weighted cost in ms} or None on a cache hit)."""
        self._sync_stream()
        w = ctypes.c_int32(0)
        costs = (ctypes.c_double * 4)(*([float("nan")] * 4))
        _check(_lib.hjb_autotune(self._h, None if cache_path is None else os.fsencode(cache_path), ctypes.byref(w),
                                 costs))
        c = {16 << q: float(costs[q]) for q in range(4)}
        return int(w.value), (None if all(v != v for v in c.values()) else c)

    def profile_enable(self, kernel: int, max_launches: int = 4096):
        self._sync_stream()
        _check(_lib.hjb_profile_enable(self._h, int(kernel), int(max_launches)))

    def profile_sample(self, period: int):
        """Time one V-cycle (and one launch of each other class) in `period`; 1 times every launch."""
        _check(_lib.hjb_profile_sample(self._h, int(period)))

    def profile_read(self, kernel: int):
        """(launches, total_ms, algorithmic_bytes, algorithmic_flops) recorded since profile_enable."""
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        by = ctypes.c_double(0.0)
        fl = ctypes.c_double(0.0)
        _check(_lib.hjb_profile_read(self._h, int(kernel), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by),
                                     ctypes.byref(fl)))
        return int(n.value), float(ms.value), float(by.value), float(fl.value)

    def solve(self, g, psi, f0, f1, dts, thetas, s, U_final, policies=None, values=None, psi1=None) -> SolveStats:
        """hjb_solve; psi1 (optional): Dirichlet data psi(t) = psi + t psi1."""
        self._sync_stream()
        dts = np.ascontiguousarray(dts, dtype=np.float64)
        thetas = np.ascontiguousarray(thetas, dtype=np.float64)
        st = SolveStats()
        _check(_lib.hjb_solve(self._h, _ptr(g), _ptr(psi), _ptr(psi1), _ptr(f0), _ptr(f1), int(len(dts)),
                              dts.ctypes.data, thetas.ctypes.data, float(s), _ptr(U_final), _ptr(policies),
                              _ptr(values), ctypes.byref(st)))
        return st


class Batch:
    """hjb_setup_batch / hjb_solve_batch: many independent instances (uneven grids and coefficients)
    advanced together; arrays are the instances' arrays concatenated (see offsets)."""

    def __init__(self, instances, options: Optional[Options] = None):
        self.options = options or Options()
        self.instances = list(instances)
        B = len(self.instances)
        descs = (Desc * B)()
        self._keep = []
        for b, inst in enumerate(self.instances):
            field = inst.sigma is None
            sig = np.ascontiguousarray(inst.sigma_node if field else inst.sigma, dtype=np.float64)
            dr = None if inst.drift is None else np.ascontiguousarray(inst.drift, dtype=np.float64)
            cc = None if inst.c is None else np.ascontiguousarray(inst.c, dtype=np.float64)
            self._keep += [sig, dr, cc]
            d = descs[b]
            _lib.hjb_desc_default(ctypes.byref(d))
            d.dim = inst.dim
            for a in range(3):
                d.n[a] = int(inst.n[a]) if a < inst.dim else 1
                d.lo[a] = float(inst.lo[a]) if a < inst.dim else 0.0
            d.h = float(inst.h)
            d.K, d.P = int(inst.K), sig.shape[1]
            d.coef_model = COEF_FIELD if field else (
                COEF_XSCALED if getattr(inst, "coef_model", "const") == "xscaled" else COEF_CONST)
            d.f_per_control = 1 if np.ndim(inst.f0) == 2 else 0
            d.sigma = sig.ctypes.data
            d.drift = None if dr is None else dr.ctypes.data
            d.c = None if cc is None else cc.ctypes.data
            Solver._fill_options(d, self.options)
            d.stream = _setup_stream()
        h = ctypes.c_void_p()
        _check(_lib.hjb_setup_batch(descs, B, ctypes.byref(h)))
        self._h = h
        offs = (ctypes.c_int64 * B)()
        tot = ctypes.c_int64(0)
        _check(_lib.hjb_batch_layout(self._h, offs, ctypes.byref(tot)))
        self.offsets = [int(v) for v in offs]
        self.total = int(tot.value)

    def set_tile_widths(self, widths):
        """hjb_batch_set_tile_widths: one tile width (16, 32, 64, 128) per instance."""
        w = (ctypes.c_int32 * len(self.instances))(*[int(v) for v in widths])
        _check(_lib.hjb_batch_set_tile_widths(self._h, w))

    def autotune(self, cache_path: Optional[str] = None):
        """hjb_batch_autotune: per-instance tile widths from the timing autotuner (one run per distinct
        instance key, results cached in cache_path); returns the widths."""
        w = (ctypes.c_int32 * len(self.instances))()
        _check(_lib.hjb_batch_autotune(self._h, cache_path.encode() if cache_path else None, w))
        return [int(v) for v in w]

    def close(self):
        if getattr(self, "_h", None):
            _lib.hjb_destroy_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def concat(self, field: str):
        """Host FP64 array of the named instance field in the batch layout."""
        out = np.empty(self.total)
        for inst, o in zip(self.instances, self.offsets):
            out[o:o + inst.N] = getattr(inst, field)
        return out

    def split(self, a):
        """Per-instance views of a batch-layout array (numpy or tensor)."""
        return [a[o:o + inst.N] for inst, o in zip(self.instances, self.offsets)]

    def solve(self, g, psi, f0, f1, dts, thetas, s, U_final, policies=None):
        """hjb_solve_batch; returns per-instance SolveStats."""
        _check(_lib.hjb_batch_set_stream(self._h, _stream()))
        dts = np.ascontiguousarray(dts, dtype=np.float64)
        thetas = np.ascontiguousarray(thetas, dtype=np.float64)
        st = (SolveStats * len(self.instances))()
        _check(_lib.hjb_solve_batch(self._h, _ptr(g), _ptr(psi), _ptr(f0), _ptr(f1), int(len(dts)),
                                    dts.ctypes.data, thetas.ctypes.data, float(s), _ptr(U_final), _ptr(policies), st))
        return list(st)


def _autograd_function():
    import torch

    class HJBMarch(torch.autograd.Function):
        """U^N = march(g, f0, f1, s) as a differentiable function; the backward pass is the discrete
        adjoint at the forward policies (hjb_adjoint)."""

        @staticmethod
        def forward(ctx, g, f0, f1, s, solver, psi, dts, thetas, store_values):
            N, n = g.numel(), len(dts)
            U = torch.empty_like(g)
            pol = torch.empty((n, N), dtype=torch.int16, device=g.device)
            stride = 1
            if store_values == "checkpoints":
                stride = max(1, math.ceil(math.sqrt(n)))
            vals = None
            if store_values:
                vals = torch.empty((n // stride + 1, N), dtype=torch.float64, device=g.device)
            with _value_stride(solver, stride):
                solver.solve(g, psi, f0, f1, dts, thetas, float(s), U, pol, vals)
            saved = (g, f0, f1, psi, pol) + ((vals,) if vals is not None else ())
            ctx.save_for_backward(*saved)
            ctx.meta = (solver, float(s), np.asarray(dts, np.float64), np.asarray(thetas, np.float64), stride)
            return U

        @staticmethod
        def backward(ctx, gU):
            g, f0, f1, psi, pol = ctx.saved_tensors[:5]
            vals = ctx.saved_tensors[5] if len(ctx.saved_tensors) > 5 else None
            solver, s, dts, thetas, stride = ctx.meta
            df0, df1, dg = torch.empty_like(g), torch.empty_like(g), torch.empty_like(g)
            with _value_stride(solver, stride):
                ds, _ = solver.adjoint(g, psi, f0, f1, dts, thetas, s, pol, gU.contiguous(), df0, dg, dJ_df1=df1,
                                       values=vals)
            dsv = torch.tensor(ds, dtype=torch.float64, device=g.device)
            return dg, df0, df1, dsv, None, None, None, None, None

    return HJBMarch


class _value_stride:
    """Context: the solver's value_stride option set to `stride` (restored on exit)."""

    def __init__(self, solver, stride):
        self.solver, self.stride = solver, int(stride)

    def __enter__(self):
        self.saved = self.solver.options
        if self.saved.value_stride != self.stride:
            self.solver.set_options(dataclasses.replace(self.saved, value_stride=self.stride))

    def __exit__(self, *exc):
        if self.solver.options is not self.saved:
            self.solver.set_options(self.saved)
        return False


def hjb_march(solver: Solver, g, psi, f0, f1, dts, thetas, s, store_values="checkpoints"):
    """Differentiable march: returns U^N; gradients flow to g, f0, f1 and s (a 0-d FP64 tensor or float).

    The forward pass keeps the int16 policies of every step.  store_values="checkpoints" (default) also keeps
    every ceil(sqrt(n_steps))-th FP64 level, from which the backward pass recomputes the values it needs one
    segment at a time (n_steps fixed-policy solves); False keeps no values (the adjoint first recomputes the
    checkpoints, 2 n_steps solves); True keeps every level (n_steps + 1 full-grid arrays, no recomputation)."""
    import torch
    F = _autograd_function()
    if not torch.is_tensor(s):
        s = torch.tensor(float(s), dtype=torch.float64, device=g.device)
    if store_values not in (True, False, "checkpoints"):
        raise ValueError("store_values: True, False or 'checkpoints'")
    return F.apply(g, f0, f1, s, solver, psi, dts, thetas, store_values)
