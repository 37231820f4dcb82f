"""Python binding of librttda.so (ctypes): argument marshalling only.

Every step of the computation runs in the library's HIP kernels; this module
only checks shapes and dtypes, hands device pointers of torch tensors to the C
ABI (include/rttda.h) and keeps the tensors alive.  It fails loudly if the
shared library has not been built.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# RTTDA_LIB selects another build of the same library (the host-sanitizer build of the CPU tests)
LIB_PATH = os.environ.get("RTTDA_LIB") or os.path.join(HERE, "librttda.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_STATE, E_UNSTABLE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
F64, F32, BF16 = 0, 1, 2
PREC_FP32, PREC_MIXED_BF16 = 1, 2
PULSE_NONE, PULSE_DELTA, PULSE_CW, PULSE_GAUSS, PULSE_CHIRP, PULSE_DELTA_EXACT = 0, 1, 2, 3, 4, 5

_lib = None


class RttdaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rttda status {status}: {msg}")
        self.status = status


class CPulse(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("e0", ctypes.c_double),
                ("omega", ctypes.c_double), ("t0", ctypes.c_double), ("fwhm", ctypes.c_double),
                ("beta", ctypes.c_double), ("phase", ctypes.c_double), ("dir", ctypes.c_double * 3)]


class CDesc(ctypes.Structure):
    _fields_ = [("n_occ", ctypes.c_int32), ("n_virt", ctypes.c_int32), ("n_aux", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("b_dtype", ctypes.c_int32), ("max_rhs", ctypes.c_int32),
                ("cx", ctypes.c_double), ("e_occ", ctypes.c_void_p), ("e_virt", ctypes.c_void_p),
                ("b_ov", ctypes.c_void_p), ("b_oo", ctypes.c_void_p), ("b_vv", ctypes.c_void_p),
                ("mu", ctypes.c_void_p), ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("stream", ctypes.c_void_p)]


class CTuning(ctypes.Structure):
    _fields_ = [("exchange_variant", ctypes.c_int32), ("exchange_splits", ctypes.c_int32),
                ("coulomb_splits", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("steps_per_graph", ctypes.c_int32), ("exchange_chunk", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("small_path", ctypes.c_int32), ("coulomb_path", ctypes.c_int32)]


class CProfile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 4), ("ms", ctypes.c_double * 4)]


PROFILE_CLASSES = ("exchange", "coulomb", "field", "epilogue")

_VP, _I32, _I64, _SZ, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
INTEG_RK4, INTEG_SSO = 0, 1

EXPORTS = {
    "rttda_pool_create": (ctypes.c_int, [_SZ, ctypes.POINTER(_VP)]),
    "rttda_pool_destroy": (ctypes.c_int, [_VP]),
    "rttda_pool_admit": (ctypes.c_int, [_VP, _VP, _I32, ctypes.POINTER(CPulse), _D, _I64, _I32, _VP, _VP, _VP, _SZ,
                                        ctypes.POINTER(_I32)]),
    "rttda_pool_step": (ctypes.c_int, [_VP, _I64, ctypes.POINTER(_I32)]),
    "rttda_pool_poll": (ctypes.c_int, [_VP, _I32, ctypes.POINTER(_I64), ctypes.POINTER(_I32)]),
    "rttda_pool_result": (ctypes.c_int, [_VP, _I32, ctypes.POINTER(_I64)]),
    "rttda_pool_release": (ctypes.c_int, [_VP, _I32]),
    "rttda_pool_usage": (ctypes.c_int, [_VP, ctypes.POINTER(_SZ), ctypes.POINTER(_I32)]),
    "rttda_set_profiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "rttda_get_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CProfile)]),
    "rttda_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(CDesc), ctypes.POINTER(ctypes.c_size_t)]),
    "rttda_create": (ctypes.c_int, [ctypes.POINTER(CDesc), ctypes.POINTER(ctypes.c_void_p)]),
    "rttda_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "rttda_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "rttda_sigma": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p]),
    "rttda_propagate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(CPulse), ctypes.c_double,
                                       ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "rttda_propagate_sso": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(CPulse),
                                           ctypes.c_double, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rttda_set_correlation": (ctypes.c_int, [_VP, _VP]),
    "rttda_set_energy": (ctypes.c_int, [_VP, _VP]),
    "rttda_set_populations": (ctypes.c_int, [_VP, _I32, _VP, _VP]),
    "rttda_spectrum": (ctypes.c_int, [_VP, _I32, _VP, _I32, _I32, _D, _D, _I32, _D, _D, _I32, _VP]),
    "rttda_sigma_noalloc": (ctypes.c_int, [ctypes.POINTER(CDesc), _I32, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double), _VP, _VP, _VP, _VP]),
    "rttda_dipole_trace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rttda_guard": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "rttda_spectral_radius": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double)]),
    "rttda_eigen_workspace_bytes": (ctypes.c_int, [_VP, _I32, _I32, ctypes.POINTER(_SZ)]),
    "rttda_eigen_lowest": (ctypes.c_int, [_VP, _I32, _I32, _I32, _D, _VP, _SZ, ctypes.POINTER(_D), ctypes.POINTER(_D),
                                          _VP, ctypes.POINTER(_I32)]),
    "rttda_populations": (ctypes.c_int, [_VP, _I32, _VP, _I32, _VP, _VP, _SZ, ctypes.POINTER(_D)]),
    "rttda_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CTuning)]),
    "rttda_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CTuning)]),
    "rttda_exchange_splits_max": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_I32)]),
    "rttda_exchange_variants": (ctypes.c_int32, [ctypes.c_int32]),
    "rttda_exchange_variant_name": (ctypes.c_char_p, [ctypes.c_int32, ctypes.c_int32]),
    "rttda_last_error": (ctypes.c_char_p, []),
    "rttda_version": (ctypes.c_char_p, []),
}


def load(path: str = LIB_PATH):
    """Load librttda.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"librttda.so not built at {path}; run `python -m paper_2601_16949_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != OK:
        raise RttdaError(status, load().rttda_last_error().decode())


def _ptr(t) -> int:
    return t.data_ptr()


def _dev_check(t, dtype, shape, name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def make_pulses(pulses) -> ctypes.Array:
    arr = (CPulse * len(pulses))()
    for k, p in enumerate(pulses):
        d = np.asarray(p.direction, dtype=np.float64)
        d = d / np.linalg.norm(d)
        arr[k].kind = int(p.kind)
        arr[k].reserved = 0
        arr[k].e0 = float(p.e0)
        arr[k].omega = float(p.omega)
        arr[k].t0 = float(p.t0)
        arr[k].fwhm = float(p.fwhm)
        arr[k].beta = float(p.beta)
        arr[k].phase = float(p.phase)
        for i in range(3):
            arr[k].dir[i] = float(d[i])
    return arr


class DeviceProblem:
    """Stored inputs of one molecule as device tensors (what the C ABI points at)."""

    @classmethod
    def from_tensors(cls, shape, tensors: dict, precision: str):
        self = cls.__new__(cls)
        self.o, self.v, self.nq = shape.o, shape.v, shape.nq
        self.cx = float(shape.cx)
        self.precision = precision
        for k in ("e_occ", "e_virt", "b_ov", "b_oo", "b_vv", "mu"):
            setattr(self, k, tensors[k])
        return self

    def __init__(self, problem, precision: str = "fp32", device: str = "cuda:0"):
        import torch

        self.o, self.v, self.nq = problem.o, problem.v, problem.nq
        self.cx = float(problem.cx)
        self.precision = precision
        bt = torch.float32 if precision == "fp32" else torch.bfloat16
        if precision == "mixed" and problem.shape.storage != "bf16":
            raise ValueError("mixed precision takes BF16-stored factors")
        self.e_occ = torch.from_numpy(np.ascontiguousarray(problem.e_occ)).to(device)
        self.e_virt = torch.from_numpy(np.ascontiguousarray(problem.e_virt)).to(device)
        self.b_ov = torch.from_numpy(np.ascontiguousarray(problem.b_ov)).to(device).to(bt).contiguous()
        self.b_oo = torch.from_numpy(np.ascontiguousarray(problem.b_oo)).to(device).to(bt).contiguous()
        self.b_vv = torch.from_numpy(np.ascontiguousarray(problem.b_vv)).to(device).to(bt).contiguous()
        self.mu = torch.from_numpy(np.ascontiguousarray(problem.mu)).to(device)

    @property
    def nbytes(self) -> int:
        return sum(t.numel() * t.element_size() for t in (self.e_occ, self.e_virt, self.b_ov, self.b_oo, self.b_vv,
                                                          self.mu))


class Context:
    """One operator on the GPU: rttda_create + workspace, with sigma / propagate / dipole_trace."""

    def __init__(self, dev: DeviceProblem, max_rhs: int, stream=None, sync_streams: bool = True):
        import torch

        lib = load()
        self.sync_streams = sync_streams
        self.lib = lib
        self.dev = dev
        self.max_rhs = int(max_rhs)
        self.o, self.v = dev.o, dev.v
        self.device = dev.e_occ.device
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        prec = PREC_FP32 if dev.precision == "fp32" else PREC_MIXED_BF16
        d = CDesc()
        d.n_occ, d.n_virt, d.n_aux = dev.o, dev.v, dev.nq
        d.precision = prec
        d.b_dtype = F32 if prec == PREC_FP32 else BF16
        d.max_rhs = self.max_rhs
        d.cx = dev.cx
        d.e_occ, d.e_virt, d.mu = _ptr(dev.e_occ), _ptr(dev.e_virt), _ptr(dev.mu)
        if dev.nq > 0:
            d.b_ov, d.b_oo, d.b_vv = _ptr(dev.b_ov), _ptr(dev.b_oo), _ptr(dev.b_vv)
        nbytes = ctypes.c_size_t(0)
        _check(lib.rttda_workspace_bytes(ctypes.byref(d), ctypes.byref(nbytes)))
        self.workspace = torch.empty(max(int(nbytes.value), 256) + 256, dtype=torch.uint8, device=self.device)
        base = _ptr(self.workspace)
        aligned = (base + 255) // 256 * 256
        d.workspace = aligned
        d.workspace_bytes = int(nbytes.value)
        d.stream = self.stream.cuda_stream
        self.desc = d
        h = ctypes.c_void_p()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        _check(lib.rttda_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h

    # -- stream ordering with torch's current stream --------------------------------------------
    def _enter(self):
        import torch

        if self.sync_streams:
            self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        import torch

        if self.sync_streams:
            torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def close(self):
        if getattr(self, "handle", None):
            _check(self.lib.rttda_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points ---------------------------------------------------------------------------
    def sigma(self, field: Sequence[float], dirs, c0, c, s0=None, s=None):
        import torch

        nrhs = c.shape[0]
        _dev_check(c0, torch.float64, (nrhs, 2), "c0")
        _dev_check(c, torch.float64, (nrhs, 2, self.o, self.v), "c")
        s0 = torch.empty_like(c0) if s0 is None else s0
        s = torch.empty_like(c) if s is None else s
        f = (ctypes.c_double * nrhs)(*[float(x) for x in field])
        dd = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(nrhs, 3))
        dd = dd / np.linalg.norm(dd, axis=1, keepdims=True)
        dptr = dd.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self._enter()
        try:
            _check(self.lib.rttda_sigma(self.handle, nrhs, f, dptr, _ptr(c0), _ptr(c), _ptr(s0), _ptr(s)))
        finally:
            self._leave()
        return s0, s

    def propagate(self, pulses, dt: float, n_steps: int, c0, c, step0: int = 0, trace=None, norms=None,
                  want_trace: bool = True, want_norms: bool = False, integrator: str = "rk4", corr=None,
                  pops=None, pop_vectors=None, energy=None):
        """Advance in place with RK4 (rttda_propagate) or the symplectic split operator
        (integrator="sso", rttda_propagate_sso).  corr: a device FP64 tensor [n_steps+1, nrhs, 2]
        that receives the time-correlation function (rttda_set_correlation), or None.  pops: a
        device FP64 tensor [n_steps+1, nrhs, k] that receives the populations of the k unit vectors
        pop_vectors [k, o, v] at every step (rttda_set_populations), or None.  energy: a device FP64
        tensor [n_steps+1, nrhs] that receives <X|diag(0,A)|X> at every step (rttda_set_energy,
        RK4 only), or None."""
        import torch

        if integrator not in ("rk4", "sso"):
            raise ValueError(f"integrator must be 'rk4' or 'sso', not {integrator!r}")
        fn = self.lib.rttda_propagate if integrator == "rk4" else self.lib.rttda_propagate_sso

        nrhs = c.shape[0]
        _dev_check(c0, torch.float64, (nrhs, 2), "c0")
        _dev_check(c, torch.float64, (nrhs, 2, self.o, self.v), "c")
        if want_trace and trace is None:
            trace = torch.empty((n_steps + 1, nrhs), dtype=torch.float64, device=self.device)
        if want_norms and norms is None:
            norms = torch.empty((n_steps + 1, nrhs), dtype=torch.float64, device=self.device)
        cp = make_pulses(pulses)
        if corr is not None:
            _dev_check(corr, torch.float64, (n_steps + 1, nrhs, 2), "corr")
        if pops is not None:
            k = int(pop_vectors.shape[0])
            _dev_check(pop_vectors, torch.float64, (k, self.o, self.v), "pop_vectors")
            _dev_check(pops, torch.float64, (n_steps + 1, nrhs, k), "pops")
        if energy is not None:
            _dev_check(energy, torch.float64, (n_steps + 1, nrhs), "energy")
        self._enter()
        try:
            try:
                if corr is not None:
                    _check(self.lib.rttda_set_correlation(self.handle, _ptr(corr)))
                if pops is not None:
                    _check(self.lib.rttda_set_populations(self.handle, k, _ptr(pop_vectors), _ptr(pops)))
                if energy is not None:
                    _check(self.lib.rttda_set_energy(self.handle, _ptr(energy)))
            except RttdaError:
                # the outputs apply to the next propagate call: none may stay pending for a later one
                self.lib.rttda_set_correlation(self.handle, None)
                self.lib.rttda_set_populations(self.handle, 0, None, None)
                self.lib.rttda_set_energy(self.handle, None)
                raise
            _check(fn(self.handle, nrhs, cp, float(dt), int(step0), int(n_steps), _ptr(c0), _ptr(c),
                      _ptr(trace) if trace is not None else None, _ptr(norms) if norms is not None else None))
        finally:
            self._leave()
        if want_norms:
            return trace, norms
        return trace

    def spectral_radius(self, n_iter: int = 30):
        """(rho, rho_bound) of A from n_iter Lanczos steps on the device (rttda_spectral_radius)."""
        rho, bound = ctypes.c_double(), ctypes.c_double()
        self._enter()
        try:
            _check(self.lib.rttda_spectral_radius(self.handle, int(n_iter), ctypes.byref(rho), ctypes.byref(bound)))
        finally:
            self._leave()
        return rho.value, bound.value

    def eigen_lowest(self, k: int, m_max: int = 0, max_iter: int = 200, tol: float = 1e-5, want_vectors: bool = True):
        """The k lowest eigenpairs of A by block Davidson on the device (rttda_eigen_lowest):
        (evals [k] numpy, residual norms [k] numpy, Ritz vectors torch [k, o, v] FP64 or None,
        iterations).  m_max defaults to min(64, max(4k, 16), o*v)."""
        import torch

        k = int(k)
        if not m_max:
            m_max = min(64, max(4 * k, 16), self.o * self.v)
        nbytes = ctypes.c_size_t()
        _check(self.lib.rttda_eigen_workspace_bytes(self.handle, k, int(m_max), ctypes.byref(nbytes)))
        work = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        base = (work.data_ptr() + 255) // 256 * 256
        evecs = torch.empty((k, self.o, self.v), dtype=torch.float64, device=self.device) if want_vectors else None
        ev = (ctypes.c_double * k)()
        rs = (ctypes.c_double * k)()
        its = ctypes.c_int32()
        self._enter()
        try:
            _check(self.lib.rttda_eigen_lowest(self.handle, k, int(m_max), int(max_iter), float(tol), base,
                                               int(nbytes.value), ev, rs, _ptr(evecs) if evecs is not None else None,
                                               ctypes.byref(its)))
        finally:
            self._leave()
        return np.array(ev[:]), np.array(rs[:]), evecs, int(its.value)

    def populations(self, evecs, c):
        """|<U_I, c_r>|^2 for unit vectors evecs [k, o, v] and states c [nrhs, 2, o, v] (device,
        FP64): numpy [nrhs, k] (rttda_populations)."""
        import torch

        k, nrhs = int(evecs.shape[0]), int(c.shape[0])
        _dev_check(evecs, torch.float64, (k, self.o, self.v), "evecs")
        _dev_check(c, torch.float64, (nrhs, 2, self.o, self.v), "c")
        work = torch.empty(k * 2 * nrhs, dtype=torch.float64, device=self.device)
        out = (ctypes.c_double * (k * nrhs))()
        self._enter()
        try:
            _check(self.lib.rttda_populations(self.handle, k, _ptr(evecs), nrhs, _ptr(c), _ptr(work),
                                              work.numel() * 8, out))
        finally:
            self._leave()
        return np.array(out[:]).reshape(nrhs, k)

    def dipole_trace(self, dirs, c0, c, out=None):
        import torch

        nrhs = c.shape[0]
        _dev_check(c0, torch.float64, (nrhs, 2), "c0")
        _dev_check(c, torch.float64, (nrhs, 2, self.o, self.v), "c")
        out = torch.empty(nrhs, dtype=torch.float64, device=self.device) if out is None else out
        dd = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(nrhs, 3))
        dd = dd / np.linalg.norm(dd, axis=1, keepdims=True)
        self._enter()
        try:
            _check(self.lib.rttda_dipole_trace(self.handle, nrhs, dd.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                               _ptr(c0), _ptr(c), _ptr(out)))
        finally:
            self._leave()
        return out

    def guard(self) -> int:
        bad = ctypes.c_int64(0)
        st = self.lib.rttda_guard(self.handle, ctypes.byref(bad))
        if st not in (OK, E_UNSTABLE):
            _check(st)
        return int(bad.value)

    def set_tuning(self, exchange_variant=0, exchange_splits=0, coulomb_splits=0, use_graph=0, steps_per_graph=0,
                   exchange_chunk=0, overlap=0, small_path=0, coulomb_path=0):
        t = CTuning(exchange_variant, exchange_splits, coulomb_splits, use_graph, steps_per_graph, exchange_chunk,
                    overlap, small_path, coulomb_path)
        _check(self.lib.rttda_set_tuning(self.handle, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        t = CTuning()
        _check(self.lib.rttda_get_tuning(self.handle, ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in CTuning._fields_}

    def max_splits(self) -> int:
        """Largest exchange split count the workspace holds."""
        n = _I32()
        _check(self.lib.rttda_exchange_splits_max(self.handle, ctypes.byref(n)))
        return max(1, int(n.value))

    def use_tuned(self, nrhs: int, integrator: str = "rk4") -> bool:
        """Apply the packaged autotune choice for (shape, nrhs, integrator) if there is one."""
        from . import autotune

        if self.get_tuning()["small_path"] == 1:
            return False  # the small-problem path has no exchange tile to choose
        e = autotune.lookup(self, nrhs, integrator=integrator)
        return bool(e) and autotune.apply(self, e)

    def set_profiling(self, on: bool):
        _check(self.lib.rttda_set_profiling(self.handle, 1 if on else 0))

    def get_profile(self) -> dict:
        p = CProfile()
        _check(self.lib.rttda_get_profile(self.handle, ctypes.byref(p)))
        return {name: {"launches": int(p.launches[k]), "ms": float(p.ms[k])} for k, name in enumerate(PROFILE_CLASSES)}

    def variant_name(self, k: int) -> str:
        return self.lib.rttda_exchange_variant_name(self.desc.precision, k).decode()


def sigma_noalloc(dev: DeviceProblem, field: Sequence[float], dirs, c0, c, s0=None, s=None, stream=None):
    """rttda_sigma_noalloc: s = H X for the operator dev without a context or workspace (the
    library's static device scratch).  Returns (s0, s); s0 and s may be passed preallocated."""
    import torch

    lib = load()
    nrhs = c.shape[0]
    _dev_check(c0, torch.float64, (nrhs, 2), "c0")
    _dev_check(c, torch.float64, (nrhs, 2, dev.o, dev.v), "c")
    s0 = torch.empty_like(c0) if s0 is None else s0
    s = torch.empty_like(c) if s is None else s
    d = CDesc()
    d.n_occ, d.n_virt, d.n_aux = dev.o, dev.v, dev.nq
    d.precision = PREC_FP32 if dev.precision == "fp32" else PREC_MIXED_BF16
    d.b_dtype = F32 if d.precision == PREC_FP32 else BF16
    d.max_rhs = nrhs
    d.cx = dev.cx
    d.e_occ, d.e_virt, d.mu = _ptr(dev.e_occ), _ptr(dev.e_virt), _ptr(dev.mu)
    if dev.nq > 0:
        d.b_ov, d.b_oo, d.b_vv = _ptr(dev.b_ov), _ptr(dev.b_oo), _ptr(dev.b_vv)
    st = stream if stream is not None else torch.cuda.current_stream(c.device)
    d.stream = st.cuda_stream
    f = (ctypes.c_double * nrhs)(*[float(x) for x in field])
    dd = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(nrhs, 3))
    dd = dd / np.linalg.norm(dd, axis=1, keepdims=True)
    _check(lib.rttda_sigma_noalloc(ctypes.byref(d), nrhs, f, dd.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   _ptr(c0), _ptr(c), _ptr(s0), _ptr(s)))
    return s0, s


def workspace_bytes(o: int, v: int, nq: int, precision: str, max_rhs: int) -> int:
    """Workspace a context of this shape needs (host-side query, no device work)."""
    d = CDesc()
    d.n_occ, d.n_virt, d.n_aux = o, v, nq
    d.precision = PREC_FP32 if precision == "fp32" else PREC_MIXED_BF16
    d.b_dtype = F32 if precision == "fp32" else BF16
    d.max_rhs = max_rhs
    n = ctypes.c_size_t(0)
    _check(load().rttda_workspace_bytes(ctypes.byref(d), ctypes.byref(n)))
    return int(n.value)


def ground_state(nrhs: int, o: int, v: int, device="cuda:0"):
    """c0 = 1, C = 0 for nrhs states (the Kohn-Sham ground state)."""
    import torch

    c0 = torch.zeros((nrhs, 2), dtype=torch.float64, device=device)
    c0[:, 0] = 1.0
    c = torch.zeros((nrhs, 2, o, v), dtype=torch.float64, device=device)
    return c0, c


def spectrum(signal, dt: float, omega, kappa: float = 1.0, average: bool = False, stream=None):
    """Spectra of device signals on the uniform grid omega (rttda_spectrum): a dipole trace
    [n_t, nsig] (kind 0, divided by kappa) or a time correlation [n_t, nsig, 2] (kind 1).  Returns
    a device tensor [nsig, n_omega], or [n_omega] averaged over the signals."""
    import torch

    lib = load()
    omega = np.asarray(omega, dtype=np.float64).reshape(-1)
    if signal.dim() not in (2, 3) or (signal.dim() == 3 and signal.shape[2] != 2):
        raise ValueError(f"signal must be [n_t, nsig] or [n_t, nsig, 2], got {tuple(signal.shape)}")
    kind = 0 if signal.dim() == 2 else 1
    n_t, nsig = int(signal.shape[0]), int(signal.shape[1])
    _dev_check(signal, torch.float64, tuple(signal.shape), "signal")
    if omega.size == 0:
        raise ValueError("omega must hold at least one frequency")
    dw = float(omega[1] - omega[0]) if omega.size > 1 else 0.0
    if omega.size > 2 and not np.allclose(np.diff(omega), dw, rtol=1e-9, atol=1e-12 * max(1.0, abs(dw))):
        raise ValueError("omega must be a uniform grid")
    out = torch.empty((omega.size,) if average else (nsig, omega.size), dtype=torch.float64, device=signal.device)
    st = stream if stream is not None else torch.cuda.current_stream(signal.device)
    _check(lib.rttda_spectrum(st.cuda_stream, kind, _ptr(signal), n_t, nsig, float(dt), float(kappa), int(omega.size),
                              float(omega[0]), dw, 1 if average else 0, _ptr(out)))
    return out


def to_planes(c0: np.ndarray, c: np.ndarray, device="cuda:0"):
    """complex (nrhs,), (nrhs, o, v) -> device f64 planes (nrhs, 2), (nrhs, 2, o, v)."""
    import torch

    c0p = np.stack([c0.real, c0.imag], axis=-1)
    cp = np.stack([c.real, c.imag], axis=1)
    return (torch.from_numpy(np.ascontiguousarray(c0p)).to(device),
            torch.from_numpy(np.ascontiguousarray(cp)).to(device))


def from_planes(c0p, cp):
    a = c0p.detach().cpu().numpy()
    b = cp.detach().cpu().numpy()
    return a[:, 0] + 1j * a[:, 1], b[:, 0] + 1j * b[:, 1]


class Pool:
    """The library's serving pool (rttda_pool_*): admission by HBM footprint against a budget,
    chunked stepping of every admitted request on its own context's stream, polling, release."""

    def __init__(self, budget_bytes: int):
        self.lib = load()
        h = ctypes.c_void_p()
        _check(self.lib.rttda_pool_create(int(budget_bytes), ctypes.byref(h)))
        self.handle = h
        self._keep = {}  # slot -> objects that must outlive it (pulse array, tensors)

    def admit(self, ctx: "Context", pulses, dt: float, n_steps: int, c0, c, trace=None, footprint: int = 0,
              integrator: str = "rk4") -> int:
        """Slot id; raises RttdaError(E_NOMEM) when the footprint does not fit."""
        import torch

        nrhs = c.shape[0]
        _dev_check(c0, torch.float64, (nrhs, 2), "c0")
        _dev_check(c, torch.float64, (nrhs, 2, ctx.o, ctx.v), "c")
        if trace is not None:
            _dev_check(trace, torch.float64, (n_steps + 1, nrhs), "trace")
        cp = make_pulses(pulses)
        slot = ctypes.c_int32()
        ctx._enter()  # the request's chunks run on the context's stream, after work queued so far
        _check(self.lib.rttda_pool_admit(self.handle, ctx.handle, nrhs, cp, float(dt), int(n_steps),
                                         INTEG_RK4 if integrator == "rk4" else INTEG_SSO, _ptr(c0), _ptr(c),
                                         _ptr(trace) if trace is not None else None, int(footprint),
                                         ctypes.byref(slot)))
        self._keep[slot.value] = (cp, ctx, c0, c, trace)
        return slot.value

    def step(self, chunk_steps: int) -> int:
        """Enqueue the next chunk of every request whose previous chunk finished; returns the count."""
        n = ctypes.c_int32()
        _check(self.lib.rttda_pool_step(self.handle, int(chunk_steps), ctypes.byref(n)))
        return n.value

    def poll(self, slot: int):
        """(steps enqueued, finished) of a slot, without blocking."""
        done, fin = ctypes.c_int64(), ctypes.c_int32()
        _check(self.lib.rttda_pool_poll(self.handle, int(slot), ctypes.byref(done), ctypes.byref(fin)))
        return done.value, bool(fin.value)

    def result(self, slot: int) -> int:
        """Wait for a slot and return the first step at which its norm guard tripped (-1 if
        never); raises RttdaError with the slot's status if one of its chunks failed."""
        bad = ctypes.c_int64(-1)
        st = self.lib.rttda_pool_result(self.handle, int(slot), ctypes.byref(bad))
        if st not in (OK, E_UNSTABLE):
            _check(st)
        return int(bad.value)

    def release(self, slot: int):
        _check(self.lib.rttda_pool_release(self.handle, int(slot)))
        self._keep.pop(slot, None)

    def usage(self):
        used, active = ctypes.c_size_t(), ctypes.c_int32()
        _check(self.lib.rttda_pool_usage(self.handle, ctypes.byref(used), ctypes.byref(active)))
        return used.value, active.value

    def close(self):
        if self.handle:
            self.lib.rttda_pool_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
