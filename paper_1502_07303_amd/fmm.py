"""Python binding of ``libfmm.so`` (argument marshalling only).

Every step of the solve runs in the HIP library; torch provides device memory
and the current stream.  The library must have been built (``build.py``);
importing this module without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# FMM_LIB selects another build of the same sources (the sanitizer test
# runs the host-side ABI checks against a build whose host code carries
# AddressSanitizer this way)
LIB_PATH = os.environ.get("FMM_LIB") or os.path.join(_HERE, "libfmm.so")

FMM_OK, FMM_EINVAL, FMM_ENOMEM, FMM_EHIP, FMM_ENOCONV, FMM_EDEVICE = 0, -1, -2, -3, -4, -5
FMM_F32, FMM_F64 = 0, 1
FMM_VALIDATE = 1
FMM_TIMING = 2
FMM_ONE_MARCH = 4

DERR = {1: "seed index out of range", 2: "duplicate seed", 4: "non-finite seed value",
        8: "non-finite speed", 16: "restart limit", 32: "barrier timeout", 64: "round cap",
        128: "launch", 256: "time limit"}

ST_FAR, ST_BAND, ST_ACCEPTED, ST_SEED, ST_NEG = 0, 1, 2, 3, 0x80


class FmmOpts(ctypes.Structure):
    _fields_ = [("band_width", ctypes.c_double), ("stride", ctypes.c_double),
                ("inner_stride", ctypes.c_double), ("tile_edge", ctypes.c_int32), ("max_restarts", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("time_limit_s", ctypes.c_uint32), ("stride_h", ctypes.c_double),
                ("axis_scale", ctypes.c_double * 3)]


class FmmStats(ctypes.Structure):
    _fields_ = [("n_accepted", ctypes.c_int64), ("n_restarts", ctypes.c_int64),
                ("n_reopened", ctypes.c_int64), ("n_tile_marches", ctypes.c_int64),
                ("n_solves", ctypes.c_int64), ("n_rounds", ctypes.c_int64),
                ("max_abs_T", ctypes.c_double), ("device_error", ctypes.c_uint32),
                ("tile_edge", ctypes.c_uint32), ("n_workgroups", ctypes.c_int64),
                ("ms_prepare", ctypes.c_double), ("ms_driver", ctypes.c_double),
                ("ms_finalize", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FmmProblem(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_int64), ("n1", ctypes.c_int64), ("n2", ctypes.c_int64), ("h", ctypes.c_double),
                ("F", ctypes.c_void_p), ("seed_idx", ctypes.c_void_p), ("seed_val", ctypes.c_void_p),
                ("n_seeds", ctypes.c_int64), ("T_out", ctypes.c_void_p), ("status_out", ctypes.c_void_p)]


class FmmAdjointProblem(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_int64), ("n1", ctypes.c_int64), ("n2", ctypes.c_int64), ("h", ctypes.c_double),
                ("F", ctypes.c_void_p), ("T", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("dL_dT", ctypes.c_void_p), ("dL_dF", ctypes.c_void_p), ("axis_scale", ctypes.c_double * 3)]


class FmmAdjointStats(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("n_levels", ctypes.c_int64), ("device_error", ctypes.c_uint32),
                ("pad", ctypes.c_uint32)]


class FmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfmm.so and declare its C signatures; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_1502_07303_amd/build.py (or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
    lib.fmm_default_opts.argtypes = [ctypes.POINTER(FmmOpts)]
    lib.fmm_default_opts.restype = None
    lib.fmm_workspace_bytes.argtypes = [i64, i64, i64, i64, ctypes.c_int, ctypes.POINTER(FmmOpts)]
    lib.fmm_workspace_bytes.restype = ctypes.c_size_t
    lib.fmm_solve.argtypes = [i64, i64, i64, dbl, P, ctypes.c_int, P, P, i64, ctypes.POINTER(FmmOpts),
                              P, P, P, ctypes.c_size_t, P]
    lib.fmm_solve.restype = ctypes.c_int
    lib.fmm_get_stats.argtypes = [P, ctypes.POINTER(FmmStats), P]
    lib.fmm_get_stats.restype = ctypes.c_int
    lib.fmm_solve_noalloc.argtypes = [i64, i64, i64, dbl, P, ctypes.c_int, P, P, i64, ctypes.POINTER(FmmOpts),
                                      P, P, P, P]
    lib.fmm_solve_noalloc.restype = ctypes.c_int
    lib.fmm_eval_godunov.argtypes = [P, P, P, i64, P]
    lib.fmm_eval_godunov.restype = ctypes.c_int
    PP = ctypes.POINTER(FmmProblem)
    lib.fmm_batch_workspace_bytes.argtypes = [i64, PP, ctypes.c_int, ctypes.POINTER(FmmOpts)]
    lib.fmm_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.fmm_solve_batch.argtypes = [i64, PP, ctypes.c_int, ctypes.POINTER(FmmOpts), P, ctypes.c_size_t, P]
    lib.fmm_solve_batch.restype = ctypes.c_int
    lib.fmm_get_batch_stats.argtypes = [P, i64, ctypes.POINTER(FmmStats), P]
    lib.fmm_get_batch_stats.restype = ctypes.c_int
    lib.fmm_tune_batch.argtypes = [i64, PP, ctypes.c_int, ctypes.POINTER(FmmOpts), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int32, P,
                                   ctypes.c_size_t, P, ctypes.POINTER(FmmOpts), ctypes.POINTER(ctypes.c_float)]
    lib.fmm_tune_batch.restype = ctypes.c_int
    PA = ctypes.POINTER(FmmAdjointProblem)
    lib.fmm_adjoint_workspace_bytes.argtypes = [i64, PA]
    lib.fmm_adjoint_workspace_bytes.restype = ctypes.c_size_t
    lib.fmm_adjoint_batch.argtypes = [i64, PA, ctypes.c_int, P, ctypes.c_size_t, P]
    lib.fmm_adjoint_batch.restype = ctypes.c_int
    lib.fmm_adjoint.argtypes = [i64, i64, i64, dbl, P, ctypes.c_int, P, P, P, P, P, ctypes.c_size_t, P]
    lib.fmm_adjoint.restype = ctypes.c_int
    lib.fmm_get_adjoint_stats.argtypes = [P, ctypes.POINTER(FmmAdjointStats), P]
    lib.fmm_get_adjoint_stats.restype = ctypes.c_int
    lib.fmm_strerror.argtypes = [ctypes.c_int]
    lib.fmm_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load_library().fmm_strerror(int(code)).decode()


def make_opts(band_width=math.inf, stride=None, tile_edge=0, max_restarts=0, validate=False,
              time_limit_s=0, timing=False, inner_stride=None, one_march=False, stride_h=None,
              axis_scale=None) -> FmmOpts:
    o = FmmOpts()
    load_library().fmm_default_opts(ctypes.byref(o))
    o.band_width = float(band_width)
    o.stride = 0.0 if stride is None else float(stride)
    o.inner_stride = 0.0 if inner_stride is None else float(inner_stride)
    o.tile_edge = int(tile_edge)
    o.max_restarts = int(max_restarts)
    o.flags = (FMM_VALIDATE if validate else 0) | (FMM_TIMING if timing else 0) | (FMM_ONE_MARCH if one_march else 0)
    o.time_limit_s = int(time_limit_s)
    o.stride_h = 0.0 if stride_h is None else float(stride_h)
    if axis_scale is not None:
        for a in range(3):
            o.axis_scale[a] = float(axis_scale[a])
    return o


def workspace_bytes(shape, n_seeds, opts: Optional[FmmOpts] = None, f_dtype=FMM_F64) -> int:
    n0, n1, n2 = shape
    return int(load_library().fmm_workspace_bytes(n0, n1, n2, n_seeds, int(f_dtype),
                                                  ctypes.byref(opts) if opts else None))


def _check_cuda(name: str, t: torch.Tensor, device) -> None:
    """Every tensor handed to the library must live on the solve's GPU: a
    host pointer reaching a kernel would fault instead of failing cleanly."""
    if not t.is_cuda or t.device != device:
        raise FmmError(FMM_EINVAL, f"{name} must be a CUDA tensor on {device} (got {t.device})")


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Solver:
    """Reusable solve context: owns the workspace for one grid shape and the
    option set, so repeated solves allocate nothing."""

    def __init__(self, shape, n_seeds, h, band_width=math.inf, stride=None, tile_edge=0, max_restarts=0,
                 validate=False, device="cuda", time_limit_s=0, timing=False, inner_stride=None,
                 speed_dtype=torch.float64, one_march=False, axis_scale=None):
        self.lib = load_library()
        self.shape = tuple(int(x) for x in shape)
        self.h = float(h)
        self.opts = make_opts(band_width, stride, tile_edge, max_restarts, validate, time_limit_s, timing,
                              inner_stride, one_march, axis_scale=axis_scale)
        if speed_dtype not in (torch.float32, torch.float64):
            raise FmmError(FMM_EINVAL, f"unsupported speed dtype {speed_dtype}")
        self.speed_dtype = speed_dtype
        nbytes = workspace_bytes(self.shape, n_seeds, self.opts,
                                 FMM_F32 if speed_dtype == torch.float32 else FMM_F64)
        if nbytes == 0:
            raise FmmError(FMM_EINVAL, "invalid problem or options")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.workspace.data_ptr()) % 256
        self.ws = self.workspace[off:off + nbytes]
        self.nbytes = nbytes

    def solve_into(self, F: torch.Tensor, seed_idx: torch.Tensor, seed_val: torch.Tensor, T: torch.Tensor,
                   status: Optional[torch.Tensor] = None, stream=None) -> None:
        """Enqueue a solve on the current (or given) stream; no synchronisation."""
        if F.dtype == torch.float32:
            dt = FMM_F32
        elif F.dtype == torch.float64:
            dt = FMM_F64
        else:
            raise FmmError(FMM_EINVAL, f"unsupported speed dtype {F.dtype}")
        if F.dtype != self.speed_dtype:
            raise FmmError(FMM_EINVAL, f"solver was sized for {self.speed_dtype} speeds, got {F.dtype}")
        if tuple(F.shape) != self.shape or not F.is_contiguous() or not F.is_cuda:
            raise FmmError(FMM_EINVAL, "F must be a contiguous CUDA tensor of the solver's shape")
        if seed_idx.dtype != torch.int64 or seed_val.dtype != torch.float64:
            raise FmmError(FMM_EINVAL, "seed_idx must be int64 and seed_val float64")
        if not (seed_idx.is_contiguous() and seed_val.is_contiguous()) or seed_idx.numel() != seed_val.numel():
            raise FmmError(FMM_EINVAL, "seed arrays must be contiguous and of equal length")
        if T.dtype != torch.float64 or tuple(T.shape) != self.shape or not T.is_contiguous():
            raise FmmError(FMM_EINVAL, "T must be a contiguous float64 tensor of the solver's shape")
        if status is not None and (status.dtype != torch.uint8 or tuple(status.shape) != self.shape
                                   or not status.is_contiguous()):
            raise FmmError(FMM_EINVAL, "status must be a contiguous uint8 tensor of the solver's shape")
        ns = seed_idx.numel()
        if ns:
            _check_cuda("seed_idx", seed_idx, F.device)
            _check_cuda("seed_val", seed_val, F.device)
        _check_cuda("T", T, F.device)
        if status is not None:
            _check_cuda("status", status, F.device)
        if self.ws.device != F.device:
            raise FmmError(FMM_EINVAL, f"solver workspace is on {self.ws.device}, F on {F.device}")
        n0, n1, n2 = self.shape
        rc = self.lib.fmm_solve(n0, n1, n2, self.h, _ptr(F), dt, _ptr(seed_idx) if ns else None,
                                _ptr(seed_val) if ns else None, ns, ctypes.byref(self.opts), _ptr(T),
                                _ptr(status), _ptr(self.ws), self.nbytes, _stream_handle(stream))
        if rc != FMM_OK:
            raise FmmError(rc, f"fmm_solve: {strerror(rc)}")

    def stats(self, stream=None, check=True) -> FmmStats:
        """Synchronise the stream and read the statistics of the last solve."""
        st = FmmStats()
        rc = self.lib.fmm_get_stats(_ptr(self.ws), ctypes.byref(st), _stream_handle(stream))
        if check and rc != FMM_OK:
            bits = [m for b, m in DERR.items() if st.device_error & b]
            raise FmmError(rc, f"fmm_solve failed on the device: {strerror(rc)} ({', '.join(bits)})")
        return st


def solve(F: torch.Tensor, h: float, seed_idx: torch.Tensor, seed_val: torch.Tensor, band_width=math.inf,
          stride=None, tile_edge=0, max_restarts=0, validate=False, with_status=True, check=True,
          time_limit_s=0, inner_stride=None, one_march=False, axis_scale=None):
    """One solve on F's device; returns (T, status, stats) after synchronising."""
    s = Solver(F.shape, seed_idx.numel(), h, band_width, stride, tile_edge, max_restarts, validate, F.device,
               time_limit_s, inner_stride=inner_stride, speed_dtype=F.dtype, one_march=one_march,
               axis_scale=axis_scale)
    T = torch.empty(F.shape, dtype=torch.float64, device=F.device)
    status = torch.empty(F.shape, dtype=torch.uint8, device=F.device) if with_status else None
    s.solve_into(F, seed_idx, seed_val, T, status)
    st = s.stats(check=check)
    return T, status, st


NOALLOC_MAX_BYTES = 64 << 20  # FMM_NOALLOC_MAX_BYTES


def solve_noalloc_into(F: torch.Tensor, h: float, seed_idx: torch.Tensor, seed_val: torch.Tensor, T: torch.Tensor,
                       status: Optional[torch.Tensor] = None, error: Optional[torch.Tensor] = None,
                       opts: Optional[FmmOpts] = None, stream=None) -> None:
    """Enqueue fmm_solve_noalloc(): a solve whose workspace is the library's
    fixed per-GPU array (nothing is allocated).  ``error`` (a 1-element uint32
    CUDA tensor, optional) receives the device error bits in stream order.
    Calls that overlap on one GPU race; order them on one stream."""
    dev = F.device
    _check_cuda("F", F, dev)
    dt = _dtype_code(F.dtype)
    shape = tuple(F.shape)
    if F.dim() != 3 or not F.is_contiguous():
        raise FmmError(FMM_EINVAL, "F must be a contiguous 3-D CUDA tensor")
    if seed_idx.dtype != torch.int64 or seed_val.dtype != torch.float64 or seed_idx.numel() != seed_val.numel():
        raise FmmError(FMM_EINVAL, "seed_idx must be int64 and seed_val float64, of equal length")
    if not (seed_idx.is_contiguous() and seed_val.is_contiguous()):
        raise FmmError(FMM_EINVAL, "seed arrays must be contiguous")
    ns = seed_idx.numel()
    if ns:
        _check_cuda("seed_idx", seed_idx, dev)
        _check_cuda("seed_val", seed_val, dev)
    if T.dtype != torch.float64 or tuple(T.shape) != shape or not T.is_contiguous():
        raise FmmError(FMM_EINVAL, "T must be a contiguous float64 tensor of F's shape")
    _check_cuda("T", T, dev)
    if status is not None:
        if status.dtype != torch.uint8 or tuple(status.shape) != shape or not status.is_contiguous():
            raise FmmError(FMM_EINVAL, "status must be a contiguous uint8 tensor of F's shape")
        _check_cuda("status", status, dev)
    if error is not None:
        if error.dtype not in (torch.int32, torch.uint32) or error.numel() < 1 or not error.is_contiguous():
            raise FmmError(FMM_EINVAL, "error must be a contiguous 32-bit integer tensor")
        _check_cuda("error", error, dev)
    o = opts if opts is not None else make_opts()
    n0, n1, n2 = shape
    rc = load_library().fmm_solve_noalloc(n0, n1, n2, float(h), _ptr(F), dt, _ptr(seed_idx) if ns else None,
                                          _ptr(seed_val) if ns else None, ns, ctypes.byref(o), _ptr(T),
                                          _ptr(status), _ptr(error), _stream_handle(stream))
    if rc != FMM_OK:
        raise FmmError(rc, f"fmm_solve_noalloc: {strerror(rc)}")


def eval_godunov(a: torch.Tensor, r: torch.Tensor) -> torch.Tensor:
    """Device local solver on (n, 3) upwind values and (n,) r = h/F."""
    a = a.contiguous()
    r = r.contiguous()
    out = torch.empty(r.shape, dtype=torch.float64, device=r.device)
    rc = load_library().fmm_eval_godunov(_ptr(a), _ptr(r), _ptr(out), r.numel(), _stream_handle())
    if rc != FMM_OK:
        raise FmmError(rc, f"fmm_eval_godunov: {strerror(rc)}")
    return out


# ---------------------------------------------------------------------------
# Batches


def _dtype_code(dt):
    if dt == torch.float32:
        return FMM_F32
    if dt == torch.float64:
        return FMM_F64
    raise FmmError(FMM_EINVAL, f"unsupported speed dtype {dt}")


class BatchSolver:
    """Many problems in one persistent launch.

    ``problems`` is a list of dicts with keys F (contiguous CUDA tensor, one
    dtype for the batch), h, seed_idx (int64), seed_val (float64); T and
    status outputs are allocated here (``self.T[i]``, ``self.status[i]``).
    The descriptors hold raw device addresses: the tensors must stay alive and
    in place for the solver's lifetime (a solve reads their current values).
    """

    def __init__(self, problems, band_width=math.inf, stride=None, stride_h=None, tile_edge=0, max_restarts=0,
                 validate=False, time_limit_s=0, timing=False, inner_stride=None, one_march=False,
                 with_status=True, workspace_edges=None, T_out=None, status_out=None, axis_scale=None):
        self.lib = load_library()
        if not problems:
            raise FmmError(FMM_EINVAL, "empty batch")
        self.keep = []
        dt = problems[0]["F"].dtype
        self.dtype = _dtype_code(dt)
        dev = problems[0]["F"].device
        n = len(problems)
        arr = (FmmProblem * n)()
        self.T, self.status = [], []
        for i, q in enumerate(problems):
            F, idx, val = q["F"], q["seed_idx"], q["seed_val"]
            if F.dtype != dt or not F.is_cuda or not F.is_contiguous() or F.dim() != 3:
                raise FmmError(FMM_EINVAL, f"problem {i}: F must be a contiguous 3-D CUDA tensor of the batch dtype")
            if idx.dtype != torch.int64 or val.dtype != torch.float64 or idx.numel() != val.numel():
                raise FmmError(FMM_EINVAL, f"problem {i}: seed_idx int64 and seed_val float64 of equal length")
            if not (idx.is_contiguous() and val.is_contiguous()):
                raise FmmError(FMM_EINVAL, f"problem {i}: seed arrays must be contiguous")
            if F.device != dev:
                raise FmmError(FMM_EINVAL, f"problem {i}: F is on {F.device}, the batch on {dev}")
            if idx.numel():
                _check_cuda(f"problem {i}: seed_idx", idx, dev)
                _check_cuda(f"problem {i}: seed_val", val, dev)
            if T_out is not None:
                T = T_out[i]
                if T.dtype != torch.float64 or T.shape != F.shape or not T.is_contiguous():
                    raise FmmError(FMM_EINVAL, f"problem {i}: T_out must be contiguous float64 of F's shape")
            else:
                T = torch.empty(F.shape, dtype=torch.float64, device=dev)
            if status_out is not None:
                st = status_out[i]
                if st.dtype != torch.uint8 or st.shape != F.shape or not st.is_contiguous():
                    raise FmmError(FMM_EINVAL, f"problem {i}: status_out must be contiguous uint8 of F's shape")
            else:
                st = torch.empty(F.shape, dtype=torch.uint8, device=dev) if with_status else None
            _check_cuda(f"problem {i}: T_out", T, dev)
            if st is not None:
                _check_cuda(f"problem {i}: status_out", st, dev)
            self.T.append(T)
            self.status.append(st)
            self.keep += [F, idx, val]
            p = arr[i]
            p.n0, p.n1, p.n2 = (int(x) for x in F.shape)
            p.h = float(q["h"])
            p.F = F.data_ptr()
            p.n_seeds = idx.numel()
            p.seed_idx = idx.data_ptr() if idx.numel() else None
            p.seed_val = val.data_ptr() if idx.numel() else None
            p.T_out = T.data_ptr()
            p.status_out = st.data_ptr() if st is not None else None
        self.n = n
        self.problems = arr
        self.opts = make_opts(band_width, stride, tile_edge, max_restarts, validate, time_limit_s, timing,
                              inner_stride, one_march, stride_h, axis_scale)
        edges = workspace_edges or [self.opts.tile_edge or 8]
        nbytes = 0
        for e in edges:
            o = make_opts(band_width, stride, e, max_restarts, validate, time_limit_s, timing, inner_stride,
                          one_march, stride_h, axis_scale)
            b = int(self.lib.fmm_batch_workspace_bytes(n, arr, self.dtype, ctypes.byref(o)))
            if b == 0:
                raise FmmError(FMM_EINVAL, "invalid batch or options")
            nbytes = max(nbytes, b)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-self.workspace.data_ptr()) % 256
        self.ws = self.workspace[off:off + nbytes]
        self.nbytes = nbytes

    def solve(self, stream=None) -> None:
        """Enqueue the batch solve on the current (or given) stream."""
        rc = self.lib.fmm_solve_batch(self.n, self.problems, self.dtype, ctypes.byref(self.opts), _ptr(self.ws),
                                      self.nbytes, _stream_handle(stream))
        if rc != FMM_OK:
            raise FmmError(rc, f"fmm_solve_batch: {strerror(rc)}")

    def stats(self, stream=None, check=True):
        """Synchronise and return the per-problem statistics."""
        st = (FmmStats * self.n)()
        rc = self.lib.fmm_get_batch_stats(_ptr(self.ws), self.n, st, _stream_handle(stream))
        if check and rc != FMM_OK:
            bits = [m for b, m in DERR.items() if st[0].device_error & b]
            raise FmmError(rc, f"batch solve failed on the device: {strerror(rc)} ({', '.join(bits)})")
        return list(st)

    def tune(self, edges=(4, 8, 16), strides_h=(1.0, 2.0, 4.0, 8.0), reps=1, stream=None):
        """Time every (tile edge, stride) pair with the library's autotuner and
        adopt the fastest.  Returns {(edge, stride_h): ms}."""
        ne, ns = len(edges), len(strides_h)
        e_arr = (ctypes.c_int32 * ne)(*[int(e) for e in edges])
        s_arr = (ctypes.c_double * ns)(*[float(x) for x in strides_h])
        ms = (ctypes.c_float * (ne * ns))()
        best = FmmOpts()
        rc = self.lib.fmm_tune_batch(self.n, self.problems, self.dtype, ctypes.byref(self.opts), e_arr, ne, s_arr,
                                     ns, int(reps), _ptr(self.ws), self.nbytes, _stream_handle(stream),
                                     ctypes.byref(best), ms)
        if rc != FMM_OK:
            raise FmmError(rc, f"fmm_tune_batch: {strerror(rc)}")
        best.flags = self.opts.flags
        self.opts = best
        return {(int(edges[a]), float(strides_h[b])): float(ms[a * ns + b]) for a in range(ne) for b in range(ns)}


# ---------------------------------------------------------------------------
# Adjoint


class AdjointSolver:
    """Reusable adjoint context for a fixed list of problem shapes.

    ``problems``: list of dicts with F, h, T, status (the forward solution),
    dL_dT and dL_dF (output; problems may share one dL_dF tensor, whose result
    is then the sum of their gradients)."""

    def __init__(self, problems):
        self.lib = load_library()
        if not problems:
            raise FmmError(FMM_EINVAL, "empty adjoint batch")
        dt = problems[0]["F"].dtype
        self.dtype = _dtype_code(dt)
        n = len(problems)
        arr = (FmmAdjointProblem * n)()
        self.keep = []
        for i, q in enumerate(problems):
            F, T, st, gT, gF = q["F"], q["T"], q["status"], q["dL_dT"], q["dL_dF"]
            shape = tuple(F.shape)
            for name, t, want in (("T", T, torch.float64), ("status", st, torch.uint8),
                                  ("dL_dT", gT, torch.float64), ("dL_dF", gF, torch.float64)):
                if t.dtype != want or tuple(t.shape) != shape or not t.is_contiguous() or not t.is_cuda:
                    raise FmmError(FMM_EINVAL, f"adjoint problem {i}: {name} must be a contiguous CUDA {want} "
                                               f"tensor of shape {shape}")
            if F.dtype != dt or not F.is_contiguous() or F.dim() != 3:
                raise FmmError(FMM_EINVAL, f"adjoint problem {i}: F must be contiguous 3-D of the batch dtype")
            dev0 = problems[0]["F"].device
            for name, t in (("F", F), ("T", T), ("status", st), ("dL_dT", gT), ("dL_dF", gF)):
                _check_cuda(f"adjoint problem {i}: {name}", t, dev0)
            self.keep += [F, T, st, gT, gF]
            p = arr[i]
            p.n0, p.n1, p.n2 = shape
            p.h = float(q["h"])
            p.F, p.T, p.status = F.data_ptr(), T.data_ptr(), st.data_ptr()
            p.dL_dT, p.dL_dF = gT.data_ptr(), gF.data_ptr()
            sc = q.get("axis_scale")
            if sc is not None:
                for a in range(3):
                    p.axis_scale[a] = float(sc[a])
        self.n = n
        self.problems = arr
        nbytes = int(self.lib.fmm_adjoint_workspace_bytes(n, arr))
        if nbytes == 0:
            raise FmmError(FMM_EINVAL, "invalid adjoint batch")
        dev = problems[0]["F"].device
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-self.workspace.data_ptr()) % 256
        self.ws = self.workspace[off:off + nbytes]
        self.nbytes = nbytes

    def run(self, stream=None) -> None:
        rc = self.lib.fmm_adjoint_batch(self.n, self.problems, self.dtype, _ptr(self.ws), self.nbytes,
                                        _stream_handle(stream))
        if rc != FMM_OK:
            raise FmmError(rc, f"fmm_adjoint_batch: {strerror(rc)}")

    def stats(self, stream=None, check=True) -> FmmAdjointStats:
        st = FmmAdjointStats()
        rc = self.lib.fmm_get_adjoint_stats(_ptr(self.ws), ctypes.byref(st), _stream_handle(stream))
        if check and rc != FMM_OK:
            raise FmmError(rc, f"adjoint failed on the device: {strerror(rc)}")
        return st


def adjoint(F, h, T, status, dL_dT, axis_scale=None):
    """dL/dF (float64, F's shape) for one solved problem."""
    gF = torch.empty(F.shape, dtype=torch.float64, device=F.device)
    a = AdjointSolver([{"F": F, "h": h, "T": T, "status": status, "dL_dT": dL_dT.contiguous(), "dL_dF": gF,
                        "axis_scale": axis_scale}])
    a.run()
    a.stats()
    return gF


class Eikonal(torch.autograd.Function):
    """T = solve(F) with the library's adjoint as backward: dL/dF from dL/dT.

    ``forward(F, h, seed_idx, seed_val, band_width=inf, stride=None,
    axis_scale=None)`` returns (T, status); status is not differentiable."""

    @staticmethod
    def forward(ctx, F, h, seed_idx, seed_val, band_width=math.inf, stride=None, axis_scale=None):
        T, st, _ = solve(F.detach().contiguous(), h, seed_idx, seed_val, band_width=band_width, stride=stride,
                         axis_scale=axis_scale)
        ctx.save_for_backward(F, T, st)
        ctx.h = float(h)
        ctx.axis_scale = axis_scale
        ctx.mark_non_differentiable(st)
        return T, st

    @staticmethod
    def backward(ctx, gT, gst):
        F, T, st = ctx.saved_tensors
        g = adjoint(F.detach().contiguous(), ctx.h, T, st, gT.to(torch.float64).contiguous(), ctx.axis_scale)
        return g.to(F.dtype), None, None, None, None, None, None


class EikonalShots(torch.autograd.Function):
    """Many sources ("shots") over one speed model, solved as one batch: T has
    shape (shots, n0, n1, n2), and the backward pass sums the shots'
    gradients into one dL/dF inside the library.

    ``forward(F, h, seeds, opts)``: seeds is a list of (seed_idx, seed_val);
    opts a dict of BatchSolver options."""

    @staticmethod
    def forward(ctx, F, h, seeds, opts=None):
        Fd = F.detach().contiguous()
        S = len(seeds)
        T = torch.empty((S,) + tuple(F.shape), dtype=torch.float64, device=F.device)
        st = torch.empty((S,) + tuple(F.shape), dtype=torch.uint8, device=F.device)
        probs = [{"F": Fd, "h": h, "seed_idx": i, "seed_val": v} for i, v in seeds]
        b = BatchSolver(probs, T_out=[T[k] for k in range(S)], status_out=[st[k] for k in range(S)], **(opts or {}))
        b.solve()
        b.stats()
        ctx.save_for_backward(Fd, T, st)
        ctx.h = float(h)
        ctx.axis_scale = (opts or {}).get("axis_scale")
        ctx.mark_non_differentiable(st)
        return T, st

    @staticmethod
    def backward(ctx, gT, gst):
        F, T, st = ctx.saved_tensors
        gT = gT.to(torch.float64).contiguous()
        gF = torch.empty(F.shape, dtype=torch.float64, device=F.device)
        a = AdjointSolver([{"F": F, "h": ctx.h, "T": T[k], "status": st[k], "dL_dT": gT[k], "dL_dF": gF,
                            "axis_scale": ctx.axis_scale} for k in range(T.shape[0])])
        a.run()
        a.stats()
        return gF.to(F.dtype), None, None, None
