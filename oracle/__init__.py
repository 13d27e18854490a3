"""CPU oracle for the narrow-band fast marching method -- TEST INFRASTRUCTURE.

Only the test suite, the package smoke check and the benchmark's CPU baseline
may import this package.  The product path (``paper_1502_07303_amd``) never
imports it and shares no code with it.

``solve`` is the paper's sequentialised reference (Alg. 8, Alg. 9, one pass of
Alg. 12 with Alg. 10/11, bound = band width); ``godunov`` is the local solver
of Alg. 11; ``sweep`` is an independent fast-sweeping solver used only to pin
the marcher.  All arithmetic is FP64.  Parity unpinned: none (see the tests).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FMM_ORACLE_LIB selects another build of the same source (the sanitizer
# test runs the oracle suite against an AddressSanitizer build this way)
_LIB_PATH = os.environ.get("FMM_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

ST_FAR, ST_BAND, ST_ACCEPTED, ST_SEED, ST_NEG = 0, 1, 2, 3, 0x80


class OracleStats(ctypes.Structure):
    _fields_ = [("n_accepted", ctypes.c_int64), ("n_popped", ctypes.c_int64),
                ("n_solves", ctypes.c_int64), ("n_reopened", ctypes.c_int64),
                ("max_abs_T", ctypes.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64, dbl = ctypes.c_int64, ctypes.c_double
    lib.oracle_godunov.argtypes = [dbl, dbl, dbl, dbl]
    lib.oracle_godunov.restype = dbl
    lib.oracle_godunov_k.argtypes = [dbl, dbl, dbl, dbl, ctypes.POINTER(ctypes.c_int)]
    lib.oracle_godunov_k.restype = dbl
    lib.oracle_godunov_batch.argtypes = [P, P, P, i64]
    lib.oracle_godunov_batch.restype = None
    lib.oracle_solve.argtypes = [i64, i64, i64, dbl, P, ctypes.c_int, P, P, i64, dbl, P, P, P, i64,
                                 ctypes.POINTER(OracleStats), P]
    lib.oracle_godunov_w.argtypes = [dbl, dbl, dbl, dbl, dbl, dbl, dbl, ctypes.POINTER(ctypes.c_int)]
    lib.oracle_godunov_w.restype = dbl
    lib.oracle_solve.restype = ctypes.c_int
    lib.oracle_sweep.argtypes = [i64, i64, i64, dbl, P, P, P, i64, P, i64]
    lib.oracle_sweep.restype = i64
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def godunov(a1, a2, a3, r):
    """Local solver G(a1, a2, a3, r) of Alg. 11 (per-axis upwind values, +inf if absent)."""
    return _load().oracle_godunov(float(a1), float(a2), float(a3), float(r))


def godunov_k(a1, a2, a3, r):
    """(G, k): the local solve and how many of the sorted upwind values its root uses."""
    k = ctypes.c_int(0)
    u = _load().oracle_godunov_k(float(a1), float(a2), float(a3), float(r), ctypes.byref(k))
    return u, k.value


def godunov_w(a1, a2, a3, s1, s2, s3, r):
    """(G, k) with per-axis spacing factors s (weights 1 / s^2)."""
    k = ctypes.c_int(0)
    u = _load().oracle_godunov_w(float(a1), float(a2), float(a3), float(s1), float(s2), float(s3), float(r),
                                 ctypes.byref(k))
    return u, k.value


def godunov_batch(a, r):
    """Vectorised G over an (n, 3) array of upwind values and n values of r."""
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1, 3)
    r = np.ascontiguousarray(r, dtype=np.float64).reshape(-1)
    out = np.empty(r.shape, dtype=np.float64)
    _load().oracle_godunov_batch(_ptr(a), _ptr(r), _ptr(out), len(r))
    return out


def solve(F, h, seed_idx, seed_val, width=np.inf, record_order=False, axis_scale=None):
    """Sequential narrow-band FMM on the grid ``F.shape`` (C order, axis 2 fastest).

    ``axis_scale`` (3 positive factors, optional): grid spacing h * s_a along
    axis a.  Returns ``(T, status, stats, order)``; ``order`` lists the
    accepted points in pop order when ``record_order`` is set.
    """
    lib = _load()
    F = np.ascontiguousarray(F)
    if F.ndim != 3 or F.dtype not in (np.float32, np.float64):
        raise ValueError("F must be a 3-D float32/float64 array")
    n0, n1, n2 = F.shape
    N = n0 * n1 * n2
    seed_idx = np.ascontiguousarray(seed_idx, dtype=np.int64).reshape(-1)
    seed_val = np.ascontiguousarray(seed_val, dtype=np.float64).reshape(-1)
    if seed_idx.shape != seed_val.shape:
        raise ValueError("seed_idx and seed_val differ in length")
    T = np.empty(F.shape, dtype=np.float64)
    status = np.empty(F.shape, dtype=np.uint8)
    order = np.full(N, -1, dtype=np.int64) if record_order else None
    sc = None if axis_scale is None else np.ascontiguousarray(axis_scale, dtype=np.float64).reshape(3)
    st = OracleStats()
    rc = lib.oracle_solve(n0, n1, n2, float(h), _ptr(F), int(F.dtype == np.float64),
                          _ptr(seed_idx) if len(seed_idx) else None,
                          _ptr(seed_val) if len(seed_val) else None, len(seed_idx), float(width),
                          _ptr(T), _ptr(status), _ptr(order), N if record_order else 0,
                          ctypes.byref(st), _ptr(sc))
    if rc != 0:
        raise RuntimeError(f"oracle_solve failed with code {rc}")
    if record_order:
        order = order[:int(st.n_popped)]
    return T, status, st, order


def sweep(F, h, seed_idx, seed_val, max_cycles=10000):
    """Fast sweeping to a bitwise fixed point (one-sided). Returns ``(T, cycles)``."""
    lib = _load()
    F = np.ascontiguousarray(F, dtype=np.float64)
    n0, n1, n2 = F.shape
    seed_idx = np.ascontiguousarray(seed_idx, dtype=np.int64).reshape(-1)
    seed_val = np.ascontiguousarray(seed_val, dtype=np.float64).reshape(-1)
    T = np.empty(F.shape, dtype=np.float64)
    cyc = lib.oracle_sweep(n0, n1, n2, float(h), _ptr(F), _ptr(seed_idx), _ptr(seed_val),
                           len(seed_idx), _ptr(T), int(max_cycles))
    if cyc < 0:
        raise RuntimeError(f"oracle_sweep failed with code {cyc}")
    return T, int(cyc)
