"""ctypes front end of the plain C oracle (``oracle/mpref.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark.  The GPU library never imports it.

A matrix of L-limb numbers is a tuple of L C-contiguous float64 numpy arrays
(limb planes), limb 0 the leading one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpref.c")
_LIB = os.path.join(_HERE, "libmpref.so")
_lib = None

# -ffp-contract=off: no a*b+c fusion, every rounding is the one written.
CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no GPU toolchain involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        # MPREF_LIB: another build of the same source (the sanitizer test's)
        path = os.environ.get("MPREF_LIB") or build()
        _lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(dp)
        i64 = ctypes.c_int64
        ci = ctypes.c_int
        _lib.orc_two_sum.argtypes = [i64, dp, dp, dp, dp]
        _lib.orc_fast_two_sum.argtypes = [i64, dp, dp, dp, dp]
        _lib.orc_two_prod.argtypes = [i64, ci, dp, dp, dp, dp]
        _lib.orc_num_op.argtypes = [ci, ci, i64, dp, dp, dp]
        _lib.orc_gemm_simple.argtypes = [ci, i64, i64, i64, pp, i64, pp, i64, pp, i64, ci]
        _lib.orc_gemm_strassen.argtypes = [ci, ci, ci, i64, i64, i64, pp, i64, pp, i64, pp, i64, ci]
        _lib.orc_gemm_strassen.restype = ci
        _lib.orc_gemm_exact.argtypes = [ci, ci, ci, i64, i64, i64, pp, i64, pp, i64, pp, i64, ci]
        _lib.orc_absprod_exact.argtypes = [ci, ci, i64, i64, i64, pp, i64, pp, i64, dp, i64, ci]
        _lib.orc_exact_diff.argtypes = [ci, ci, i64, pp, pp, dp]
        _lib.orc_max_threads.restype = ci
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _planes(ps):
    ps = [np.ascontiguousarray(p, dtype=np.float64) for p in ps]
    arr = (ctypes.POINTER(ctypes.c_double) * len(ps))(*[_dp(p) for p in ps])
    return ps, arr


def max_threads() -> int:
    return int(lib().orc_max_threads())


# --- element-wise error-free transforms and number ops -------------------

def two_sum(a, b):
    a = np.ascontiguousarray(a, np.float64); b = np.ascontiguousarray(b, np.float64)
    s = np.empty_like(a); e = np.empty_like(a)
    lib().orc_two_sum(a.size, _dp(a), _dp(b), _dp(s), _dp(e))
    return s, e


def fast_two_sum(a, b):
    a = np.ascontiguousarray(a, np.float64); b = np.ascontiguousarray(b, np.float64)
    s = np.empty_like(a); e = np.empty_like(a)
    lib().orc_fast_two_sum(a.size, _dp(a), _dp(b), _dp(s), _dp(e))
    return s, e


def two_prod(a, b, use_fma: bool = False):
    a = np.ascontiguousarray(a, np.float64); b = np.ascontiguousarray(b, np.float64)
    p = np.empty_like(a); e = np.empty_like(a)
    lib().orc_two_prod(a.size, int(use_fma), _dp(a), _dp(b), _dp(p), _dp(e))
    return p, e


def num_op(op: str, x, y):
    """x, y: tuples of L limb arrays (same shape).  op in {'add', 'mul'}."""
    L = len(x)
    X = np.ascontiguousarray(np.stack(x, axis=-1), np.float64)
    Y = np.ascontiguousarray(np.stack(y, axis=-1), np.float64)
    out = np.empty_like(X)
    n = X.size // L
    lib().orc_num_op(L, 0 if op == "add" else 1, n, _dp(X), _dp(Y), _dp(out))
    return tuple(np.ascontiguousarray(out[..., q]) for q in range(L))


# --- GEMM -----------------------------------------------------------------

def _shape(A, B):
    m, l = A[0].shape
    l2, n = B[0].shape
    assert l == l2
    return m, n, l


def gemm_simple(A, B, threads: int = 0):
    """Eq. (1) step by step in DD (2 limbs) or QD (4 limbs)."""
    L = len(A)
    assert len(B) == L and L in (2, 4)
    m, n, l = _shape(A, B)
    C = tuple(np.zeros((m, n)) for _ in range(L))
    Ap, Aa = _planes(A); Bp, Ba = _planes(B); Cp, Ca = _planes(C)
    lib().orc_gemm_simple(L, m, n, l, Aa, l, Ba, n, Ca, n, threads)
    return Cp


def gemm_strassen(A, B, depth: int, variant: str = "classic", threads: int = 0):
    """Eq. (3) (variant='classic') or Winograd (variant='winograd')."""
    L = len(A)
    m, n, l = _shape(A, B)
    C = tuple(np.zeros((m, n)) for _ in range(L))
    Ap, Aa = _planes(A); Bp, Ba = _planes(B); Cp, Ca = _planes(C)
    rc = lib().orc_gemm_strassen(L, 0 if variant == "classic" else 1, depth, m, n, l,
                                 Aa, l, Ba, n, Ca, n, threads)
    if rc != 0:
        raise MemoryError("oracle Strassen allocation failed")
    return Cp


def gemm_exact(A, B, out_limbs: int | None = None, threads: int = 0):
    """Exact AB (Eq. 1 with no rounding), rounded limb by limb to nearest."""
    La, Lb = len(A), len(B)
    Lc = out_limbs or max(La, Lb)
    m, n, l = _shape(A, B)
    C = tuple(np.zeros((m, n)) for _ in range(Lc))
    Ap, Aa = _planes(A); Bp, Ba = _planes(B); Cp, Ca = _planes(C)
    lib().orc_gemm_exact(La, Lb, Lc, m, n, l, Aa, l, Ba, n, Ca, n, threads)
    return Cp


def absprod_exact(A, B, threads: int = 0):
    """(|A| |B|)_ij rounded to nearest double."""
    m, n, l = _shape(A, B)
    C = np.zeros((m, n))
    Ap, Aa = _planes(A); Bp, Ba = _planes(B)
    lib().orc_absprod_exact(len(A), len(B), m, n, l, Aa, l, Ba, n, _dp(C), n, threads)
    return C


def exact_diff(X, Y):
    """Nearest double to sum(X limbs) - sum(Y limbs), element-wise."""
    shape = X[0].shape
    Xp, Xa = _planes([np.ravel(x) for x in X])
    Yp, Ya = _planes([np.ravel(y) for y in Y])
    out = np.empty(Xp[0].size)
    lib().orc_exact_diff(len(X), len(Y), out.size, Xa, Ya, _dp(out))
    return out.reshape(shape)
