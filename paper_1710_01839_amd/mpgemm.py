"""Thin ctypes binding of libmpgemm.so (include/mpgemm.h).

Argument marshalling only: torch tensors (float64, CUDA/HIP device, row-major
with unit column stride) are turned into device pointers, sizes and leading
dimensions, the calls run on torch's current stream, and every non-zero
status raises MpgemmError.  All arithmetic happens in the HIP library; if it
is not built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MPGEMM_LIB") or os.path.join(_HERE, "libmpgemm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -c 'import __graft_entry__ as g; g.build()'`")

_lib = ctypes.CDLL(LIB_PATH)

MPG_OK, MPG_ERR_ARG, MPG_ERR_UNSUPPORTED, MPG_ERR_HIP, MPG_ERR_NOMEM, MPG_ERR_ALIAS, MPG_ERR_STATE = \
    0, -1, -2, -3, -4, -5, -6
MPG_AUTO, MPG_SIMPLE, MPG_BLOCK, MPG_STRASSEN, MPG_OZAKI, MPG_OZAKI_CRT, MPG_SPLITK = 0, 1, 2, 3, 4, 5, 6
MPG_KCLASS_GEMM, MPG_KCLASS_AUX = 0, 1
ALGOS = {"auto": MPG_AUTO, "simple": MPG_SIMPLE, "block": MPG_BLOCK,
         "strassen": MPG_STRASSEN, "ozaki": MPG_OZAKI, "ozaki_crt": MPG_OZAKI_CRT, "splitk": MPG_SPLITK}
# pairs_mode of the split product: all digit pairs, the triangle, the residue form
PAIR_MODES = {"all": 0, "triangle": 1, "crt": 2}


class mpg_tile(ctypes.Structure):
    _fields_ = [("bm", ctypes.c_int), ("bn", ctypes.c_int), ("bk", ctypes.c_int),
                ("tm", ctypes.c_int), ("tn", ctypes.c_int), ("depth", ctypes.c_int),
                ("slices", ctypes.c_int), ("splits", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class mpg_int_algo(ctypes.Structure):
    _fields_ = [("chunk_words", ctypes.c_int), ("karatsuba_depth", ctypes.c_int)]

    def as_dict(self):
        return {"chunk_words": self.chunk_words, "karatsuba_depth": self.karatsuba_depth}


class mpg_dd_problem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("l", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("ldb", ctypes.c_int64), ("ldc", ctypes.c_int64),
                ("A_hi", ctypes.c_void_p), ("A_lo", ctypes.c_void_p),
                ("B_hi", ctypes.c_void_p), ("B_lo", ctypes.c_void_p),
                ("C_hi", ctypes.c_void_p), ("C_lo", ctypes.c_void_p)]


class MpgemmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_ci = ctypes.c_int
_pp = ctypes.POINTER(ctypes.c_void_p)
_pd = ctypes.POINTER(ctypes.c_double)


def _sig(name, args, res=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_sig("mpg_create", [ctypes.POINTER(_vp), _ci])
_sig("mpg_destroy", [_vp])
_sig("mpg_set_stream", [_vp, _vp])
_sig("mpg_status_string", [_ci], ctypes.c_char_p)
_sig("mpg_last_error", [_vp], ctypes.c_char_p)
_sig("mpg_num_variants", [_ci])
_sig("mpg_variant", [_ci, _ci, ctypes.POINTER(mpg_tile)])
_sig("mpg_variant_resident", [_vp, _ci, _ci, ctypes.POINTER(_ci)])
_sig("mpgemm_dd", [_vp, _i64, _i64, _i64, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _i64, _ci,
                   ctypes.POINTER(mpg_tile)])
_sig("mpgemm_qd", [_vp, _i64, _i64, _i64, _pp, _i64, _pp, _i64, _pp, _i64, _ci,
                   ctypes.POINTER(mpg_tile)])
_sig("mpgemm_ozaki_dd", [_vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _i64, _ci, _ci])
_sig("mpgemm_dd_ozaki", [_vp, _i64, _i64, _i64, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _i64, _ci, _ci])
_sig("mpg_ozaki_slices_exact", [_vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, ctypes.POINTER(_ci)])
_sig("mpg_ozaki_split", [_vp, _ci, _i64, _i64, _vp, _i64, _ci, _vp, _i64, _i64, _vp])
_sig("mpg_method_bound", [_ci, _ci, _ci, ctypes.POINTER(mpg_tile), _ci, _i64, _i64, _i64], ctypes.c_double)
_sig("mpg_select_method", [_vp, _i64, _i64, _i64, _ci, _ci, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                           ctypes.POINTER(mpg_tile), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_double)])
_sig("mpg_ozaki_slices_for_bits", [_ci, _ci])
_sig("mpg_ozaki_tune", [_vp, _i64, _i64, _i64, _ci, _vp, _i64, _vp, _i64, ctypes.POINTER(ctypes.c_int),
                        ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)])
_sig("mpg_ozaki_last_slices", [_vp])
_sig("mpg_ozaki_last_moduli", [_vp])
_sig("mpg_crt_moduli_for", [_ci, _i64])
_sig("mpg_rgemm", [_vp, _ci, _ci, _ci, _i64, _i64, _i64, _pd, _pp, _i64, _pp, _i64, _pd, _pp, _i64,
                   _ci, ctypes.POINTER(mpg_tile)])
_sig("mpg_zgemm_dd", [_vp, _ci, _ci, _i64, _i64, _i64, _pd, _pp, _i64, _pp, _i64, _pd, _pp, _i64,
                      _ci, ctypes.POINTER(mpg_tile)])
_sig("mpg_int_gemm", [_vp, _i64, _i64, _i64, _vp, _ci, _i64, _i64, _vp, _ci, _i64, _i64, _vp, _ci, _i64, _i64])
_sig("mpg_int_words_needed", [_ci, _ci, _i64])
_sig("mpg_int_gemm_ex", [_vp, _i64, _i64, _i64, _vp, _ci, _i64, _i64, _vp, _ci, _i64, _i64, _vp, _ci, _i64, _i64,
                         ctypes.POINTER(mpg_int_algo)])
_sig("mpg_int_num_candidates", [_ci, _ci, _i64])
_sig("mpg_int_candidate", [_ci, _ci, _i64, _ci, ctypes.POINTER(mpg_int_algo)])
_sig("mpg_int_products", [_ci, _ci, _i64, ctypes.POINTER(mpg_int_algo)], _i64)
_sig("mpg_int_time", [_vp, _i64, _i64, _i64, _ci, _ci, ctypes.POINTER(mpg_int_algo), _ci,
                      ctypes.POINTER(ctypes.c_double)])
_sig("mpg_int_predict", [_vp, _i64, _i64, _i64, _ci, _ci, ctypes.POINTER(mpg_int_algo),
                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)])
_sig("mpg_int_tune", [_vp, _i64, _i64, _i64, _ci, _ci, _ci, _ci, ctypes.POINTER(mpg_int_algo),
                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_ci)])
_sig("mpgemm_dd_batched", [_vp, _ci, ctypes.POINTER(mpg_dd_problem), ctypes.POINTER(mpg_tile)])
_sig("mpgemm_dd_batched_noalloc", [_vp, _ci, ctypes.POINTER(mpg_dd_problem), ctypes.POINTER(mpg_tile)])
_sig("mpg_batch_plan_create", [_vp, _ci, ctypes.POINTER(mpg_dd_problem), ctypes.POINTER(mpg_tile),
                               ctypes.POINTER(_vp)])
_sig("mpg_batch_plan_launch", [_vp, _vp])
_sig("mpg_batch_plan_update", [_vp, ctypes.POINTER(mpg_dd_problem)])
_sig("mpg_batch_plan_destroy", [_vp])
_f = ctypes.POINTER(ctypes.c_float)
_d = ctypes.POINTER(ctypes.c_double)
_sig("mpg_num_candidates", [_ci, _i64, _i64, _i64])
_sig("mpg_candidate", [_ci, _i64, _i64, _i64, _ci, ctypes.POINTER(_ci), ctypes.POINTER(mpg_tile)])
_sig("mpg_tune_set_db", [_vp, ctypes.c_char_p])
_sig("mpg_time_candidate", [_vp, _ci, _i64, _i64, _i64, _ci, ctypes.POINTER(mpg_tile), _ci, _d])
_sig("mpg_predict_block", [_vp, _ci, _i64, _i64, _i64, ctypes.POINTER(mpg_tile), _ci, _d, _d])
_sig("mpg_predict_slab", [_ci, _i64, _i64, _i64, ctypes.POINTER(mpg_tile), _ci, _ci, _ci,
                          ctypes.POINTER(_i64), ctypes.POINTER(_i64), _d])
_sig("mpg_tune", [_vp, _ci, _i64, _i64, _i64, _ci, _ci, ctypes.POINTER(_ci), ctypes.POINTER(mpg_tile),
                  _d, _d, ctypes.POINTER(_ci)])
_sig("mpg_tune_table_set", [_vp, _ci, _i64, _i64, _i64, _ci, ctypes.POINTER(mpg_tile)])
_sig("mpg_mlp_features", [_ci, _i64, _i64, _i64, _ci, ctypes.POINTER(mpg_tile), _ci, _f])
_sig("mpg_mlp_num_params", [])
_sig("mpg_mlp_set_params", [_vp, _f, _ci])
_sig("mpg_mlp_get_params", [_vp, _f, _ci])
_sig("mpg_mlp_grad", [_vp, _f, _f, _ci, _f, _f])
_sig("mpg_mlp_train", [_vp, _f, _f, _ci, _ci, ctypes.c_float, _f])
_sig("mpg_mlp_train_db", [_vp, ctypes.c_char_p, _ci, ctypes.c_float, _f, ctypes.POINTER(_ci)])
_sig("mpg_mlp_predict", [_vp, _f, _ci, _f])
_sig("mpg_mlp_save", [_vp, ctypes.c_char_p])
_sig("mpg_mlp_load", [_vp, ctypes.c_char_p])
_sig("mpg_prof_enable", [_vp, _ci])
_sig("mpg_prof_read", [_vp, _ci, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)])
_sig("mpg_test_inject", [_vp, _ci, _ci])
_sig("mpg_int8_mfma_rate", [_vp, ctypes.POINTER(ctypes.c_double)])


def lib():
    return _lib


def status_string(status: int) -> str:
    return _lib.mpg_status_string(status).decode()


class Context:
    """Owns an mpg_ctx on one device; every call uses torch's current stream."""

    def __init__(self, device: int | None = None):
        if device is None:
            device = torch.cuda.current_device()
        self.device = device
        h = _vp()
        st = _lib.mpg_create(ctypes.byref(h), device)
        if st != MPG_OK:
            raise MpgemmError(st, "mpg_create: " + status_string(st))
        self.handle = h

    def close(self):
        if self.handle:
            _lib.mpg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st: int, what: str):
        if st != MPG_OK:
            detail = _lib.mpg_last_error(self.handle).decode()
            raise MpgemmError(st, f"{what}: {status_string(st)}: {detail}")

    def bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        _lib.mpg_set_stream(self.handle, _vp(s))

    def variant_resident(self, precision, index: int) -> int:
        """Workgroups of a block variant resident per CU (occupancy calculator)."""
        b = _ci()
        self.check(_lib.mpg_variant_resident(self.handle, _prec(precision), index, ctypes.byref(b)),
                   "mpg_variant_resident")
        return b.value

    def inject(self, kind: str, count: int):
        """Failure injection for tests: the next `count` workspace
        allocations ("alloc") or kernel launches ("launch") of this context
        fail without touching the GPU."""
        self.check(_lib.mpg_test_inject(self.handle, {"alloc": 1, "launch": 2}[kind], count),
                   "mpg_test_inject")

    # --- kernel timing -------------------------------------------------
    def prof_enable(self, on: bool = True):
        self.check(_lib.mpg_prof_enable(self.handle, int(on)), "mpg_prof_enable")

    def prof_read(self, kclass: int = MPG_KCLASS_GEMM):
        ms = ctypes.c_double()
        n = _i64()
        self.check(_lib.mpg_prof_read(self.handle, kclass, ctypes.byref(ms), ctypes.byref(n)),
                   "mpg_prof_read")
        return ms.value, n.value


def make_tile(tile=None) -> mpg_tile | None:
    if tile is None:
        return None
    if isinstance(tile, mpg_tile):
        return tile
    t = mpg_tile()
    for k, v in dict(tile).items():
        setattr(t, k, int(v))
    return t


def variants(precision=2):
    out = []
    precision = _prec(precision)
    for i in range(_lib.mpg_num_variants(precision)):
        t = mpg_tile()
        _lib.mpg_variant(precision, i, ctypes.byref(t))
        out.append(t.as_dict())
    return out


def _ptr(t):
    return _vp(t.data_ptr()) if t is not None else _vp(0)


def _mat(t: torch.Tensor, name: str):
    if t.dtype != torch.float64 or not t.is_cuda:
        raise MpgemmError(MPG_ERR_ARG, f"{name} must be a float64 device tensor")
    if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1):
        raise MpgemmError(MPG_ERR_ARG, f"{name} must be 2-D with unit column stride")
    return t.shape[0], t.shape[1], max(t.stride(0), 1)


def mpgemm_dd(ctx: Context, A, B, C, algo="block", tile=None):
    """C := A B in double-double.  A, B, C: (hi, lo) tuples of tensors."""
    m, l, lda = _mat(A[0], "A_hi")
    l2, n, ldb = _mat(B[0], "B_hi")
    m2, n2, ldc = _mat(C[0], "C_hi")
    if l2 != l or m2 != m or n2 != n:
        raise MpgemmError(MPG_ERR_ARG, f"shape mismatch {tuple(A[0].shape)} {tuple(B[0].shape)} "
                                       f"{tuple(C[0].shape)}")
    for t, nm in ((A[1], "A_lo"), (B[1], "B_lo"), (C[1], "C_lo")):
        _mat(t, nm)
    t = make_tile(tile)
    ctx.bind_stream()
    st = _lib.mpgemm_dd(ctx.handle, m, n, l, _ptr(A[0]), _ptr(A[1]), lda, _ptr(B[0]), _ptr(B[1]),
                        ldb, _ptr(C[0]), _ptr(C[1]), ldc, ALGOS.get(algo, algo) if isinstance(algo, str) else algo,
                        ctypes.byref(t) if t is not None else None)
    ctx.check(st, "mpgemm_dd")
    return C


def _limb_array(ts):
    arr = (ctypes.c_void_p * 4)(*[t.data_ptr() for t in ts])
    return ctypes.cast(arr, _pp), arr


def mpgemm_qd(ctx: Context, A, B, C, algo="block", tile=None):
    """C := A B in quad-double.  A, B, C: 4-tuples of limb tensors."""
    m, l, lda = _mat(A[0], "A[0]")
    l2, n, ldb = _mat(B[0], "B[0]")
    m2, n2, ldc = _mat(C[0], "C[0]")
    if l2 != l or m2 != m or n2 != n:
        raise MpgemmError(MPG_ERR_ARG, "shape mismatch")
    for q in range(4):
        _mat(A[q], f"A[{q}]"); _mat(B[q], f"B[{q}]"); _mat(C[q], f"C[{q}]")
    pa, ka = _limb_array(A)
    pb, kb = _limb_array(B)
    pc, kc = _limb_array(C)
    t = make_tile(tile)
    ctx.bind_stream()
    st = _lib.mpgemm_qd(ctx.handle, m, n, l, pa, lda, pb, ldb, pc, ldc,
                        ALGOS.get(algo, algo) if isinstance(algo, str) else algo,
                        ctypes.byref(t) if t is not None else None)
    ctx.check(st, "mpgemm_qd")
    return C


OPS = {"N": 0, "T": 1, "C": 2}


def _planes(X, count: int, name: str):
    """Shape and common leading dimension of `count` limb planes."""
    if len(X) != count:
        raise MpgemmError(MPG_ERR_ARG, f"{name} needs {count} planes")
    r, c, ld = _mat(X[0], f"{name}[0]")
    for q in range(1, count):
        if _mat(X[q], f"{name}[{q}]") != (r, c, ld):
            raise MpgemmError(MPG_ERR_ARG, f"{name} planes differ in shape or leading dimension")
    return r, c, ld


def _scalar(x, count: int):
    v = [float(x)] if isinstance(x, (int, float)) else [float(y) for y in x]
    v = (v + [0.0] * count)[:count]
    return (ctypes.c_double * count)(*v)


def _op_shape(r, c, trans):
    return (r, c) if trans == "N" else (c, r)


def rgemm(ctx: Context, A, B, C, alpha=1.0, beta=0.0, transa="N", transb="N", algo="block",
          tile=None):
    """C := alpha op(A) op(B) + beta C in DD (2-tuples of planes) or QD
    (4-tuples).  alpha, beta: a float or a sequence of limbs.  transa,
    transb: 'N', 'T' or 'C' (the transpose for real matrices)."""
    L = len(C)
    mc, nc, ldc = _planes(C, L, "C")
    ar, ac, lda = _planes(A, L, "A")
    br, bc, ldb = _planes(B, L, "B")
    m, k = _op_shape(ar, ac, transa)
    k2, n = _op_shape(br, bc, transb)
    if (m, n) != (mc, nc) or k != k2:
        raise MpgemmError(MPG_ERR_ARG, "shape mismatch")
    pa, ka = _limb_array(A)
    pb, kb = _limb_array(B)
    pc, kc = _limb_array(C)
    t = make_tile(tile)
    ctx.bind_stream()
    st = _lib.mpg_rgemm(ctx.handle, L, OPS[transa], OPS[transb], m, n, k,
                        ctypes.cast(_scalar(alpha, L), _pd), pa, lda, pb, ldb,
                        ctypes.cast(_scalar(beta, L), _pd), pc, ldc,
                        ALGOS.get(algo, algo) if isinstance(algo, str) else algo,
                        ctypes.byref(t) if t is not None else None)
    ctx.check(st, "mpg_rgemm")
    return C


def zgemm_dd(ctx: Context, A, B, C, alpha=(1.0, 0.0, 0.0, 0.0), beta=(0.0, 0.0, 0.0, 0.0),
             transa="N", transb="N", algo="block", tile=None):
    """Complex DD C := alpha op(A) op(B) + beta C.  Each matrix is a 4-tuple
    (re hi, re lo, im hi, im lo) of planes; alpha, beta are 4 limbs in the
    same order.  transa, transb: 'N', 'T' or 'C' (conjugate transpose)."""
    mc, nc, ldc = _planes(C, 4, "C")
    ar, ac, lda = _planes(A, 4, "A")
    br, bc, ldb = _planes(B, 4, "B")
    m, k = _op_shape(ar, ac, transa)
    k2, n = _op_shape(br, bc, transb)
    if (m, n) != (mc, nc) or k != k2:
        raise MpgemmError(MPG_ERR_ARG, "shape mismatch")
    pa, ka = _limb_array(A)
    pb, kb = _limb_array(B)
    pc, kc = _limb_array(C)
    t = make_tile(tile)
    ctx.bind_stream()
    st = _lib.mpg_zgemm_dd(ctx.handle, OPS[transa], OPS[transb], m, n, k,
                           ctypes.cast(_scalar(alpha, 4), _pd), pa, lda, pb, ldb,
                           ctypes.cast(_scalar(beta, 4), _pd), pc, ldc,
                           ALGOS.get(algo, algo) if isinstance(algo, str) else algo,
                           ctypes.byref(t) if t is not None else None)
    ctx.check(st, "mpg_zgemm_dd")
    return C


def int_words_needed(words_a: int, words_b: int, l: int) -> int:
    return int(_lib.mpg_int_words_needed(int(words_a), int(words_b), int(l)))


def _words(t: torch.Tensor, name: str):
    if t.dtype != torch.int32 or not t.is_cuda or t.dim() != 3 or not t.is_contiguous():
        raise MpgemmError(MPG_ERR_ARG, f"{name} must be a contiguous int32 device tensor (words, rows, cols)")
    return t.shape[0], t.shape[1], t.shape[2]


def _int_algo(algo):
    if algo is None:
        return None
    if isinstance(algo, mpg_int_algo):
        return algo
    a = mpg_int_algo()
    a.chunk_words = int(algo.get("chunk_words", 4))
    a.karatsuba_depth = int(algo.get("karatsuba_depth", 0))
    return a


def int_gemm(ctx: Context, A, B, C, algo=None):
    """C := A B exactly for long integers stored as word planes: int32 device
    tensors of shape (words, rows, cols), word 0 least significant, two's
    complement over all words (the bits are read as unsigned words).  algo:
    {"chunk_words", "karatsuba_depth"} or None (tuning table, else 128-bit
    chunks without splitting)."""
    wa, m, l = _words(A, "A")
    wb, l2, n = _words(B, "B")
    wc, m2, n2 = _words(C, "C")
    if l2 != l or (m2, n2) != (m, n):
        raise MpgemmError(MPG_ERR_ARG, "shape mismatch")
    a = _int_algo(algo)
    ctx.bind_stream()
    st = _lib.mpg_int_gemm_ex(ctx.handle, m, n, l, _ptr(A), wa, l, m * l, _ptr(B), wb, n, l * n,
                              _ptr(C), wc, n, m * n, ctypes.byref(a) if a is not None else None)
    ctx.check(st, "mpg_int_gemm_ex")
    return C


def int_candidates(words_a: int, words_b: int, l: int):
    out = []
    for i in range(_lib.mpg_int_num_candidates(words_a, words_b, l)):
        a = mpg_int_algo()
        _lib.mpg_int_candidate(words_a, words_b, l, i, ctypes.byref(a))
        out.append(a.as_dict())
    return out


def int_products(words_a: int, words_b: int, l: int, algo) -> int:
    a = _int_algo(algo)
    return int(_lib.mpg_int_products(words_a, words_b, l, ctypes.byref(a)))


def mpgemm_ozaki_dd(ctx: Context, A, B, C, slices: int = 0, mode: str = "all"):
    """C := A B to DD accuracy on INT8 MFMA.  A, B: float64 device tensors;
    C: (hi, lo).  slices = 0 picks the exact slice count."""
    m, l, lda = _mat(A, "A")
    l2, n, ldb = _mat(B, "B")
    m2, n2, ldc = _mat(C[0], "C_hi")
    _mat(C[1], "C_lo")
    if l2 != l or m2 != m or n2 != n:
        raise MpgemmError(MPG_ERR_ARG, "shape mismatch")
    ctx.bind_stream()
    st = _lib.mpgemm_ozaki_dd(ctx.handle, m, n, l, _ptr(A), lda, _ptr(B), ldb, _ptr(C[0]),
                              _ptr(C[1]), ldc, int(slices), PAIR_MODES.get(mode, mode))
    ctx.check(st, "mpgemm_ozaki_dd")
    return C


def mpgemm_dd_ozaki(ctx: Context, A, B, C, slices: int = 0, mode: str = "all"):
    """C := A B for double-double inputs on INT8 MFMA.  A, B, C: (hi, lo)
    tuples of float64 device tensors.  slices = 0 picks the exact count."""
    m, l, lda = _mat(A[0], "A_hi")
    l2, n, ldb = _mat(B[0], "B_hi")
    m2, n2, ldc = _mat(C[0], "C_hi")
    if l2 != l or m2 != m or n2 != n:
        raise MpgemmError(MPG_ERR_ARG, "shape mismatch")
    for t, nm, ld in ((A[1], "A_lo", lda), (B[1], "B_lo", ldb), (C[1], "C_lo", ldc)):
        if _mat(t, nm)[2] != ld:
            raise MpgemmError(MPG_ERR_ARG, f"{nm} must share its hi limb's leading dimension")
    ctx.bind_stream()
    st = _lib.mpgemm_dd_ozaki(ctx.handle, m, n, l, _ptr(A[0]), _ptr(A[1]), lda, _ptr(B[0]), _ptr(B[1]),
                              ldb, _ptr(C[0]), _ptr(C[1]), ldc, int(slices), PAIR_MODES.get(mode, mode))
    ctx.check(st, "mpgemm_dd_ozaki")
    return C


def int8_mfma_rate(ctx: Context) -> float:
    """Sustained INT8 matrix-core rate of the device, TOP/s."""
    t = ctypes.c_double()
    ctx.bind_stream()
    ctx.check(_lib.mpg_int8_mfma_rate(ctx.handle, ctypes.byref(t)), "mpg_int8_mfma_rate")
    return t.value


def ozaki_last_slices(ctx: Context) -> int:
    return int(_lib.mpg_ozaki_last_slices(ctx.handle))


def ozaki_last_moduli(ctx: Context) -> int:
    """Moduli of the last residue-form ('crt') product."""
    return int(_lib.mpg_ozaki_last_moduli(ctx.handle))


def crt_moduli_for(slices: int, l: int) -> int:
    return int(_lib.mpg_crt_moduli_for(int(slices), int(l)))


def method_bound(in_limbs, precision, algo, tile=None, mode="all", m=1, n=1, l=1) -> float:
    """A-priori normwise bound of a method (units of l max|A| max|B|)."""
    t = make_tile(tile)
    return float(_lib.mpg_method_bound(int(in_limbs), _prec(precision),
                                       ALGOS.get(algo, algo) if isinstance(algo, str) else algo,
                                       ctypes.byref(t) if t is not None else None,
                                       PAIR_MODES.get(mode, mode), m, n, l))


def ozaki_slices_for_bits(bits: int, mode: str = "all") -> int:
    """Fewest slices whose a-priori bound meets 2^-bits (0: unreachable)."""
    return int(_lib.mpg_ozaki_slices_for_bits(int(bits), 1 if mode in ("triangle", 1) else 0))


def ozaki_slices_exact(ctx: Context, A, B) -> int:
    m, l, lda = _mat(A, "A")
    _, n, ldb = _mat(B, "B")
    out = ctypes.c_int()
    ctx.bind_stream()
    ctx.check(_lib.mpg_ozaki_slices_exact(ctx.handle, m, n, l, _ptr(A), lda, _ptr(B), ldb,
                                          ctypes.byref(out)), "mpg_ozaki_slices_exact")
    return out.value


def ozaki_split(ctx: Context, X, slices: int, side: int = 0):
    """Digit planes and exponents of X's rows (side 0) or columns (side 1).
    Returns (planes int8 [slices, lines_pad, len_pad], exps int32)."""
    rows, cols, ldx = _mat(X, "X")
    lines, length = (rows, cols) if side == 0 else (cols, rows)
    lp, kp = -(-lines // 64) * 64, -(-length // 64) * 64
    out = torch.zeros((slices, lp, kp), dtype=torch.int8, device=X.device)
    exps = torch.zeros(lines, dtype=torch.int32, device=X.device)
    ctx.bind_stream()
    ctx.check(_lib.mpg_ozaki_split(ctx.handle, side, rows, cols, _ptr(X), ldx, slices, _ptr(out),
                                   kp, lp * kp, _ptr(exps)), "mpg_ozaki_split")
    return out, exps


def _problems(probs):
    """probs: list of (A, B, C) with A, B, C (hi, lo) tensor pairs."""
    arr = (mpg_dd_problem * max(1, len(probs)))()
    for i, (A, B, C) in enumerate(probs):
        m, l, lda = _mat(A[0], "A_hi")
        l2, n, ldb = _mat(B[0], "B_hi")
        m2, n2, ldc = _mat(C[0], "C_hi")
        if l2 != l or m2 != m or n2 != n:
            raise MpgemmError(MPG_ERR_ARG, f"problem {i}: shape mismatch")
        arr[i] = mpg_dd_problem(m, n, l, lda, ldb, ldc, A[0].data_ptr(), A[1].data_ptr(),
                                B[0].data_ptr(), B[1].data_ptr(), C[0].data_ptr(), C[1].data_ptr())
    return arr


def mpgemm_dd_batched(ctx: Context, probs, tile=None):
    arr = _problems(probs)
    t = make_tile(tile)
    ctx.bind_stream()
    ctx.check(_lib.mpgemm_dd_batched(ctx.handle, len(probs), arr,
                                     ctypes.byref(t) if t is not None else None), "mpgemm_dd_batched")


def mpgemm_dd_batched_noalloc(ctx: Context, probs, tile=None):
    """mpgemm_dd_batched without allocation (a fixed device array per GPU)."""
    arr = _problems(probs)
    t = make_tile(tile)
    ctx.bind_stream()
    ctx.check(_lib.mpgemm_dd_batched_noalloc(ctx.handle, len(probs), arr,
                                             ctypes.byref(t) if t is not None else None),
              "mpgemm_dd_batched_noalloc")


class BatchPlan:
    """A persistent batched launch captured once in a HIP graph."""

    def __init__(self, ctx: Context, probs, tile=None):
        self.ctx = ctx
        self.count = len(probs)
        self._keep = probs
        arr = _problems(probs)
        t = make_tile(tile)
        h = _vp()
        ctx.bind_stream()
        ctx.check(_lib.mpg_batch_plan_create(ctx.handle, self.count, arr,
                                             ctypes.byref(t) if t is not None else None,
                                             ctypes.byref(h)), "mpg_batch_plan_create")
        self.handle = h

    def launch(self):
        self.ctx.bind_stream()
        self.ctx.check(_lib.mpg_batch_plan_launch(self.handle, None), "mpg_batch_plan_launch")

    def update(self, probs):
        if len(probs) != self.count:
            raise MpgemmError(MPG_ERR_ARG, "update needs the same problem count")
        self._keep = probs
        self.ctx.bind_stream()
        self.ctx.check(_lib.mpg_batch_plan_update(self.handle, _problems(probs)), "mpg_batch_plan_update")

    def close(self):
        if getattr(self, "handle", None):
            _lib.mpg_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MLP_FEATURES = 15
TUNE_MODES = {"exhaustive": 0, "paper": 1, "mlp": 2}
PRECISION = {"dd": 2, "qd": 4}


def _prec(p):
    return PRECISION.get(p, p) if isinstance(p, str) else int(p)


def candidates(precision, m, n, l):
    p = _prec(precision)
    out = []
    for i in range(_lib.mpg_num_candidates(p, m, n, l)):
        a, t = ctypes.c_int(), mpg_tile()
        _lib.mpg_candidate(p, m, n, l, i, ctypes.byref(a), ctypes.byref(t))
        out.append((a.value, t.as_dict()))
    return out


def predict_slab(precision, m, n, l, tile=None, rule=0, num_cu=256, resident=1):
    """Slabs the block-time prediction times (host only): (rows, rows2,
    scale); rows2 = 0 for a single slab."""
    rows, rows2, scale = _i64(), _i64(), ctypes.c_double()
    t = make_tile(tile)
    st = _lib.mpg_predict_slab(_prec(precision), m, n, l, ctypes.byref(t) if t is not None else None,
                               rule, num_cu, resident, ctypes.byref(rows), ctypes.byref(rows2),
                               ctypes.byref(scale))
    if st != MPG_OK:
        raise MpgemmError(st, "mpg_predict_slab")
    return rows.value, rows2.value, scale.value


def mlp_features(precision, m, n, l, algo, tile=None, batch=1):
    import numpy as np
    out = np.zeros(MLP_FEATURES, dtype=np.float32)
    t = make_tile(tile)
    st = _lib.mpg_mlp_features(_prec(precision), m, n, l, ALGOS.get(algo, algo) if isinstance(algo, str) else algo,
                               ctypes.byref(t) if t is not None else None, batch,
                               out.ctypes.data_as(_f))
    if st != MPG_OK:
        raise MpgemmError(st, "mpg_mlp_features")
    return out


def _fp(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(_f)


class Tuner:
    """Tuner calls on a context (library-owned timing buffers)."""

    def __init__(self, ctx: Context):
        self.ctx = ctx

    def set_db(self, path):
        self.ctx.check(_lib.mpg_tune_set_db(self.ctx.handle, path.encode() if path else None),
                       "mpg_tune_set_db")

    def time(self, precision, m, n, l, algo, tile=None, reps=3):
        ms = ctypes.c_double()
        t = make_tile(tile)
        self.ctx.bind_stream()
        self.ctx.check(_lib.mpg_time_candidate(self.ctx.handle, _prec(precision), m, n, l,
                                               ALGOS.get(algo, algo) if isinstance(algo, str) else algo,
                                               ctypes.byref(t) if t is not None else None, reps,
                                               ctypes.byref(ms)), "mpg_time_candidate")
        return ms.value

    def predict_block(self, precision, m, n, l, tile=None, rule=0):
        pred, slab = ctypes.c_double(), ctypes.c_double()
        t = make_tile(tile)
        self.ctx.bind_stream()
        self.ctx.check(_lib.mpg_predict_block(self.ctx.handle, _prec(precision), m, n, l,
                                              ctypes.byref(t) if t is not None else None, rule,
                                              ctypes.byref(pred), ctypes.byref(slab)), "mpg_predict_block")
        return pred.value, slab.value

    def tune(self, precision, m, n, l, mode="exhaustive", topk=0):
        a, t = ctypes.c_int(), mpg_tile()
        ms, secs, trials = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        self.ctx.bind_stream()
        self.ctx.check(_lib.mpg_tune(self.ctx.handle, _prec(precision), m, n, l,
                                     TUNE_MODES.get(mode, mode), topk, ctypes.byref(a), ctypes.byref(t),
                                     ctypes.byref(ms), ctypes.byref(secs), ctypes.byref(trials)), "mpg_tune")
        return {"algo": a.value, "tile": t.as_dict(), "ms": ms.value, "seconds": secs.value,
                "trials": trials.value}

    def tune_slices(self, m, n, l, bits, A=None, B=None):
        """Slice count and pair set of the FP64-input split product for a
        target of `bits`, by measured time; A, B (device tensors) let the
        exact slice count of the data compete."""
        S, pm, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        self.ctx.bind_stream()
        lda = _mat(A, "A")[2] if A is not None else 0
        ldb = _mat(B, "B")[2] if B is not None else 0
        self.ctx.check(_lib.mpg_ozaki_tune(self.ctx.handle, m, n, l, int(bits), _ptr(A), lda, _ptr(B), ldb,
                                           ctypes.byref(S), ctypes.byref(pm), ctypes.byref(ms)), "mpg_ozaki_tune")
        return {"slices": S.value, "pairs": "triangle" if pm.value else "all", "ms": ms.value}

    def select(self, m, n, l, bits, in_limbs=2):
        """Fastest method whose a-priori normwise bound meets 2^-bits
        (max |C - AB| <= 2^-bits l max|A| max|B|) for inputs of in_limbs."""
        p, a, pm = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        t = mpg_tile()
        bb, ms = ctypes.c_double(), ctypes.c_double()
        self.ctx.bind_stream()
        self.ctx.check(_lib.mpg_select_method(self.ctx.handle, m, n, l, int(in_limbs), int(bits), ctypes.byref(p),
                                              ctypes.byref(a), ctypes.byref(t), ctypes.byref(pm), ctypes.byref(bb),
                                              ctypes.byref(ms)), "mpg_select_method")
        return {"precision": p.value, "algo": a.value, "tile": t.as_dict(),
                "pairs": ("all", "triangle", "crt")[pm.value], "bound_bits": bb.value, "ms": ms.value}

    def int_time(self, m, n, l, words_a, words_b, algo, reps=3):
        ms = ctypes.c_double()
        a = _int_algo(algo)
        self.ctx.bind_stream()
        self.ctx.check(_lib.mpg_int_time(self.ctx.handle, m, n, l, words_a, words_b, ctypes.byref(a), reps,
                                         ctypes.byref(ms)), "mpg_int_time")
        return ms.value

    def int_predict(self, m, n, l, words_a, words_b, algo):
        pred, slab = ctypes.c_double(), ctypes.c_double()
        a = _int_algo(algo)
        self.ctx.bind_stream()
        self.ctx.check(_lib.mpg_int_predict(self.ctx.handle, m, n, l, words_a, words_b, ctypes.byref(a),
                                            ctypes.byref(pred), ctypes.byref(slab)), "mpg_int_predict")
        return pred.value, slab.value

    def int_tune(self, m, n, l, words_a, words_b, mode="exhaustive", topk=0):
        a = mpg_int_algo()
        ms, secs, trials = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        self.ctx.bind_stream()
        self.ctx.check(_lib.mpg_int_tune(self.ctx.handle, m, n, l, words_a, words_b, TUNE_MODES.get(mode, mode),
                                         topk, ctypes.byref(a), ctypes.byref(ms), ctypes.byref(secs),
                                         ctypes.byref(trials)), "mpg_int_tune")
        return {"algo": a.as_dict(), "ms": ms.value, "seconds": secs.value, "trials": trials.value}

    def table_set(self, precision, m, n, l, algo, tile=None):
        """Put a choice into the table MPG_AUTO follows."""
        t = make_tile(tile)
        self.ctx.check(_lib.mpg_tune_table_set(self.ctx.handle, _prec(precision), m, n, l,
                                               ALGOS.get(algo, algo) if isinstance(algo, str) else algo,
                                               ctypes.byref(t) if t is not None else None),
                       "mpg_tune_table_set")


class MLP:
    """The run-time model owned by a context (GPU kernels)."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self.nparams = _lib.mpg_mlp_num_params()

    def set_params(self, flat):
        a, p = _fp(flat)
        self.ctx.check(_lib.mpg_mlp_set_params(self.ctx.handle, p, a.size), "mpg_mlp_set_params")

    def get_params(self):
        import numpy as np
        out = np.zeros(self.nparams, dtype=np.float32)
        self.ctx.check(_lib.mpg_mlp_get_params(self.ctx.handle, out.ctypes.data_as(_f), out.size),
                       "mpg_mlp_get_params")
        return out

    def grad(self, X, y):
        import numpy as np
        Xa, Xp = _fp(X)
        ya, yp = _fp(y)
        g = np.zeros(self.nparams, dtype=np.float32)
        loss = ctypes.c_float()
        self.ctx.bind_stream()
        self.ctx.check(_lib.mpg_mlp_grad(self.ctx.handle, Xp, yp, ya.size, ctypes.byref(loss),
                                         g.ctypes.data_as(_f)), "mpg_mlp_grad")
        return loss.value, g

    def train(self, X, y, epochs, lr=1e-3):
        import numpy as np
        Xa, Xp = _fp(X)
        ya, yp = _fp(y)
        losses = np.zeros(epochs, dtype=np.float32)
        self.ctx.bind_stream()
        self.ctx.check(_lib.mpg_mlp_train(self.ctx.handle, Xp, yp, ya.size, epochs, lr,
                                          losses.ctypes.data_as(_f)), "mpg_mlp_train")
        return losses

    def train_db(self, path, epochs, lr=1e-3):
        loss, rows = ctypes.c_float(), ctypes.c_int()
        self.ctx.bind_stream()
        self.ctx.check(_lib.mpg_mlp_train_db(self.ctx.handle, path.encode(), epochs, lr,
                                             ctypes.byref(loss), ctypes.byref(rows)), "mpg_mlp_train_db")
        return loss.value, rows.value

    def predict(self, X):
        import numpy as np
        Xa, Xp = _fp(X)
        out = np.zeros(Xa.shape[0], dtype=np.float32)
        self.ctx.bind_stream()
        self.ctx.check(_lib.mpg_mlp_predict(self.ctx.handle, Xp, Xa.shape[0], out.ctypes.data_as(_f)),
                       "mpg_mlp_predict")
        return out

    def save(self, path):
        self.ctx.check(_lib.mpg_mlp_save(self.ctx.handle, path.encode()), "mpg_mlp_save")

    def load(self, path):
        self.ctx.check(_lib.mpg_mlp_load(self.ctx.handle, path.encode()), "mpg_mlp_load")


def empty_like_limbs(m: int, n: int, limbs: int, device="cuda"):
    return tuple(torch.empty((m, n), dtype=torch.float64, device=device) for _ in range(limbs))


def to_device(planes, device="cuda"):
    return tuple(torch.as_tensor(p).to(device=device, dtype=torch.float64).contiguous() for p in planes)


def to_host(planes):
    return tuple(p.detach().cpu().numpy() for p in planes)
