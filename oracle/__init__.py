"""CPU oracle for ILU(0)-preconditioned multiple-precision Krylov solvers.

TEST INFRASTRUCTURE ONLY: plain, slow, sequential C (``mpk_oracle.c``)
behind ctypes.  Only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline of ``bench.py`` may import this package; the product library never
uses it.  It shares no code with the HIP path.

Arrays follow the layout of the C side: a vector is float64 of shape
(n, C, K) (C = 1 real, 2 complex; K limbs, highest first); a CSR matrix is
(row_ptr int32[n+1], col_idx int32[nnz], val float64[nnz, C]); an ILU(0)
factor is float64[nnz, C, kf] in the pattern of A.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmpk_oracle.so")
_lib = None

METHODS = {"bicg": 0, "cgs": 1, "bicgstab": 2, "gpbicg": 3}
STATUS = {0: "ok", 1: "not_converged", 2: "breakdown", -4: "zero_pivot", -5: "no_diag"}

_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)


def lib():
    """Load (building first if needed) the oracle shared library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        i64, i32, c_int, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_int, ctypes.c_double
        L.or_add.argtypes = [c_int, _D, _D, _D]
        L.or_mul.argtypes = [c_int, _D, _D, _D]
        L.or_mul_fp.argtypes = [c_int, _D, dbl, _D]
        L.or_mul_k.argtypes = [c_int, _D, _D, c_int, _D]
        L.or_div_k.argtypes = [c_int, _D, _D, c_int, _D]
        L.or_renorm.argtypes = [_D, c_int, c_int, _D]
        L.or_two_sum.argtypes = [dbl, dbl, _D, _D]
        L.or_two_prod.argtypes = [dbl, dbl, _D, _D]
        L.or_cmul.argtypes = [c_int, _D, _D, _D]
        L.or_cdiv.argtypes = [c_int, _D, _D, _D]
        L.or_spmv.argtypes = [i64, _I32, _I32, _D, c_int, c_int, _D, _D]
        L.or_spmv_h.argtypes = [i64, _I32, _I32, _D, c_int, c_int, _D, _D]
        L.or_csr_conj_transpose.argtypes = [i64, _I32, _I32, _D, c_int, c_int, _I32, _I32, _D]
        L.or_ilu0.argtypes = [i64, _I32, _I32, _D, c_int, c_int, _D, _I64]
        L.or_ilu0.restype = c_int
        L.or_ilu0_apply.argtypes = [i64, _I32, _I32, _D, c_int, c_int, c_int, _D, _D]
        L.or_ilu0_apply_h.argtypes = [i64, _I32, _I32, _D, c_int, c_int, c_int, _D, _D]
        L.or_dot.argtypes = [i64, c_int, c_int, _D, _D, _D]
        L.or_residual.argtypes = [i64, _I32, _I32, _D, c_int, _D, c_int, _D, c_int, _D]
        L.or_krylov.argtypes = [c_int, i64, _I32, _I32, _D, c_int, c_int, c_int, _D, _D,
                                dbl, dbl, i64, _I64, _D, _D, _I64, _D, i64]
        L.or_krylov.restype = c_int
        L.or_krylov_with_factor.argtypes = [c_int, i64, _I32, _I32, _D, c_int, c_int, c_int, _D,
                                            _D, _D, dbl, dbl, i64, _I64, _D, _D, _I64, _D, i64]
        L.or_krylov_with_factor.restype = c_int
        L.or_greedy_color.argtypes = [i64, _I32, _I32, _I32]
        L.or_greedy_color.restype = i32
        L.or_color_perm.argtypes = [i64, _I32, i32, _I32]
        L.or_csr_permute.argtypes = [i64, _I32, _I32, _D, c_int, _I32, _I32, _I32, _D]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_D)


def _i32(a):
    return a.ctypes.data_as(_I32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _csr(rp, ci, val, C):
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    val = _f64(val).reshape(-1, C)
    return rp, ci, val


# ----------------------------------------------------------------- scalars
def add(x, y):
    x, y = _f64(x), _f64(y)
    z = np.zeros_like(x)
    lib().or_add(len(x), _d(x), _d(y), _d(z))
    return z


def mul(x, y):
    x, y = _f64(x), _f64(y)
    z = np.zeros_like(x)
    lib().or_mul(len(x), _d(x), _d(y), _d(z))
    return z


def mul_fp(x, a):
    x = _f64(x)
    z = np.zeros_like(x)
    lib().or_mul_fp(len(x), _d(x), float(a), _d(z))
    return z


def mul_k(x, y):
    """x (K limbs) times y (ky <= K limbs), result K limbs."""
    x, y = _f64(x), _f64(y)
    z = np.zeros_like(x)
    lib().or_mul_k(len(x), _d(x), _d(y), len(y), _d(z))
    return z


def div_k(x, y):
    """x (K limbs) divided by y (ky <= K limbs), result K limbs."""
    x, y = _f64(x), _f64(y)
    z = np.zeros_like(x)
    lib().or_div_k(len(x), _d(x), _d(y), len(y), _d(z))
    return z


def renorm(t, K):
    t = _f64(t)
    z = np.zeros(K)
    lib().or_renorm(_d(t), len(t), K, _d(z))
    return z


def two_sum(a, b):
    s, e = ctypes.c_double(), ctypes.c_double()
    lib().or_two_sum(float(a), float(b), ctypes.byref(s), ctypes.byref(e))
    return s.value, e.value


def two_prod(a, b):
    p, e = ctypes.c_double(), ctypes.c_double()
    lib().or_two_prod(float(a), float(b), ctypes.byref(p), ctypes.byref(e))
    return p.value, e.value


def cmul(s, x):
    """Complex product of (2, K) arrays [re limbs, im limbs]."""
    s, x = _f64(s), _f64(x)
    K = s.shape[-1]
    z = np.zeros((2, K))
    lib().or_cmul(K, _d(s), _d(x), _d(z))
    return z


def cdiv(x, d):
    x, d = _f64(x), _f64(d)
    K = x.shape[-1]
    z = np.zeros((2, K))
    lib().or_cdiv(K, _d(x), _d(d), _d(z))
    return z


# ------------------------------------------------------------------ sparse
def spmv(rp, ci, val, x, trans=False):
    """y = A x (or A^H x).  x: float64 (n, C, K)."""
    x = _f64(x)
    n, C, K = x.shape
    rp, ci, val = _csr(rp, ci, val, C)
    y = np.zeros_like(x)
    f = lib().or_spmv_h if trans else lib().or_spmv
    f(n, _i32(rp), _i32(ci), _d(val), C, K, _d(x), _d(y))
    return y


def conj_transpose(rp, ci, val, C, kv=1):
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    val = _f64(val)
    n = len(rp) - 1
    nnz = int(rp[-1])
    trp = np.zeros(n + 1, np.int32)
    tci = np.zeros(max(nnz, 1), np.int32)
    tval = np.zeros(max(nnz, 1) * C * kv)
    lib().or_csr_conj_transpose(n, _i32(rp), _i32(ci), _d(val), C, kv, _i32(trp), _i32(tci),
                                _d(tval))
    return trp, tci[:nnz], tval[: nnz * C * kv].reshape((nnz, C, kv) if kv > 1 else (nnz, C))


def ilu0(rp, ci, val, C, kf):
    """ILU(0) factor in kf limbs: returns (status, bad_row, f[nnz, C, kf])."""
    rp, ci, val = _csr(rp, ci, val, C)
    n = len(rp) - 1
    nnz = int(rp[-1])
    f = np.zeros((max(nnz, 1), C, kf))
    bad = ctypes.c_int64(-1)
    st = lib().or_ilu0(n, _i32(rp), _i32(ci), _d(val), C, kf, _d(f), ctypes.byref(bad))
    return st, bad.value, f[:nnz]


def ilu0_apply(rp, ci, f, r, conj_trans=False):
    """z = (L U)^{-1} r (or (L U)^{-H} r); f: float64 (nnz, C, kf)."""
    r = _f64(r)
    f = _f64(f)
    n, C, K = r.shape
    kf = f.shape[-1]
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    z = np.zeros_like(r)
    fn = lib().or_ilu0_apply_h if conj_trans else lib().or_ilu0_apply
    fn(n, _i32(rp), _i32(ci), _d(f), C, kf, K, _d(r), _d(z))
    return z


def dot(a, b):
    """<a, b> = sum conj(a_i) b_i in the working precision: (C, K)."""
    a, b = _f64(a), _f64(b)
    n, C, K = a.shape
    out = np.zeros((C, K))
    lib().or_dot(n, C, K, _d(a), _d(b), _d(out))
    return out


def residual(rp, ci, val, b, x):
    """r = b - A x computed without rounding (a long accumulator), each
    component then rounded to binary64: float64 (n, C).  b: (n, C, kb),
    x: (n, C, kx), any limb counts."""
    b, x = _f64(b), _f64(x)
    n, C, kb = b.shape
    kx = x.shape[2]
    if x.shape[:2] != (n, C):
        raise ValueError("b and x must have the same (n, C)")
    rp, ci, val = _csr(rp, ci, val, C)
    r = np.zeros((n, C))
    lib().or_residual(n, _i32(rp), _i32(ci), _d(val), C, _d(b), kb, _d(x), kx, _d(r))
    return r


def true_relres(rp, ci, val, b, x):
    """||b - A x||_2 / ||b||_2 with the residual computed exactly (see
    residual); the norms are formed in binary64 from the rounded
    components."""
    r = residual(rp, ci, val, b, x)
    zero = np.zeros((b.shape[0], b.shape[1], 1))
    bb = residual(rp, ci, val, b, zero)
    nb = float(np.sqrt(np.sum(bb * bb)))
    nr = float(np.sqrt(np.sum(r * r)))
    return nr / nb if nb > 0 else nr


def krylov(method, rp, ci, val, b, kf, tol_rel, tol_abs=0.0, max_iter=1000, x0=None,
           hist_len=0, factor=None):
    """Run one of the four methods.  b: (n, C, K).  Returns a dict.  With
    ``factor`` (float64 [nnz, C, kf] in A's pattern) that factor is used
    instead of computing ILU(0)."""
    b = _f64(b)
    n, C, K = b.shape
    rp, ci, val = _csr(rp, ci, val, C)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    iters = ctypes.c_int64(0)
    rr = ctypes.c_double(0)
    rt = ctypes.c_double(0)
    bad = ctypes.c_int64(-1)
    hist = np.zeros(max(hist_len, 1))
    if factor is not None:
        f = _f64(np.asarray(factor, dtype=np.float64).reshape(len(ci), C, kf))
        st = lib().or_krylov_with_factor(METHODS[method], n, _i32(rp), _i32(ci), _d(val), C, K,
                                         kf, _d(f), _d(b), _d(x), float(tol_rel),
                                         float(tol_abs), int(max_iter), ctypes.byref(iters),
                                         ctypes.byref(rr), ctypes.byref(rt), ctypes.byref(bad),
                                         _d(hist), hist_len)
        return {"status": st, "x": x, "iters": iters.value, "relres_recursive": rr.value,
                "relres_true": rt.value, "bad_row": bad.value,
                "hist": hist[: min(hist_len, iters.value)]}
    st = lib().or_krylov(METHODS[method], n, _i32(rp), _i32(ci), _d(val), C, K, kf, _d(b),
                         _d(x), float(tol_rel), float(tol_abs), int(max_iter),
                         ctypes.byref(iters), ctypes.byref(rr), ctypes.byref(rt),
                         ctypes.byref(bad), _d(hist), hist_len)
    return {"status": st, "x": x, "iters": iters.value, "relres_recursive": rr.value,
            "relres_true": rt.value, "bad_row": bad.value,
            "hist": hist[: min(hist_len, iters.value)]}


# ------------------------------------------------- multicolour ordering
# A labelled variant beyond the paper's method (its Section 5 leaves the
# parallelisation of ILU(0) to future work): ILU(0) of P A P^T for an
# ordering P by colours.


def greedy_color(rp, ci):
    """Greedy colouring of the graph of A + A^T in natural order (vertex i
    takes the smallest colour absent from its neighbours j < i): returns
    (color int32[n], number of colours)."""
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    n = len(rp) - 1
    color = np.zeros(max(n, 1), dtype=np.int32)
    ncol = lib().or_greedy_color(n, _i32(rp), _i32(ci), _i32(color))
    return color[:n], int(ncol)


def color_perm(color, ncol):
    """perm[k] = the row placed at position k: ascending colour, original
    order within a colour."""
    color = np.ascontiguousarray(color, dtype=np.int32)
    n = len(color)
    perm = np.zeros(max(n, 1), dtype=np.int32)
    lib().or_color_perm(n, _i32(color), int(ncol), _i32(perm))
    return perm[:n]


def multicolor_perm(rp, ci):
    """The multicolour ordering of A's pattern: (perm, number of colours)."""
    color, ncol = greedy_color(rp, ci)
    return color_perm(color, ncol), ncol


def csr_permute(rp, ci, val, C, perm):
    """B = P A P^T (b_kl = a_{perm[k], perm[l]}), columns ascending per row:
    (brp, bci, bval[nnz, C])."""
    rp, ci, val = _csr(rp, ci, val, C)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    n = len(rp) - 1
    nnz = int(rp[-1])
    brp = np.zeros(n + 1, dtype=np.int32)
    bci = np.zeros(max(nnz, 1), dtype=np.int32)
    bval = np.zeros((max(nnz, 1), C))
    lib().or_csr_permute(n, _i32(rp), _i32(ci), _d(val), C, _i32(perm), _i32(brp), _i32(bci),
                         _d(bval))
    return brp, bci[:nnz], bval[:nnz]
