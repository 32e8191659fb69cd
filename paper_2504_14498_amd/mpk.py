"""Thin Python binding of libmpk.so (the C-ABI in include/mpk.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  torch supplies device memory and streams.  Vectors are float64
CUDA tensors of shape (n, C, K): C = 1 real / 2 complex, K limbs (1 D, 2 DD,
3 TD, 4 QD), leading limb first.  There is no CPU fallback: if the library
is not built, loading raises.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpk.so")

METHODS = {"bicg": 0, "cgs": 1, "bicgstab": 2, "gpbicg": 3}
STATUS = {0: "ok", 1: "not_converged", 2: "breakdown", -1: "einval", -2: "edevice",
          -3: "eworkspace", -4: "ezero_pivot", -5: "eno_diag", -6: "eunsupported",
          -7: "enonfinite", -8: "epattern", -9: "ewatchdog"}
ILU0_ADJOINT = 1


class MpkError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__("%s: %s (%d)" % (what, _lib().mpk_status_str(status).decode(), status))


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class _Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("bad_row", ctypes.c_int64),
                ("status", ctypes.c_int32), ("relres_recursive", ctypes.c_double),
                ("relres_true", ctypes.c_double), ("setup_ms", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("res_history", ctypes.c_void_p),
                ("res_history_len", ctypes.c_int64)]


_L = None

# (name, restype, argtypes) of every exported entry point
_P, _I, _S, _D, _I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_double, ctypes.c_int64
_CSRP = ctypes.POINTER(_Csr)
_INFOP = ctypes.POINTER(_Info)
SIGNATURES = [
    ("mpk_status_str", ctypes.c_char_p, [_I]),
    ("mpk_version", _I, []),
    ("mpk_spmv_workspace_bytes", _S, [_CSRP, _I, _I]),
    ("mpk_dcsr_spmv", _I, [_I, _CSRP, _I, _P, _P, _P, _S, _P]),
    ("mpk_zcsr_spmv", _I, [_I, _CSRP, _I, _P, _P, _P, _S, _P]),
    ("mpk_ilu0_workspace_bytes", _S, [_CSRP, _I, _I, _I]),
    ("mpk_dilu0_factor", _I, [_I, _CSRP, _I, _P, _S, ctypes.POINTER(_P), _INFOP, _P]),
    ("mpk_zilu0_factor", _I, [_I, _CSRP, _I, _P, _S, ctypes.POINTER(_P), _INFOP, _P]),
    ("mpk_dilu0_apply", _I, [_P, _I, _I, _P, _P, _P]),
    ("mpk_zilu0_apply", _I, [_P, _I, _I, _P, _P, _P]),
    ("mpk_ilu0_destroy", None, [_P]),
    ("mpk_krylov_workspace_bytes", _S, [_I, _I, _I, _CSRP, _I]),
    ("mpk_dkrylov_solve", _I, [_I, _I, _I, _D, _D, _I64, _CSRP, _P, _P, _P, _S, _INFOP, _P]),
    ("mpk_zkrylov_solve", _I, [_I, _I, _I, _D, _D, _I64, _CSRP, _P, _P, _P, _S, _INFOP, _P]),
    ("mpk_krylov_batched_workspace_bytes", _S, [_I, _I, _I, ctypes.c_int32, _CSRP]),
    ("mpk_dkrylov_solve_batched", _I, [_I, _I, _I, _D, _D, _I64, ctypes.c_int32, _CSRP,
                                       ctypes.POINTER(_P), ctypes.POINTER(_P), _P, _S, _INFOP,
                                       ctypes.c_char_p, _P]),
    ("mpk_krylov_precond_workspace_bytes", _S, [_I, _I, _CSRP, _I]),
    ("mpk_dkrylov_solve_precond", _I, [_I, _I, _P, _D, _D, _I64, _CSRP, _P, _P, _P, _S, _INFOP,
                                       _P]),
    ("mpk_zkrylov_solve_precond", _I, [_I, _I, _P, _D, _D, _I64, _CSRP, _P, _P, _P, _S, _INFOP,
                                       _P]),
    ("mpk_gnn_param_count", _I64, []),
    ("mpk_gnn_init", _I, [_P, ctypes.c_uint64, _P]),
    ("mpk_gnn_graph_bytes", _S, [_CSRP]),
    ("mpk_gnn_graph_setup", _I, [_CSRP, _P, _P, _S, _P]),
    ("mpk_gnn_workspace_bytes", _S, [_CSRP]),
    ("mpk_gnn_forward", _I, [_CSRP, _P, _P, _P, _P, _S, _P]),
    ("mpk_gnn_backward", _I, [_CSRP, _P, _P, _P, _P, _P, _S, _P]),
    ("mpk_gnn_saved", _I, [_CSRP, _P, _S, _I, _I, _P, _P]),
    ("mpk_gnn_loss_workspace_bytes", _S, [_CSRP, ctypes.c_int32]),
    ("mpk_gnn_factor_loss", _I, [_CSRP, _P, _P, _P, ctypes.c_int32, _P, _P, _P, _P, _S, _P]),
    ("mpk_gnn_adam", _I, [_I64, _I64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                          ctypes.c_float, _P, _P, _P, _P, _P]),
    ("mpk_ilu0_correct", _I, [_P, _P, ctypes.POINTER(ctypes.c_int32), _P]),
    ("mpk_spmv_set_lanes", _I, [_CSRP, _I]),
    ("mpk_spmv_tune", _I, [_I, _CSRP, _I, _P, _P, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_double),
                           _P]),
    ("mpk_dot_workspace_bytes", _S, [_I64, _I, _I]),
    ("mpk_dot", _I, [_I, _I, _I64, _P, _P, _P, _P, _S, _P]),
    ("mpk_dot_noalloc_max_elements", _S, [_I, _I]),
    ("mpk_dot_noalloc", _I, [_I, _I, _I64, _P, _P, _P, _P]),
    ("mpk_dcsr_residual", _I, [_I, _CSRP, _P, _P, _P, _P]),
    ("mpk_zcsr_residual", _I, [_I, _CSRP, _P, _P, _P, _P]),
    ("mpk_multicolor_order", _I, [_CSRP, _P, ctypes.POINTER(ctypes.c_int32), _P]),
    ("mpk_csr_permute_workspace_bytes", _S, [_I64]),
    ("mpk_dcsr_permute", _I, [_CSRP, _P, _P, _P, _P, _P, _S, _P]),
    ("mpk_zcsr_permute", _I, [_CSRP, _P, _P, _P, _P, _P, _S, _P]),
    ("mpk_vec_permute", _I, [_I, _I, _I64, _P, _I, _P, _P, _P]),
]


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmpk.so is not built (run __graft_entry__.build() or "
                              "python paper_2504_14498_amd/build.py): " + LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _L = L
    return _L


def library():
    """The loaded ctypes library (raises if it is not built)."""
    return _lib()


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check(st, what):
    if st < 0:
        raise MpkError(st, what)
    return st


def _workspace(nbytes, device):
    # 256-byte aligned device buffer owned by torch
    nbytes = max(int(nbytes), 1)
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off, nbytes


class Csr:
    """CSR matrix on the device: row_ptr/col_idx int32, val float64 (nnz,)
    real or (nnz, 2) complex."""

    def __init__(self, row_ptr, col_idx, val, device="cuda"):
        def dev(a, dtype):
            if not isinstance(a, torch.Tensor):
                a = torch.as_tensor(np.asarray(a))
            return a.to(device=device, dtype=dtype).contiguous()
        self.row_ptr = dev(row_ptr, torch.int32)
        self.col_idx = dev(col_idx, torch.int32)
        v = dev(val, torch.float64)
        self.is_complex = v.dim() == 2
        self.val = v.contiguous()
        self.n = self.row_ptr.numel() - 1
        self.nnz = self.col_idx.numel()
        self.device = self.val.device
        self.c = _Csr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                      self.val.data_ptr())

    @property
    def C(self):
        return 2 if self.is_complex else 1

    @classmethod
    def from_problem(cls, p, device="cuda"):
        return cls(p.row_ptr, p.col_idx, p.val, device)


def _vec_check(A, v, name):
    if v.dtype != torch.float64 or not v.is_cuda or v.dim() != 3 or v.shape[0] != A.n \
            or v.shape[1] != A.C or not v.is_contiguous():
        raise ValueError("%s must be a contiguous float64 CUDA tensor of shape (n, C, K)" % name)
    return v.shape[2]


def csr_spmv(A, x, y=None, trans=False, stream=None):
    """y = A x (or A^T x / A^H x)."""
    K = _vec_check(A, x, "x")
    if y is None:
        y = torch.empty_like(x)
    fn = _lib().mpk_zcsr_spmv if A.is_complex else _lib().mpk_dcsr_spmv
    ws = None
    ws_ptr, ws_n = 0, 0
    if trans:
        nb = _lib().mpk_spmv_workspace_bytes(ctypes.byref(A.c), int(A.is_complex), 1)
        ws, ws_ptr, ws_n = _workspace(nb, A.device)
    _check(fn(K, ctypes.byref(A.c), int(trans), _ptr(x), _ptr(y), ctypes.c_void_p(ws_ptr), ws_n,
              _stream(stream)), "csr_spmv")
    return y


def csr_residual(A, b, x, r=None, stream=None):
    """r = b - A x in the vectors' precision (the solvers' true residual)."""
    K = _vec_check(A, b, "b")
    if _vec_check(A, x, "x") != K:
        raise ValueError("b and x must have the same precision")
    if r is None:
        r = torch.empty_like(b)
    fn = _lib().mpk_zcsr_residual if A.is_complex else _lib().mpk_dcsr_residual
    _check(fn(K, ctypes.byref(A.c), _ptr(b), _ptr(x), _ptr(r), _stream(stream)), "csr_residual")
    return r


def spmv_set_lanes(A, lanes):
    """Lanes per row of A's SpMV (1, 2, 4, 8, 16; 0 = forget)."""
    _check(_lib().mpk_spmv_set_lanes(ctypes.byref(A.c), int(lanes)), "spmv_set_lanes")


def spmv_tune(A, x, y=None, stream=None):
    """Time each lanes-per-row choice for A with vector x and keep the
    fastest; returns (lanes, ms per launch)."""
    n, C, K = x.shape
    if y is None:
        y = torch.empty_like(x)
    lanes = ctypes.c_int(0)
    ms = ctypes.c_double(0)
    _check(_lib().mpk_spmv_tune(K, ctypes.byref(A.c), int(C == 2), _ptr(x), _ptr(y),
                                ctypes.byref(lanes), ctypes.byref(ms), _stream(stream)),
           "spmv_tune")
    return lanes.value, ms.value


class Ilu0:
    """ILU(0) factor held in a torch-owned device workspace."""

    def __init__(self, A, handle, ws, fprec, adjoint):
        self.A = A
        self.handle = handle
        self._ws = ws
        self.fprec = fprec
        self.adjoint = adjoint

    def __del__(self):
        if getattr(self, "handle", None) and _L is not None:
            _L.mpk_ilu0_destroy(self.handle)
            self.handle = None


def ilu0_factor(A, fprec=1, adjoint=False, vprec=None, stream=None):
    """ILU(0) factorisation in binary64 (fprec=1) or with 2, 3 or 4 limbs
    (double-, triple-, quad-word).
    vprec: largest vector precision the factor will be applied with (sizes
    the on-chip blocks of the substitutions; default 4 = QD)."""
    flags = ILU0_ADJOINT if adjoint else 0
    if vprec is not None:
        flags |= int(vprec) << 4
    nb = _lib().mpk_ilu0_workspace_bytes(ctypes.byref(A.c), fprec, int(A.is_complex), flags)
    if nb == 0:
        raise ValueError("bad ILU(0) arguments")
    ws, ws_ptr, ws_n = _workspace(nb, A.device)
    h = ctypes.c_void_p()
    info = _Info()
    fn = _lib().mpk_zilu0_factor if A.is_complex else _lib().mpk_dilu0_factor
    st = fn(fprec, ctypes.byref(A.c), flags, ctypes.c_void_p(ws_ptr), ws_n, ctypes.byref(h),
            ctypes.byref(info), _stream(stream))
    if st < 0:
        e = MpkError(st, "ilu0_factor")
        e.bad_row = info.bad_row
        raise e
    return Ilu0(A, h, ws, fprec, adjoint)


def ilu0_apply(M, r, z=None, conj_trans=False, stream=None):
    """z = M^{-1} r (or M^{-H} r)."""
    K = _vec_check(M.A, r, "r")
    if z is None:
        z = torch.empty_like(r)
    fn = _lib().mpk_zilu0_apply if M.A.is_complex else _lib().mpk_dilu0_apply
    _check(fn(M.handle, K, int(conj_trans), _ptr(r), _ptr(z), _stream(stream)), "ilu0_apply")
    return z


def dot(a, b, stream=None):
    """<a, b> = sum conj(a_i) b_i in the working precision: tensor (C, K)."""
    n, C, K = a.shape
    out = torch.empty((C, K), dtype=torch.float64, device=a.device)
    nb = _lib().mpk_dot_workspace_bytes(n, int(C == 2), K)
    ws, ws_ptr, ws_n = _workspace(nb, a.device)
    _check(_lib().mpk_dot(K, int(C == 2), n, _ptr(a), _ptr(b), _ptr(out), ctypes.c_void_p(ws_ptr),
                          ws_n, _stream(stream)), "dot")
    return out


def dot_noalloc_max_elements(C, K):
    return _lib().mpk_dot_noalloc_max_elements(int(C == 2), K)


def dot_noalloc(a, b, out, stream=None):
    """<a, b> into the caller's out (C, K) with the library's fixed device
    scratch: the call itself allocates nothing."""
    n, C, K = a.shape
    _check(_lib().mpk_dot_noalloc(K, int(C == 2), n, _ptr(a), _ptr(b), _ptr(out),
                                  _stream(stream)), "dot_noalloc")
    return out


_SIDE = {}


def _side_stream(device):
    if device not in _SIDE:
        _SIDE[device] = torch.cuda.Stream(device=device)
    return _SIDE[device]


def krylov_workspace_bytes(method, A, vprec, fprec):
    return _lib().mpk_krylov_workspace_bytes(METHODS[method], vprec, fprec, ctypes.byref(A.c),
                                             int(A.is_complex))


def krylov_solve(method, A, b, x0=None, fprec=1, tol_rel=1e-25, tol_abs=0.0, max_iter=1000,
                 hist_len=0, workspace=None, graph=True):
    """Solve A x = b.  b: (n, C, K) float64 CUDA tensor; fprec 0 = no
    preconditioner, 1 = binary64 ILU(0), 2 = double-double ILU(0).
    Returns (x, info dict).  graph=True runs on a side stream so that each
    pass is replayed from a captured hipGraph."""
    K = _vec_check(A, b, "b")
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    nb = krylov_workspace_bytes(method, A, K, fprec)
    if nb == 0:
        raise ValueError("bad krylov_solve arguments")
    if workspace is None or workspace[2] < nb:
        workspace = _workspace(nb, A.device)
    ws, ws_ptr, ws_n = workspace
    hist = torch.zeros(max(hist_len, 1), dtype=torch.float64, device=A.device)
    info = _Info()
    info.res_history = hist.data_ptr() if hist_len > 0 else None
    info.res_history_len = hist_len
    fn = _lib().mpk_zkrylov_solve if A.is_complex else _lib().mpk_dkrylov_solve
    cur = torch.cuda.current_stream(A.device)
    s = _side_stream(A.device) if graph else cur
    if graph:
        s.wait_stream(cur)
    st = fn(METHODS[method], K, fprec, float(tol_rel), float(tol_abs), int(max_iter),
            ctypes.byref(A.c), _ptr(b), _ptr(x), ctypes.c_void_p(ws_ptr), ws_n, ctypes.byref(info),
            ctypes.c_void_p(s.cuda_stream))
    if graph:
        cur.wait_stream(s)
    if st < 0:
        e = MpkError(st, "krylov_solve")
        e.bad_row = info.bad_row
        raise e
    out = {"status": STATUS.get(st, st), "code": st, "iters": info.iters,
           "relres_recursive": info.relres_recursive, "relres_true": info.relres_true,
           "setup_ms": info.setup_ms, "solve_ms": info.solve_ms, "bad_row": info.bad_row,
           "hist": hist[: min(hist_len, info.iters)] if hist_len else None,
           "workspace": workspace}
    return x, out


def multicolor_order(A, stream=None):
    """Greedy colouring of A + A^T in natural order and the ordering by
    colour (a variant beyond the paper's method): returns (perm, number of
    colours), perm an int32 CUDA tensor with perm[k] = the row placed at k."""
    perm = torch.empty(A.n, dtype=torch.int32, device=A.device)
    ncol = ctypes.c_int32(0)
    _check(_lib().mpk_multicolor_order(ctypes.byref(A.c), _ptr(perm), ctypes.byref(ncol),
                                       _stream(stream)), "multicolor_order")
    return perm, ncol.value


def csr_permute(A, perm, stream=None):
    """B = P A P^T (b_kl = a_{perm[k], perm[l]}) as a new Csr."""
    rp = torch.empty(A.n + 1, dtype=torch.int32, device=A.device)
    ci = torch.empty(A.nnz, dtype=torch.int32, device=A.device)
    val = torch.empty_like(A.val)
    ws, ws_ptr, ws_n = _workspace(_lib().mpk_csr_permute_workspace_bytes(A.n), A.device)
    fn = _lib().mpk_zcsr_permute if A.is_complex else _lib().mpk_dcsr_permute
    _check(fn(ctypes.byref(A.c), _ptr(perm), _ptr(rp), _ptr(ci), _ptr(val),
              ctypes.c_void_p(ws_ptr), ws_n, _stream(stream)), "csr_permute")
    return Csr(rp, ci, val, A.device)


def vec_permute(x, perm, inverse=False, out=None, stream=None):
    """y = P x (y[k] = x[perm[k]]) or, inverse, y = P^T x (y[perm[k]] = x[k])."""
    if x.dtype != torch.float64 or not x.is_cuda or x.dim() != 3 or not x.is_contiguous():
        raise ValueError("x must be a contiguous float64 CUDA tensor of shape (n, C, K)")
    n, C, K = x.shape
    y = torch.empty_like(x) if out is None else out
    _check(_lib().mpk_vec_permute(K, int(C == 2), n, _ptr(perm), int(bool(inverse)), _ptr(x),
                                  _ptr(y), _stream(stream)), "vec_permute")
    return y


def krylov_solve_multicolor(method, A, b, fprec=1, tol_rel=1e-25, tol_abs=0.0, max_iter=1000,
                            hist_len=0, workspace=None, graph=True):
    """The multicolour variant: order A by colours, solve P A P^T y = P b
    with ILU(0) of P A P^T, return x = P^T y.  Calls, in order,
    multicolor_order, csr_permute, vec_permute, krylov_solve and
    vec_permute; info gains "ncolors"."""
    cur = torch.cuda.current_stream(A.device)
    perm, ncol = multicolor_order(A, stream=cur)
    B = csr_permute(A, perm, stream=cur)
    bp = vec_permute(b, perm, stream=cur)
    y, info = krylov_solve(method, B, bp, fprec=fprec, tol_rel=tol_rel, tol_abs=tol_abs,
                           max_iter=max_iter, hist_len=hist_len, workspace=workspace, graph=graph)
    x = vec_permute(y, perm, inverse=True, stream=cur)
    info["ncolors"] = ncol
    info["perm"] = perm
    info["B"] = B
    return x, info


def krylov_solve_batched(mats, bs, x0s=None, method="bicgstab", fprec=1, tol_rel=1e-25,
                         tol_abs=0.0, max_iter=1000, schedule=None, workspace=None, stream=None):
    """Solve len(mats) independent real systems in one persistent launch.
    mats: list of Csr; bs: list of (n, 1, K) float64 CUDA tensors.  Returns
    (list of x, list of info dicts, overall status)."""
    nsys = len(mats)
    K = bs[0].shape[2]
    for A, b in zip(mats, bs):
        if A.is_complex or _vec_check(A, b, "b") != K:
            raise ValueError("batched systems must be real with a common precision")
    xs = [torch.zeros_like(b) if x0s is None else x0s[q].clone() for q, b in enumerate(bs)]
    arr = (_Csr * nsys)(*[A.c for A in mats])
    nb = _lib().mpk_krylov_batched_workspace_bytes(METHODS[method], K, fprec, nsys, arr)
    if nb == 0:
        raise ValueError("bad batched arguments")
    if workspace is None or workspace[2] < nb:
        workspace = _workspace(nb, mats[0].device)
    ws, ws_ptr, ws_n = workspace
    bp = (_P * nsys)(*[b.data_ptr() for b in bs])
    xp = (_P * nsys)(*[x.data_ptr() for x in xs])
    infos = (_Info * nsys)()
    st = _lib().mpk_dkrylov_solve_batched(METHODS[method], K, fprec, float(tol_rel),
                                          float(tol_abs), int(max_iter), nsys, arr, bp, xp,
                                          ctypes.c_void_p(ws_ptr), ws_n, infos,
                                          schedule.encode() if schedule else None,
                                          _stream(stream))
    out = [{"status": STATUS.get(i.status, i.status), "code": i.status, "iters": i.iters,
            "relres_recursive": i.relres_recursive, "relres_true": i.relres_true,
            "bad_row": i.bad_row, "setup_ms": i.setup_ms, "solve_ms": i.solve_ms}
           for i in infos]
    if st == -1 or st == -3:
        raise MpkError(st, "krylov_solve_batched")
    return xs, out, STATUS.get(st, st), workspace


def krylov_solve_precond(method, A, M, b, x0=None, tol_rel=1e-25, tol_abs=0.0, max_iter=1000,
                         hist_len=0, workspace=None, graph=True):
    """Solve A x = b preconditioned by an existing factor M (an Ilu0 of this
    A, possibly corrected by ilu0_correct).  Returns (x, info dict)."""
    K = _vec_check(A, b, "b")
    if M.A is not A:
        raise ValueError("the factor belongs to another matrix")
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    nb = _lib().mpk_krylov_precond_workspace_bytes(METHODS[method], K, ctypes.byref(A.c),
                                                   int(A.is_complex))
    if nb == 0:
        raise ValueError("bad krylov_solve_precond arguments")
    if workspace is None or workspace[2] < nb:
        workspace = _workspace(nb, A.device)
    ws, ws_ptr, ws_n = workspace
    hist = torch.zeros(max(hist_len, 1), dtype=torch.float64, device=A.device)
    info = _Info()
    info.res_history = hist.data_ptr() if hist_len > 0 else None
    info.res_history_len = hist_len
    fn = _lib().mpk_zkrylov_solve_precond if A.is_complex else _lib().mpk_dkrylov_solve_precond
    cur = torch.cuda.current_stream(A.device)
    s = _side_stream(A.device) if graph else cur
    if graph:
        s.wait_stream(cur)
    st = fn(METHODS[method], K, M.handle, float(tol_rel), float(tol_abs), int(max_iter),
            ctypes.byref(A.c), _ptr(b), _ptr(x), ctypes.c_void_p(ws_ptr), ws_n, ctypes.byref(info),
            ctypes.c_void_p(s.cuda_stream))
    if graph:
        cur.wait_stream(s)
    if st < 0:
        raise MpkError(st, "krylov_solve_precond")
    out = {"status": STATUS.get(st, st), "code": st, "iters": info.iters,
           "relres_recursive": info.relres_recursive, "relres_true": info.relres_true,
           "setup_ms": info.setup_ms, "solve_ms": info.solve_ms, "bad_row": info.bad_row,
           "hist": hist[: min(hist_len, info.iters)] if hist_len else None,
           "workspace": workspace}
    return x, out


# ----------------------------------------------------- learned correction

def gnn_param_count():
    return int(_lib().mpk_gnn_param_count())


def gnn_init(seed, device="cuda", stream=None):
    """Initial float32 parameter vector (decoder zero: delta = 0)."""
    p = torch.empty(gnn_param_count(), dtype=torch.float32, device=device)
    _check(_lib().mpk_gnn_init(_ptr(p), int(seed), _stream(stream)), "gnn_init")
    return p


class GnnGraph:
    """Graph data of one matrix (edge rows, transposed pattern, network
    inputs from A and its plain binary64 factor M)."""

    def __init__(self, A, M, stream=None):
        if A.is_complex or M.fprec != 1:
            raise ValueError("the learned correction needs a real matrix and a binary64 factor")
        nb = _lib().mpk_gnn_graph_bytes(ctypes.byref(A.c))
        self._buf, self.ptr, self.nbytes = _workspace(nb, A.device)
        self.A = A
        _check(_lib().mpk_gnn_graph_setup(ctypes.byref(A.c), M.handle, ctypes.c_void_p(self.ptr),
                                          self.nbytes, _stream(stream)), "gnn_graph_setup")


def gnn_workspace(A):
    return _workspace(_lib().mpk_gnn_workspace_bytes(ctypes.byref(A.c)), A.device)


def gnn_forward(G, params, delta=None, workspace=None, stream=None):
    """delta[nnz] (float32) predicted for G's matrix; returns (delta, ws)."""
    A = G.A
    if delta is None:
        delta = torch.empty(A.nnz, dtype=torch.float32, device=A.device)
    if workspace is None:
        workspace = gnn_workspace(A)
    _, wp, wn = workspace
    _check(_lib().mpk_gnn_forward(ctypes.byref(A.c), ctypes.c_void_p(G.ptr), _ptr(params),
                                  _ptr(delta), ctypes.c_void_p(wp), wn, _stream(stream)),
           "gnn_forward")
    return delta, workspace


def gnn_backward(G, params, ddelta, workspace, dparams=None, stream=None):
    """Parameter gradient of sum(ddelta * delta) for the last forward in
    workspace."""
    A = G.A
    if dparams is None:
        dparams = torch.empty_like(params)
    _, wp, wn = workspace
    _check(_lib().mpk_gnn_backward(ctypes.byref(A.c), ctypes.c_void_p(G.ptr), _ptr(params),
                                   _ptr(ddelta), _ptr(dparams), ctypes.c_void_p(wp), wn,
                                   _stream(stream)), "gnn_backward")
    return dparams


GNN_SAVED = {"h": 0, "e": 1, "m": 2, "g": 3, "r": 4}


def gnn_saved(G, workspace, which, layer, stream=None):
    """A stored activation of the last forward in workspace, as int16
    (bfloat16 bit patterns) of shape (rows, 32)."""
    A = G.A
    rows = A.nnz if which in ("e", "m") else A.n
    out = torch.empty((rows, 32), dtype=torch.int16, device=A.device)
    _, wp, wn = workspace
    _check(_lib().mpk_gnn_saved(ctypes.byref(A.c), ctypes.c_void_p(wp), wn, GNN_SAVED[which],
                                int(layer), _ptr(out), _stream(stream)), "gnn_saved")
    return out


def gnn_factor_loss(G, M, delta, probes, grad=True, workspace=None, stream=None):
    """(loss (device float64 scalar tensor), d loss / d delta or None, ws).
    probes: float64 CUDA tensor (P, n)."""
    A = G.A
    P = probes.shape[0]
    if probes.dtype != torch.float64 or probes.shape[1] != A.n or not probes.is_contiguous():
        raise ValueError("probes must be a contiguous float64 (P, n) tensor")
    nb = _lib().mpk_gnn_loss_workspace_bytes(ctypes.byref(A.c), P)
    if workspace is None or workspace[2] < nb:
        workspace = _workspace(nb, A.device)
    _, wp, wn = workspace
    loss = torch.empty((), dtype=torch.float64, device=A.device)
    gd = torch.empty(A.nnz, dtype=torch.float32, device=A.device) if grad else None
    _check(_lib().mpk_gnn_factor_loss(ctypes.byref(A.c), M.handle, ctypes.c_void_p(G.ptr),
                                      _ptr(delta), P, _ptr(probes), _ptr(loss), _ptr(gd),
                                      ctypes.c_void_p(wp), wn, _stream(stream)),
           "gnn_factor_loss")
    return loss, gd, workspace


def gnn_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """In-place Adam step on params (m, v: float32 state of the same size)."""
    _check(_lib().mpk_gnn_adam(params.numel(), int(step), float(lr), float(beta1), float(beta2),
                               float(eps), _ptr(params), _ptr(grad), _ptr(m), _ptr(v),
                               _stream(stream)), "gnn_adam")


def ilu0_correct(M, delta, stream=None):
    """Apply the correction to M in place; returns True if the guards
    rejected it (M unchanged)."""
    fb = ctypes.c_int32(0)
    _check(_lib().mpk_ilu0_correct(M.handle, _ptr(delta), ctypes.byref(fb), _stream(stream)),
           "ilu0_correct")
    return bool(fb.value)
