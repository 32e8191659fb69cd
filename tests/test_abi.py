"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/mpk.h, and rejects invalid arguments before any device
work (so these calls are safe on a host without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2504_14498_amd import mpk
    return mpk.library()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mpk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpk_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_2504_14498_amd import mpk
    bound = {name for name, _, _ in mpk.SIGNATURES}
    assert set(declared_functions()) <= bound


def test_status_strings(lib):
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6, -7, -8, -9):
        s = lib.mpk_status_str(code).decode()
        assert s and s != "unknown status"
    assert lib.mpk_version() >= 100


def _csr(n, nnz, rp=1, ci=1, val=1):
    from paper_2504_14498_amd import mpk
    return mpk._Csr(n, nnz, rp, ci, val)


def test_invalid_arguments_rejected_before_device_work(lib):
    from paper_2504_14498_amd import mpk
    info = mpk._Info()
    ws = ctypes.c_void_p(256)
    # null matrix
    assert lib.mpk_dkrylov_solve(2, 2, 1, 1e-25, 0.0, 10, None, ctypes.c_void_p(8),
                                 ctypes.c_void_p(8), ws, 1 << 30, ctypes.byref(info), None) == -1
    # n <= 0, nnz < n, null pointers
    for A in (_csr(0, 0), _csr(4, 3), _csr(4, 4, rp=0), _csr(4, 4, ci=0), _csr(4, 4, val=0)):
        assert lib.mpk_dkrylov_solve(2, 2, 1, 1e-25, 0.0, 10, ctypes.byref(A), ctypes.c_void_p(8),
                                     ctypes.c_void_p(8), ws, 1 << 30, ctypes.byref(info),
                                     None) == -1
    A = _csr(4, 4)
    # bad method / precision / factor precision above the vector precision
    assert lib.mpk_dkrylov_solve(7, 2, 1, 1e-25, 0.0, 10, ctypes.byref(A), ctypes.c_void_p(8),
                                 ctypes.c_void_p(8), ws, 1 << 30, None, None) == -1
    assert lib.mpk_dkrylov_solve(2, 5, 1, 1e-25, 0.0, 10, ctypes.byref(A), ctypes.c_void_p(8),
                                 ctypes.c_void_p(8), ws, 1 << 30, None, None) == -1
    assert lib.mpk_dkrylov_solve(2, 1, 2, 1e-25, 0.0, 10, ctypes.byref(A), ctypes.c_void_p(8),
                                 ctypes.c_void_p(8), ws, 1 << 30, None, None) == -1
    assert lib.mpk_dkrylov_solve(2, 2, 3, 1e-25, 0.0, 10, ctypes.byref(A), ctypes.c_void_p(8),
                                 ctypes.c_void_p(8), ws, 1 << 30, None, None) == -1
    # negative tolerance, NaN tolerance, negative max_iter
    for tol, mi in ((-1.0, 10), (float("nan"), 10), (1e-25, -1)):
        assert lib.mpk_dkrylov_solve(2, 2, 1, tol, 0.0, mi, ctypes.byref(A), ctypes.c_void_p(8),
                                     ctypes.c_void_p(8), ws, 1 << 30, None, None) == -1
    # workspace missing, misaligned, too small
    need = lib.mpk_krylov_workspace_bytes(2, 2, 1, ctypes.byref(A), 0)
    assert need > 0
    assert lib.mpk_dkrylov_solve(2, 2, 1, 1e-25, 0.0, 10, ctypes.byref(A), ctypes.c_void_p(8),
                                 ctypes.c_void_p(8), None, need, None, None) == -3
    assert lib.mpk_dkrylov_solve(2, 2, 1, 1e-25, 0.0, 10, ctypes.byref(A), ctypes.c_void_p(8),
                                 ctypes.c_void_p(8), ctypes.c_void_p(264), need, None, None) == -3
    assert lib.mpk_dkrylov_solve(2, 2, 1, 1e-25, 0.0, 10, ctypes.byref(A), ctypes.c_void_p(8),
                                 ctypes.c_void_p(8), ws, need - 1, None, None) == -3
    # ILU(0): factor precision D..QD, not above the declared vector precision
    h = ctypes.c_void_p()
    assert lib.mpk_dilu0_factor(5, ctypes.byref(A), 0, ws, 1 << 30, ctypes.byref(h), None,
                                None) == -1
    assert lib.mpk_dilu0_factor(0, ctypes.byref(A), 0, ws, 1 << 30, ctypes.byref(h), None,
                                None) == -1
    assert lib.mpk_dilu0_factor(3, ctypes.byref(A), 2 << 4, ws, 1 << 30, ctypes.byref(h), None,
                                None) == -1
    assert lib.mpk_dilu0_factor(1, ctypes.byref(A), 4, ws, 1 << 30, ctypes.byref(h), None,
                                None) == -1
    assert lib.mpk_dilu0_apply(None, 2, 0, ctypes.c_void_p(8), ctypes.c_void_p(8), None) == -1
    # SpMV: precision out of range, null vectors
    assert lib.mpk_dcsr_spmv(0, ctypes.byref(A), 0, ctypes.c_void_p(8), ctypes.c_void_p(8), None,
                             0, None) == -1
    assert lib.mpk_dcsr_spmv(2, ctypes.byref(A), 0, None, ctypes.c_void_p(8), None, 0, None) == -1
    assert lib.mpk_dot(2, 0, 0, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(8), ws,
                       1 << 20, None) == -1


def test_workspace_queries_scale(lib):
    from paper_2504_14498_amd import mpk
    small, big = _csr(1000, 5000), _csr(100000, 500000)
    for m in range(4):
        for vp in (1, 2, 3, 4):
            for fp in range(0, vp + 1):
                a = lib.mpk_krylov_workspace_bytes(m, vp, fp, ctypes.byref(small), 0)
                b = lib.mpk_krylov_workspace_bytes(m, vp, fp, ctypes.byref(big), 1)
                assert 0 < a < b
                # vectors alone: at least 8 vectors of n C K doubles
                assert b >= 8 * 100000 * 2 * vp * 8
    assert lib.mpk_krylov_workspace_bytes(9, 2, 1, ctypes.byref(small), 0) == 0
    assert lib.mpk_ilu0_workspace_bytes(ctypes.byref(small), 5, 0, 0) == 0
    # wider factors take more room
    assert 0 < lib.mpk_ilu0_workspace_bytes(ctypes.byref(small), 2, 0, 0) < \
        lib.mpk_ilu0_workspace_bytes(ctypes.byref(small), 4, 0, 0)
    assert lib.mpk_ilu0_workspace_bytes(ctypes.byref(small), 1, 0, 1) > \
        lib.mpk_ilu0_workspace_bytes(ctypes.byref(small), 1, 0, 0)
    assert lib.mpk_spmv_workspace_bytes(ctypes.byref(small), 0, 0) == 0
    assert lib.mpk_spmv_workspace_bytes(ctypes.byref(small), 1, 1) > 5000 * 16
    assert lib.mpk_dot_workspace_bytes(1000, 0, 2) >= 4 * 2 * 8


def test_noalloc_dot_limits(lib):
    """The inner product without workspace: its size limit is a pure host
    query, and sizes past it are rejected before any device work."""
    for C in (0, 1):
        for p in (1, 2, 3, 4):
            m = lib.mpk_dot_noalloc_max_elements(C, p)
            assert m == (1 << 19) // ((2 if C else 1) * p) * 256
            assert lib.mpk_dot_noalloc(p, C, m + 1, ctypes.c_void_p(8), ctypes.c_void_p(8),
                                       ctypes.c_void_p(8), None) == -3
    assert lib.mpk_dot_noalloc_max_elements(0, 5) == 0
    assert lib.mpk_dot_noalloc(2, 0, 0, ctypes.c_void_p(8), ctypes.c_void_p(8),
                               ctypes.c_void_p(8), None) == -1
    assert lib.mpk_dot_noalloc(2, 0, 10, None, ctypes.c_void_p(8), ctypes.c_void_p(8),
                               None) == -1


def test_ordering_arguments_rejected_before_device_work(lib):
    import ctypes as C
    n32 = C.c_int32(0)
    assert lib.mpk_multicolor_order(None, C.c_void_p(8), C.byref(n32), None) == -1
    A = _csr(4, 4)
    assert lib.mpk_multicolor_order(C.byref(A), None, C.byref(n32), None) == -1
    assert lib.mpk_multicolor_order(C.byref(A), C.c_void_p(8), None, None) == -1
    assert lib.mpk_csr_permute_workspace_bytes(0) == 0
    assert lib.mpk_csr_permute_workspace_bytes(1000) >= 4000
    for fn in (lib.mpk_dcsr_permute, lib.mpk_zcsr_permute):
        assert fn(None, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), C.c_void_p(8),
                  C.c_void_p(256), 1 << 20, None) == -1
        assert fn(C.byref(A), None, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8),
                  C.c_void_p(256), 1 << 20, None) == -1
        # missing, misaligned or short workspace
        for ws, nb in ((None, 1 << 20), (C.c_void_p(264), 1 << 20), (C.c_void_p(256), 8)):
            assert fn(C.byref(A), C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), C.c_void_p(8),
                      ws, nb, None) == -3
    # precision out of range, negative n, null arrays; n = 0 does nothing
    assert lib.mpk_vec_permute(0, 0, 4, C.c_void_p(8), 0, C.c_void_p(8), C.c_void_p(8), None) == -1
    assert lib.mpk_vec_permute(5, 0, 4, C.c_void_p(8), 0, C.c_void_p(8), C.c_void_p(8), None) == -1
    assert lib.mpk_vec_permute(2, 0, -1, C.c_void_p(8), 0, C.c_void_p(8), C.c_void_p(8), None) == -1
    assert lib.mpk_vec_permute(2, 0, 4, None, 0, C.c_void_p(8), C.c_void_p(8), None) == -1
    assert lib.mpk_vec_permute(2, 1, 0, None, 0, None, None, None) == 0
