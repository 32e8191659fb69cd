"""The paper-replication harness on MatrixMarket files written from the
repository's own generators (a real nonsymmetric convection-diffusion
matrix and a complex symmetric Helmholtz matrix stand in for the paper's
SuiteSparse matrices): every method x precision (DD, TD, QD) x variant (no
preconditioner, ILU(0) in the working precision, binary64 ILU(0)) runs
through the library and is checked against the oracle's solve of the same
system: same status, pass counts within max(3, 5%), and the GPU's x passes
the paper's stopping criterion on its exact residual."""
import numpy as np
import pytest

from paper_2504_14498_amd import mtx
from paper_2504_14498_amd import workloads as W
from paper_2504_14498_amd.replicate import EPS_A, EPS_R, paper_x, ratios, run_matrix, table

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_14498_amd import mpk
    mpk.library()
    return mpk


def complex_symmetric_helmholtz(m):
    """The 9-point shifted Helmholtz stencil is complex symmetric, as the
    paper's complex test matrix is."""
    return W.config3(m)


@pytest.mark.parametrize("which", ["real", "complex"])
def test_variant_grid_matches_oracle(lib, orc, tmp_path, which):
    src = W.config1(14) if which == "real" else complex_symmetric_helmholtz(11)
    f = tmp_path / ("%s.mtx" % which)
    mtx.write(f, src)
    p = mtx.read(f, name=which)
    bs = {K: orc.spmv(p.row_ptr, p.col_idx, p.val, paper_x(p.n, p.C, K)) for K in (2, 3, 4)}
    runs = run_matrix(p, rhs=lambda K: bs[K], keep_x=True)
    assert len(runs) == 3 * 4 * 3
    for r in runs:
        b = bs[r["K"]]
        ref = orc.krylov(r["method"], p.row_ptr, p.col_idx, p.val, b, kf=r["fprec"],
                         tol_rel=EPS_R, tol_abs=EPS_A, max_iter=3 * p.n)
        assert (r["status"] == "ok") == (ref["status"] == 0), (r["variant"], r["prec"])
        assert abs(r["iters"] - ref["iters"]) <= max(3, 0.05 * ref["iters"]), \
            (r["variant"], r["prec"], r["iters"], ref["iters"])
        if r["status"] == "ok":
            nb = np.sqrt(np.sum(b[:, :, 0] ** 2))
            rel = orc.true_relres(p.row_ptr, p.col_idx, p.val, b, r["x"])
            assert rel * nb <= (EPS_R * nb + EPS_A) * (1 + 1e-8), (r["variant"], rel)
    rat = ratios(runs)
    assert len(rat) == 3 * 4
    assert all(v > 0 for q in rat for k, v in q.items() if "/" in k)
    text = table(runs)
    assert "BiCGSTAB_d_ILU(0)" in text and "QD [1]" in text
