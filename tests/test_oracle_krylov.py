"""Pins for the oracle's Krylov methods (not GPU).

Exact rational runs of the four methods establish invariants a dropped
term or wrong sign would break: finite termination, the coefficients alpha
that product-type methods share with BiCG, GPBiCG with eta forced to zero
reducing to BiCGSTAB, and BiCG reducing to CG on symmetric positive
definite matrices.  The floating-point oracle (in QD) is then tied to the
exact runs pass by pass, and checked on no-fill matrices (one pass) and on
a manufactured solution."""
import numpy as np
import pytest

from paper_2504_14498_amd import workloads as W
from tests import exact_ref as X

METHODS = ["bicg", "cgs", "bicgstab", "gpbicg"]
RUN = {"bicg": X.bicg, "cgs": X.cgs, "bicgstab": X.bicgstab, "gpbicg": X.gpbicg}


def small_system(n, seed, complex_=False, dominance=None, density=0.5):
    p = W.random_pattern(n, density, seed, complex_=complex_, dominance=dominance)
    C = p.C
    A = X.csr_to_dense_q(p.row_ptr, p.col_idx, p.val, n, C)
    rng = np.random.default_rng(seed + 1000)
    bre = rng.integers(-9, 10, n)
    bim = rng.integers(-9, 10, n) if complex_ else np.zeros(n, int)
    b = [X.Q(int(r), int(i)) for r, i in zip(bre, bim)]
    return p, A, b


@pytest.mark.parametrize("complex_", [False, True])
def test_exact_finite_termination_and_shared_alpha(complex_):
    """M = I: every method reaches r = 0 within n passes (unless it breaks
    down) and all four share BiCG's alpha_k pass by pass."""
    n = 6
    p, A, b = small_system(n, 3, complex_)
    runs = {m: RUN[m](A, b, n + 1) for m in METHODS}
    for m, out in runs.items():
        assert out[-1]["r"] is not None
        assert all(v.is_zero() for v in out[-1]["r"]), m
        assert len(out) <= n
        x = out[-1]["x"]
        assert X.matvec(A, x) == b, m
    ref = [o["alpha"] for o in runs["bicg"]]
    for m in METHODS[1:]:
        al = [o["alpha"] for o in runs[m]]
        assert al == ref[: len(al)], m


def test_exact_product_methods_share_alpha_with_ilu0():
    """M = ILU(0) (right preconditioning, shadow r0): CGS, BiCGSTAB and
    GPBiCG generate the same alpha_k and terminate within n passes."""
    n = 7
    p, A, b = small_system(n, 11, dominance=0.6, density=0.45)
    M = X.ilu0_literal(A)
    runs = {m: RUN[m](A, b, n + 1, M=M) for m in ("cgs", "bicgstab", "gpbicg")}
    for m, out in runs.items():
        assert all(v.is_zero() for v in out[-1]["r"]), m
        assert X.matvec(A, out[-1]["x"]) == b
    ref = [o["alpha"] for o in runs["cgs"]]
    for m in ("bicgstab", "gpbicg"):
        al = [o["alpha"] for o in runs[m]]
        assert al == ref[: len(al)], m


def test_exact_preconditioned_bicg_terminates():
    """Algorithm 3 with M = ILU(0) terminates within n passes with A x = b."""
    n = 7
    p, A, b = small_system(n, 12, complex_=True, dominance=0.6, density=0.45)
    M = X.ilu0_literal(A)
    out = X.bicg(A, b, n + 1, M=M)
    assert all(v.is_zero() for v in out[-1]["r"])
    assert X.matvec(A, out[-1]["x"]) == b


def test_exact_gpbicg_eta_zero_is_bicgstab():
    n = 6
    p, A, b = small_system(n, 21)
    g = X.gpbicg(A, b, n + 1, force_eta_zero=True)
    s = X.bicgstab(A, b, n + 1)
    for a, c in zip(g, s):
        assert a["x"] == c["x"]
        assert a["zeta"] == c["omega"]


def test_exact_bicg_is_cg_on_spd():
    n = 6
    rng = np.random.default_rng(5)
    B = rng.integers(-3, 4, (n, n))
    S = B @ B.T + n * np.eye(n, dtype=int)
    A = [[X.Q(int(S[i, j])) if S[i, j] != 0 or i == j else None for j in range(n)]
         for i in range(n)]
    b = [X.Q(int(v)) for v in rng.integers(-5, 6, n)]
    c = X.cg(A, b, n)
    bi = X.bicg(A, b, n)
    for a, d in zip(c, bi):
        assert a["x"] == d["x"]


def _to_float(vq, C, K):
    """Q vector -> nearest (n, C, K) limbs (via exact rationals)."""
    from fractions import Fraction as F
    out = np.zeros((len(vq), C, K))
    for i, v in enumerate(vq):
        for c, part in enumerate([v.re, v.im][:C]):
            r = F(part)
            for k in range(K):
                d = float(r)
                out[i, c, k] = d
                r -= F(d)
    return out


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("complex_", [False, True])
@pytest.mark.parametrize("precond", [False, True])
def test_oracle_qd_follows_exact_run(orc, method, complex_, precond):
    """The QD oracle after 1..3 passes agrees with the exact run (x to a
    relative 1e-45, recursive residual norms to binary64 rounding)."""
    n = 8
    p, A, b = small_system(n, 40 + (7 if complex_ else 0), complex_, dominance=0.8,
                           density=0.4)
    C = 2 if complex_ else 1
    M = None
    if precond:
        # the exact run uses the oracle's own double-word factor values, so
        # that only the QD vector arithmetic separates the two runs
        st, bad, f = orc.ilu0(p.row_ptr, p.col_idx, p.val, C, 2)
        assert st == 0
        Lq = [[X.Q(1) if i == j else None for j in range(n)] for i in range(n)]
        Uq = [[None] * n for _ in range(n)]
        for i in range(n):
            for q in range(p.row_ptr[i], p.row_ptr[i + 1]):
                j = p.col_idx[q]
                (Lq if j < i else Uq)[i][j] = X.limbs_to_q(f[q])
        M = (Lq, Uq)
    bf = _to_float(b, C, 4)
    bq = X.vec_to_q(bf)
    for passes in (1, 2, 3):
        ex = RUN[method](A, bq, passes, M=M)
        res = orc.krylov(method, p.row_ptr, p.col_idx, p.val, bf, kf=2 if precond else 0,
                         tol_rel=0.0, max_iter=passes, hist_len=passes)
        assert res["status"] == 1 and res["iters"] == passes
        xq = ex[-1]["x"]
        scale = max(abs(complex(v)) for v in xq)
        for i in range(n):
            err = abs(complex(X.limbs_to_q(res["x"][i]) - xq[i]))
            assert err <= 1e-45 * scale, (method, passes, i, err)
        rn = [float(sum((v.abs2() for v in o["r"]), 0)) for o in ex]
        assert np.allclose(res["hist"], rn[: len(res["hist"])], rtol=1e-13)


@pytest.mark.parametrize("method", METHODS)
def test_oracle_no_fill_converges_in_one_pass(orc, method):
    """Tridiagonal A: ILU(0) is exact, M = A, so one pass solves the system
    (to DD rounding)."""
    n = 300
    rng = np.random.default_rng(8)
    import scipy.sparse as sp
    A = sp.diags([rng.uniform(-1, 1, n - 1), 3 + rng.uniform(0, 1, n), rng.uniform(-1, 1, n - 1)],
                 [-1, 0, 1], format="csr")
    A.sort_indices()
    b = np.zeros((n, 1, 2))
    b[:, 0, 0] = rng.uniform(-1, 1, n)
    res = orc.krylov(method, A.indptr, A.indices, A.data, b, kf=2, tol_rel=1e-25, max_iter=5)
    assert res["status"] == 0
    assert res["iters"] == 1
    assert res["relres_true"] < 1e-25


def test_oracle_manufactured_solution_config1(orc):
    """Configuration 1 (5-point upwind, Peclet 10, b = A 1): BiCGSTAB in DD
    with a binary64 ILU(0) factor reaches 1e-20 and x = 1 to the accuracy
    the conditioning allows."""
    p = W.config1()
    x = p.x_true_limbs(2)
    b = orc.spmv(p.row_ptr, p.col_idx, p.val, x)
    res = orc.krylov("bicgstab", p.row_ptr, p.col_idx, p.val, b, kf=1, tol_rel=1e-20,
                     max_iter=2000)
    assert res["status"] == 0
    assert res["relres_true"] < 1e-20
    err = np.abs(res["x"][:, 0, 0] + res["x"][:, 0, 1] - 1.0).max()
    assert err < 1e-16
    assert 5 <= res["iters"] <= 200


def test_oracle_breakdown_and_max_iter(orc):
    # A = [[0, 1], [1, 0]], b = e1, M = I: <r~, A p> = 0 at the first pass
    rp = np.array([0, 2, 4], np.int32)
    ci = np.array([0, 1, 0, 1], np.int32)
    val = np.array([0.0, 1.0, 1.0, 0.0])
    b = np.zeros((2, 1, 2))
    b[0, 0, 0] = 1.0
    for m in ("cgs", "bicgstab", "gpbicg", "bicg"):
        res = orc.krylov(m, rp, ci, val, b, kf=0, tol_rel=1e-25, max_iter=10)
        assert res["status"] == 2, m
    p = W.config1()
    b = orc.spmv(p.row_ptr, p.col_idx, p.val, p.x_true_limbs(2))
    res = orc.krylov("bicgstab", p.row_ptr, p.col_idx, p.val, b, kf=1, tol_rel=1e-20,
                     max_iter=1)
    assert res["status"] == 1 and res["iters"] == 1
