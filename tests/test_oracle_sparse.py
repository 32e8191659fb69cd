"""Pins for the oracle's sparse kernels (not GPU): SpMV, ILU(0) factor
(Algorithm 1), substitutions (Algorithm 2), the M^H solve of Algorithm 3,
and inner products.  References: exact rationals, scipy, the literal
dense algorithms, and closed forms."""
from fractions import Fraction as F

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

from paper_2504_14498_amd import workloads as W
from tests import exact_ref as X

U = 2.0 ** -53


def fr(x):
    return sum(F(float(v)) for v in np.asarray(x).reshape(-1))


def rand_vec(rng, n, C, K):
    """Random K-limb vector with nonzero low limbs (normalised)."""
    x = np.zeros((n, C, K))
    for i in range(n):
        for c in range(C):
            v = rng.uniform(-1, 1)
            for k in range(K):
                x[i, c, k] = v
                v = v * rng.uniform(0.5, 1.0) * 2.0 ** -53
    return x


def scipy_csr(p):
    if p.C == 1:
        return sp.csr_matrix((p.val, p.col_idx, p.row_ptr), shape=(p.n, p.n))
    return sp.csr_matrix((p.val[:, 0] + 1j * p.val[:, 1], p.col_idx, p.row_ptr),
                         shape=(p.n, p.n))


def test_spmv_k1_bitwise_scipy(orc):
    p = W.random_pattern(300, 0.03, 1)
    x = np.random.default_rng(2).standard_normal(p.n)
    y = orc.spmv(p.row_ptr, p.col_idx, p.val, x.reshape(-1, 1, 1))[:, 0, 0]
    ys = scipy_csr(p) @ x
    assert np.array_equal(y, ys)


@pytest.mark.parametrize("K,C", [(2, 1), (3, 1), (4, 1), (2, 2), (4, 2)])
def test_spmv_exact_bound(orc, K, C):
    """|y - A x|_i <= (nnz_i + 1) 4 u^K (|A| |x|)_i against exact rationals."""
    p = W.random_pattern(60, 0.15, 10 + K, complex_=(C == 2))
    x = rand_vec(np.random.default_rng(K), p.n, C, K)
    y = orc.spmv(p.row_ptr, p.col_idx, p.val, x)
    A = X.csr_to_dense_q(p.row_ptr, p.col_idx, p.val, p.n, C)
    xq = X.vec_to_q(x)
    yq = X.matvec(A, xq)
    for i in range(p.n):
        mag = sum((abs(complex(A[i][j])) * abs(complex(xq[j])) for j in range(p.n)
                   if A[i][j] is not None), 0.0)
        nnz = p.row_ptr[i + 1] - p.row_ptr[i]
        err = X.limbs_to_q(y[i]) - yq[i]
        assert abs(complex(err)) <= (nnz + 1) * 4 * U ** K * mag * 1.5 + 1e-300


def test_spmv_conj_transpose(orc):
    p = W.random_pattern(40, 0.2, 5, complex_=True)
    x = rand_vec(np.random.default_rng(5), p.n, 2, 2)
    y = orc.spmv(p.row_ptr, p.col_idx, p.val, x, trans=True)
    A = X.csr_to_dense_q(p.row_ptr, p.col_idx, p.val, p.n, 2)
    yq = X.matvec_h(A, X.vec_to_q(x))
    for i in range(p.n):
        assert abs(complex(X.limbs_to_q(y[i]) - yq[i])) <= 1e-28


def test_spmv_empty_rows(orc):
    rp = np.array([0, 1, 1, 3], np.int32)
    ci = np.array([0, 0, 2], np.int32)
    val = np.array([2.0, 3.0, 4.0])
    x = np.array([[[1.0, 1e-20]], [[5.0, 0.0]], [[0.5, 0.0]]])
    y = orc.spmv(rp, ci, val, x)
    assert np.array_equal(y[1], np.zeros((1, 2)))
    assert fr(y[0]) == 2 * (F(1.0) + F(1e-20))


def ilu0_literal_float(A, mask):
    """Algorithm 1 taken literally in binary64: dense KIJ with structural
    masks, product then subtraction."""
    n = A.shape[0]
    W_ = A.copy()
    L = np.eye(n)
    Umat = np.zeros((n, n))
    for k in range(n):
        if W_[k, k] == 0:
            continue
        Umat[k, k] = W_[k, k]
        for i in range(k + 1, n):
            if not mask[i, k]:
                continue
            L[i, k] = W_[i, k] / Umat[k, k]
            for j in range(k + 1, n):
                if mask[k, j] and mask[i, j]:
                    W_[i, j] = W_[i, j] - L[i, k] * W_[k, j]
        for j in range(k + 1, n):
            if mask[k, j]:
                Umat[k, j] = W_[k, j]
    return L, Umat


def factor_to_dense(p, f):
    n = p.n
    L = np.eye(n)
    Um = np.zeros((n, n))
    for i in range(n):
        for q in range(p.row_ptr[i], p.row_ptr[i + 1]):
            j = p.col_idx[q]
            if j < i:
                L[i, j] = f[q, 0, 0]
            else:
                Um[i, j] = f[q, 0, 0]
    return L, Um


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ilu0_bitwise_literal_algorithm1(orc, seed):
    """The CSR IKJ factor equals literal KIJ Algorithm 1 bit for bit."""
    p = W.random_pattern(50, 0.12, seed, dominance=1.2)
    st, bad, f = orc.ilu0(p.row_ptr, p.col_idx, p.val, 1, 1)
    assert st == 0
    A = scipy_csr(p).toarray()
    mask = scipy_csr(p).toarray() != 0
    # explicit zeros must stay structural: rebuild the mask from the pattern
    mask = np.zeros((p.n, p.n), bool)
    for i in range(p.n):
        mask[i, p.col_idx[p.row_ptr[i]:p.row_ptr[i + 1]]] = True
    L, Um = ilu0_literal_float(A, mask)
    Lo, Uo = factor_to_dense(p, f)
    assert np.array_equal(L, Lo)
    assert np.array_equal(Um, Uo)


def test_ilu0_closed_form_5point(orc):
    """5-point stencils have no fill inside the pattern: U keeps A's upper
    entries, l_ik = a_ik / d_k and d_i = a_ii - sum_k a_ik a_ki / d_k over
    the stored k < i in ascending order (the classic ILU(0) recurrence for
    five-point matrices)."""
    p = W.config1()
    st, bad, f = orc.ilu0(p.row_ptr, p.col_idx, p.val, 1, 1)
    assert st == 0
    A = scipy_csr(p).tolil()
    n = p.n
    d = np.zeros(n)
    for i in range(n):
        di = A[i, i]
        for k in (i - 32, i - 1):
            if k >= 0 and A[i, k] != 0:
                lik = A[i, k] / d[k]
                di = di - lik * A[k, i]
        d[i] = di
    for i in range(n):
        for q in range(p.row_ptr[i], p.row_ptr[i + 1]):
            j = p.col_idx[q]
            if j == i:
                assert f[q, 0, 0] == d[i]
            elif j > i:
                assert f[q, 0, 0] == p.val[q]
            else:
                assert f[q, 0, 0] == p.val[q] / d[j]


def test_ilu0_tridiagonal_is_exact_lu(orc):
    """Tridiagonal (no fill): ILU(0) is the exact LU factorisation; compare
    with LAPACK's LU (no pivoting happens on this diagonally dominant
    matrix)."""
    n = 200
    rng = np.random.default_rng(4)
    lo, up = rng.uniform(-1, 1, n - 1), rng.uniform(-1, 1, n - 1)
    dg = 3 + rng.uniform(0, 1, n)
    A = np.diag(dg) + np.diag(lo, -1) + np.diag(up, 1)
    S = sp.csr_matrix(A)
    S.sort_indices()
    st, bad, f = orc.ilu0(S.indptr, S.indices, S.data, 1, 1)
    assert st == 0
    P, L, Um = scipy.linalg.lu(A)
    assert np.array_equal(P, np.eye(n))
    p = W.Problem("tri", n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data,
                  np.zeros(n))
    Lo, Uo = factor_to_dense(p, f)
    assert np.allclose(Lo, L, rtol=1e-14, atol=1e-15)
    assert np.allclose(Uo, Um, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("kf,C", [(1, 1), (2, 1), (1, 2), (2, 2), (3, 1), (4, 1), (3, 2), (4, 2)])
def test_ilu0_reproduces_a_on_pattern(orc, kf, C):
    """(L U)_ij = a_ij on the stored pattern, up to c u_kf (|L||U|)_ij,
    checked in exact rationals from the oracle's factor values."""
    p = W.random_pattern(24, 0.25, 30 + kf + C, complex_=(C == 2), dominance=1.1)
    st, bad, f = orc.ilu0(p.row_ptr, p.col_idx, p.val, C, kf)
    assert st == 0
    n = p.n
    Lq = [[None] * n for _ in range(n)]
    Uq = [[None] * n for _ in range(n)]
    for i in range(n):
        Lq[i][i] = X.Q(1)
        for q in range(p.row_ptr[i], p.row_ptr[i + 1]):
            j = p.col_idx[q]
            v = X.limbs_to_q(f[q])
            if j < i:
                Lq[i][j] = v
            else:
                Uq[i][j] = v
    A = X.csr_to_dense_q(p.row_ptr, p.col_idx, p.val, n, C)
    for i in range(n):
        for j in range(n):
            if A[i][j] is None:
                continue
            s = X.Q()
            mag = 0.0
            for k in range(min(i, j) + 1):
                if Lq[i][k] is not None and Uq[k][j] is not None:
                    s = s + Lq[i][k] * Uq[k][j]
                    mag += abs(complex(Lq[i][k])) * abs(complex(Uq[k][j]))
            assert abs(complex(s - A[i][j])) <= 16 * n * U ** kf * mag


@pytest.mark.parametrize("kf,C,bound", [(2, 1, 1e-28), (3, 1, 1e-44), (4, 1, 1e-59),
                                         (3, 2, 1e-44), (4, 2, 1e-59)])
def test_ilu0_literal_exact_matches_oracle(orc, kf, C, bound):
    """Literal Algorithm 1 in exact rationals vs the oracle's double-,
    triple- and quad-word factors (the paper's full-precision "ILU(0)"
    variants): every factor value agrees to a few u^kf relative."""
    p = W.random_pattern(20, 0.3, 77 + 10 * kf + C, complex_=(C == 2), dominance=1.1)
    st, bad, f = orc.ilu0(p.row_ptr, p.col_idx, p.val, C, kf)
    assert st == 0
    A = X.csr_to_dense_q(p.row_ptr, p.col_idx, p.val, p.n, C)
    L, Uq = X.ilu0_literal(A)
    worst = 0.0
    for i in range(p.n):
        for q in range(p.row_ptr[i], p.row_ptr[i + 1]):
            j = p.col_idx[q]
            ex = L[i][j] if j < i else Uq[i][j]
            got = X.limbs_to_q(f[q])
            err = abs(complex(got - ex)) / max(1.0, abs(complex(ex)))
            worst = max(worst, err)
            assert err <= bound, (i, j, err)
    # every limb counts: the error is far below the unit of a format one limb
    # shorter
    assert worst <= 2.0 ** (-53 * (kf - 1) - 20), worst


def test_ilu0_errors(orc):
    # missing diagonal
    rp = np.array([0, 2, 3], np.int32)
    ci = np.array([0, 1, 0], np.int32)
    st, bad, _ = orc.ilu0(rp, ci, np.array([1.0, 2.0, 3.0]), 1, 1)
    assert st == -5 and bad == 1
    # zero pivot: [[1, 1], [1, 1]] -> u_11 = 0
    rp = np.array([0, 2, 4], np.int32)
    ci = np.array([0, 1, 0, 1], np.int32)
    st, bad, _ = orc.ilu0(rp, ci, np.ones(4), 1, 1)
    assert st == -4 and bad == 1


def literal_algorithm2_float(L, Um, r):
    n = len(r)
    y = np.zeros(n)
    for i in range(n):
        y[i] = r[i]
        for j in range(i):
            if L[i, j] != 0:
                y[i] = y[i] - L[i, j] * y[j]
    z = np.zeros(n)
    for i in range(n - 1, -1, -1):
        z[i] = y[i]
        for j in range(i + 1, n):
            if Um[i, j] != 0:
                z[i] = z[i] - Um[i, j] * z[j]
        z[i] = z[i] / Um[i, i]
    return z


def test_apply_bitwise_literal_algorithm2(orc):
    p = W.random_pattern(60, 0.1, 3, dominance=1.3)
    st, bad, f = orc.ilu0(p.row_ptr, p.col_idx, p.val, 1, 1)
    r = np.random.default_rng(9).standard_normal(p.n)
    z = orc.ilu0_apply(p.row_ptr, p.col_idx, f, r.reshape(-1, 1, 1))[:, 0, 0]
    L, Um = factor_to_dense(p, f)
    assert np.array_equal(z, literal_algorithm2_float(L, Um, r))


def test_apply_k1_vs_scipy_triangular(orc):
    p = W.config1()
    st, bad, f = orc.ilu0(p.row_ptr, p.col_idx, p.val, 1, 1)
    L, Um = factor_to_dense(p, f)
    r = np.random.default_rng(1).standard_normal(p.n)
    z = orc.ilu0_apply(p.row_ptr, p.col_idx, f, r.reshape(-1, 1, 1))[:, 0, 0]
    from scipy.sparse.linalg import spsolve_triangular
    y = spsolve_triangular(sp.csr_matrix(L), r, lower=True, unit_diagonal=True)
    zs = spsolve_triangular(sp.csr_matrix(Um), y, lower=False)
    assert np.allclose(z, zs, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("K,kf,C", [(2, 1, 1), (2, 2, 1), (4, 1, 1), (4, 2, 1), (3, 2, 2),
                                    (2, 1, 2), (3, 3, 1), (4, 3, 1), (4, 4, 1), (3, 3, 2),
                                    (4, 4, 2)])
def test_apply_exact_bound(orc, K, kf, C):
    """z = (L U)^{-1} r and (L U)^{-H} r against exact rational solves with
    the same (oracle) factor values."""
    p = W.random_pattern(20, 0.25, 50 + K + kf, complex_=(C == 2), dominance=1.3)
    st, bad, f = orc.ilu0(p.row_ptr, p.col_idx, p.val, C, kf)
    r = rand_vec(np.random.default_rng(K), p.n, C, K)
    n = p.n
    Lq = [[None] * n for _ in range(n)]
    Uq = [[None] * n for _ in range(n)]
    for i in range(n):
        Lq[i][i] = X.Q(1)
        for q in range(p.row_ptr[i], p.row_ptr[i + 1]):
            j = p.col_idx[q]
            (Lq if j < i else Uq)[i][j] = X.limbs_to_q(f[q])
    rq = X.vec_to_q(r)
    for trans in (False, True):
        z = orc.ilu0_apply(p.row_ptr, p.col_idx, f, r, conj_trans=trans)
        zq = (X.lu_solve_h if trans else X.lu_solve)(Lq, Uq, rq)
        scale = max(abs(complex(v)) for v in zq)
        for i in range(n):
            assert abs(complex(X.limbs_to_q(z[i]) - zq[i])) <= 1e3 * n * U ** K * scale


@pytest.mark.parametrize("K,C", [(2, 1), (4, 1), (2, 2)])
def test_dot_bound(orc, K, C):
    rng = np.random.default_rng(K + C)
    n = 3000
    a = rand_vec(rng, n, C, K)
    b = rand_vec(rng, n, C, K)
    d = orc.dot(a, b)
    aq, bq = X.vec_to_q(a), X.vec_to_q(b)
    ex = X.dot(aq, bq)
    mag = sum(abs(complex(x)) * abs(complex(y)) for x, y in zip(aq, bq))
    assert abs(complex(X.limbs_to_q(d) - ex)) <= (n + 12) * 3 * U ** K * mag
