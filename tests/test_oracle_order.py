"""Pins for the oracle's multicolour ordering (not GPU): the greedy colouring
of the graph of A + A^T in natural order, the ordering by colour, and the
symmetric permutation B = P A P^T.  This ordering is a labelled variant
beyond the paper's method (its Section 5 leaves parallelising ILU(0) to
future work): ILU(0) of P A P^T is another preconditioner than ILU(0) of A.

References: closed forms of the greedy colouring on grids and on a crown
graph, a proper-colouring check and the greedy characterisation checked
from scipy's symmetrised pattern, numpy's stable sort, and numpy fancy
indexing of the dense matrix."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2504_14498_amd import workloads as W


def grid_coords(shape):
    """Coordinates of the rows of a grid numbered x fastest."""
    n = int(np.prod(shape))
    idx = np.arange(n)
    out = []
    for s in shape:
        out.append(idx % s)
        idx = idx // s
    return out


def sym_neighbours(rp, ci):
    """Adjacency lists of the graph of A + A^T without loops (scipy)."""
    n = len(rp) - 1
    A = sp.csr_matrix((np.ones(len(ci)), ci, rp), shape=(n, n))
    S = (A + A.T).tocsr()
    S.setdiag(0)
    S.eliminate_zeros()
    return [S.indices[S.indptr[i]:S.indptr[i + 1]] for i in range(n)]


def check_greedy(rp, ci, color, ncol):
    """A proper colouring in which every colour below a vertex's own is
    taken by one of its neighbours numbered before it; these two
    properties determine the natural-order greedy colouring."""
    nb = sym_neighbours(rp, ci)
    assert ncol == (int(color.max()) + 1 if len(color) else 0)
    for i, js in enumerate(nb):
        assert not np.any(color[js] == color[i]), "adjacent rows %d share a colour" % i
        below = set(color[js[js < i]].tolist())
        assert set(range(color[i])) <= below, "row %d could take a smaller colour" % i


def test_color_5point_is_red_black(orc):
    m = 13
    p = W.config1(m)
    color, ncol = orc.greedy_color(p.row_ptr, p.col_idx)
    x, y = grid_coords((m, m))
    assert ncol == 2
    np.testing.assert_array_equal(color, (x + y) % 2)


def test_color_7point_is_red_black(orc):
    m = 9
    p = W.config2(m)
    color, ncol = orc.greedy_color(p.row_ptr, p.col_idx)
    x, y, z = grid_coords((m, m, m))
    assert ncol == 2
    np.testing.assert_array_equal(color, (x + y + z) % 2)


def test_color_9point_four_colours(orc):
    # the 9-point stencil (king's moves): greedy in row-major order gives
    # colour (x mod 2) + 2 (y mod 2)
    m = 11
    offs = [(-1, -1), (0, -1), (1, -1), (-1, 0), (0, 0), (1, 0), (-1, 1), (0, 1), (1, 1)]
    rp, ci, val = W.stencil_csr((m, m), offs, [-1.0] * 4 + [8.0] + [-1.0] * 4)
    color, ncol = orc.greedy_color(rp, ci)
    x, y = grid_coords((m, m))
    assert ncol == 4
    np.testing.assert_array_equal(color, (x % 2) + 2 * (y % 2))


def test_color_crown_graph_needs_k_colours(orc):
    # crown graph: u_i ~ v_j for i != j, numbered u_1, v_1, u_2, v_2, ...;
    # it is bipartite, yet greedy in this order gives u_i and v_i colour
    # i - 1 (k colours), so a colouring that is merely proper or optimal
    # fails here
    k = 7
    n = 2 * k
    rows = []
    for i in range(n):
        side, idx = i % 2, i // 2
        cols = [2 * j + (1 - side) for j in range(k) if j != idx] + [i]
        rows.append(sorted(cols))
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.concatenate(rows).astype(np.int32)
    color, ncol = orc.greedy_color(rp, ci)
    assert ncol == k
    np.testing.assert_array_equal(color, np.arange(n) // 2)


def test_color_special_graphs(orc):
    n = 9
    # diagonal only: one colour
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    color, ncol = orc.greedy_color(rp, ci)
    assert ncol == 1 and not color.any()
    # dense: every vertex its own colour
    rp = (np.arange(n + 1) * n).astype(np.int32)
    ci = np.tile(np.arange(n), n).astype(np.int32)
    color, ncol = orc.greedy_color(rp, ci)
    assert ncol == n
    np.testing.assert_array_equal(color, np.arange(n))
    # upper bidiagonal pattern: the edges i ~ i+1 are seen only from A^T
    # when row i + 1 is coloured
    rows = [[i, i + 1] if i + 1 < n else [i] for i in range(n)]
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.concatenate(rows).astype(np.int32)
    color, ncol = orc.greedy_color(rp, ci)
    assert ncol == 2
    np.testing.assert_array_equal(color, np.arange(n) % 2)
    # empty matrix
    color, ncol = orc.greedy_color(np.zeros(1, dtype=np.int32), np.zeros(0, dtype=np.int32))
    assert ncol == 0 and len(color) == 0


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_color_random_nonsymmetric(orc, seed):
    p = W.random_pattern(120, 0.04, seed)
    color, ncol = orc.greedy_color(p.row_ptr, p.col_idx)
    check_greedy(p.row_ptr, p.col_idx, color, ncol)
    assert ncol >= 2


def test_color_random_rows_of_batched_shape(orc):
    p = W.random_dd(3000, 11)
    color, ncol = orc.greedy_color(p.row_ptr, p.col_idx)
    check_greedy(p.row_ptr, p.col_idx, color, ncol)


def test_color_perm_is_stable_sort(orc):
    p = W.random_pattern(200, 0.03, 5)
    color, ncol = orc.greedy_color(p.row_ptr, p.col_idx)
    perm = orc.color_perm(color, ncol)
    np.testing.assert_array_equal(perm, np.argsort(color, kind="stable"))
    perm2, ncol2 = orc.multicolor_perm(p.row_ptr, p.col_idx)
    np.testing.assert_array_equal(perm2, perm)
    assert ncol2 == ncol


def dense(rp, ci, val, C, n):
    v = val[:, 0] + 1j * val[:, 1] if C == 2 else val.reshape(-1)
    return sp.csr_matrix((v, ci, rp), shape=(n, n)).toarray()


@pytest.mark.parametrize("C", [1, 2])
def test_csr_permute_dense(orc, C):
    p = W.random_pattern(90, 0.06, 7, complex_=(C == 2))
    val = p.val.reshape(-1, C)
    rng = np.random.default_rng(3)
    for perm in (rng.permutation(p.n).astype(np.int32),
                 orc.multicolor_perm(p.row_ptr, p.col_idx)[0]):
        brp, bci, bval = orc.csr_permute(p.row_ptr, p.col_idx, val, C, perm)
        assert brp[-1] == p.nnz
        for k in range(p.n):
            assert np.all(np.diff(bci[brp[k]:brp[k + 1]]) > 0), "columns not ascending"
        A = dense(p.row_ptr, p.col_idx, val, C, p.n)
        B = dense(brp, bci, bval, C, p.n)
        np.testing.assert_array_equal(B, A[np.ix_(perm, perm)])
        # the stored pattern maps one to one (explicit zeros included)
        pat = dense(p.row_ptr, p.col_idx, np.ones((p.nnz, 1)), 1, p.n) != 0
        bpat = dense(brp, bci, np.ones((p.nnz, 1)), 1, p.n) != 0
        np.testing.assert_array_equal(bpat, pat[np.ix_(perm, perm)])


def test_red_black_factor_has_two_sweep_levels(orc):
    # after the red-black ordering every stored entry of L joins a black
    # row to a red one and every entry of U a red row to a black one, so
    # each substitution has two levels
    m = 10
    p = W.config1(m)
    perm, ncol = orc.multicolor_perm(p.row_ptr, p.col_idx)
    brp, bci, bval = orc.csr_permute(p.row_ptr, p.col_idx, p.val.reshape(-1, 1), 1, perm)
    nred = int(np.sum(np.arange(p.n) < p.n // 2 + p.n % 2))
    for k in range(p.n):
        cols = bci[brp[k]:brp[k + 1]]
        low = cols[cols < k]
        upp = cols[cols > k]
        if k < nred:
            assert len(low) == 0 and np.all(upp >= nred)
        else:
            assert len(upp) == 0 and np.all(low < nred)
    st, bad, f = orc.ilu0(brp, bci, bval, 1, 1)
    assert st == 0
    # red rows have no lower entries, so their U rows are B's rows; a black
    # row's multipliers each have one term, l_ik = b_ik / b_kk (red pivots
    # are never updated)
    diag = {k: bval[q, 0] for k in range(p.n) for q in range(brp[k], brp[k + 1]) if bci[q] == k}
    for k in range(p.n):
        for q in range(brp[k], brp[k + 1]):
            j = bci[q]
            if k < nred:
                assert f[q, 0, 0] == bval[q, 0]
            elif j < k:
                assert f[q, 0, 0] == bval[q, 0] / diag[j]


@pytest.mark.parametrize("method", ["bicgstab", "gpbicg"])
def test_multicolor_solve_recovers_x(orc, method):
    # solving P A P^T y = P b with ILU(0) of P A P^T and x = P^T y solves
    # A x = b, checked with the exact residual of the original system
    m = 12
    p = W.config1(m)
    K = 2
    b = np.zeros((p.n, 1, K))
    b[:, 0, 0] = 1.0
    perm, ncol = orc.multicolor_perm(p.row_ptr, p.col_idx)
    brp, bci, bval = orc.csr_permute(p.row_ptr, p.col_idx, p.val.reshape(-1, 1), 1, perm)
    res = orc.krylov(method, brp, bci, bval, b[perm], 1, 1e-25, max_iter=2000)
    assert res["status"] == 0
    x = np.empty_like(res["x"])
    x[perm] = res["x"]
    assert orc.true_relres(p.row_ptr, p.col_idx, p.val.reshape(-1, 1), b, x) < 1e-25
