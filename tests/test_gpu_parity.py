"""GPU parity: the HIP library (through its C-ABI) against the CPU oracle.

SpMV, ILU(0) factorisation + substitutions and the M^H solve keep the
oracle's per-entry operation order, so they must agree bit for bit.  Inner
products use a reduction tree, so they are checked against the oracle
within the summation error bound.  Solves are checked on what is unique:
the true residual of the GPU's x (recomputed exactly by the oracle) must
pass the tolerance, and the iteration count must be close to the
oracle's."""
import numpy as np
import pytest

from paper_2504_14498_amd import workloads as W

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def mpk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_14498_amd import mpk as m
    m.library()
    return m


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rand_vec(rng, n, C, K):
    x = np.zeros((n, C, K))
    v = rng.uniform(-1, 1, (n, C))
    for k in range(K):
        x[:, :, k] = v
        v = v * rng.uniform(0.5, 1.0, (n, C)) * 2.0 ** -53
    return x


def case(name):
    """Small/medium matrices spanning several workgroups and a ragged tail."""
    if name == "rand_real":
        return W.random_pattern(1531, 0.004, 1, dominance=1.2)
    if name == "rand_cplx":
        return W.random_pattern(1277, 0.005, 2, complex_=True, dominance=1.2)
    if name == "conv2d32":         # the 32 x 32 convection-diffusion system itself
        return W.config1(32)
    if name == "conv2d":
        return W.config1(37)
    if name == "conv2d_tail":      # several sweep blocks, the last one short
        return W.config1(150)
    if name == "conv3d":
        return W.config2(12)
    if name == "helm":
        return W.config3(41)
    if name == "rdd":
        return W.random_dd(3001, 5)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["rand_real", "rand_cplx", "conv3d", "helm", "rdd"])
@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_spmv_bitwise(mpk, orc, name, K):
    p = case(name)
    A = mpk.Csr.from_problem(p)
    x = rand_vec(np.random.default_rng(K), p.n, p.C, K)
    y = host(mpk.csr_spmv(A, dev(x)))
    yo = orc.spmv(p.row_ptr, p.col_idx, p.val, x)
    assert np.array_equal(y, yo)


@pytest.mark.parametrize("name", ["rand_real", "rand_cplx", "conv3d", "rdd"])
@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_residual_bitwise(mpk, orc, name, K):
    """r = b - A x: the oracle's SpMV, then one K-limb subtraction per
    component (exact negation, then the oracle's addition)."""
    p = case(name)
    A = mpk.Csr.from_problem(p)
    rng = np.random.default_rng(3 * K)
    x = rand_vec(rng, p.n, p.C, K)
    b = rand_vec(rng, p.n, p.C, K)
    r = host(mpk.csr_residual(A, dev(b), dev(x)))
    y = orc.spmv(p.row_ptr, p.col_idx, p.val, x)
    ro = np.empty_like(b)
    for i in range(p.n):
        for c in range(p.C):
            ro[i, c] = orc.add(b[i, c], -y[i, c])
    assert np.array_equal(r, ro)


@pytest.mark.parametrize("name", ["rand_real", "rand_cplx", "conv3d", "rdd"])
@pytest.mark.parametrize("K", [1, 2, 4])
@pytest.mark.parametrize("lanes", [2, 4, 8, 16])
def test_spmv_vector_csr_bitwise(mpk, orc, name, K, lanes):
    """Vector CSR (lanes per row > 1): the same products added in the same
    order, so y equals the oracle's bit for bit."""
    p = case(name)
    A = mpk.Csr.from_problem(p)
    mpk.spmv_set_lanes(A, lanes)
    x = rand_vec(np.random.default_rng(K + lanes), p.n, p.C, K)
    y = host(mpk.csr_spmv(A, dev(x)))
    mpk.spmv_set_lanes(A, 0)
    assert np.array_equal(y, orc.spmv(p.row_ptr, p.col_idx, p.val, x))


@pytest.mark.parametrize("C,K", [(1, 2), (2, 3)])
@pytest.mark.parametrize("lanes", [2, 4, 16])
def test_spmv_vector_csr_ragged_rows_bitwise(mpk, orc, C, K, lanes):
    """Empty rows, rows shorter and longer than a group, a last empty row."""
    rng = np.random.default_rng(71 + K + lanes)
    n = 1337
    lens = rng.choice([0, 1, 2, 3, 15, 16, 17, 33, 70], size=n)
    lens[-1] = 0
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate([np.sort(rng.choice(n, size=l, replace=False)) for l in lens if l > 0]
                        ).astype(np.int32)
    val = rng.standard_normal((len(ci), C)) if C == 2 else rng.standard_normal(len(ci))
    A = mpk.Csr(rp, ci, val)
    mpk.spmv_set_lanes(A, lanes)
    x = rand_vec(np.random.default_rng(K), n, C, K)
    y = host(mpk.csr_spmv(A, dev(x)))
    assert np.array_equal(y, orc.spmv(rp, ci, val, x))
    assert np.all(y[lens == 0] == 0)


def test_spmv_tune_keeps_results(mpk, orc):
    """The tuner picks one of the choices and the SpMV then gives the same
    bits as the oracle."""
    p = case("rdd")
    A = mpk.Csr.from_problem(p)
    x = rand_vec(np.random.default_rng(3), p.n, p.C, 2)
    lanes, ms = mpk.spmv_tune(A, dev(x))
    assert lanes in (1, 2, 4, 8, 16) and ms > 0
    y = host(mpk.csr_spmv(A, dev(x)))
    mpk.spmv_set_lanes(A, 0)
    assert np.array_equal(y, orc.spmv(p.row_ptr, p.col_idx, p.val, x))


@pytest.mark.parametrize("C", [1, 2])
@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_spmv_ragged_rows_bitwise(mpk, orc, C, K):
    """Empty rows, rows shorter and longer than the batch of entries whose
    loads are issued together, and a last row that is empty."""
    rng = np.random.default_rng(31 + K)
    n = 1300
    lens = rng.choice([0, 1, 3, 7, 8, 9, 17, 40], size=n)
    lens[-1] = 0
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate([np.sort(rng.choice(n, size=l, replace=False)) for l in lens if l > 0]
                        ).astype(np.int32)
    val = rng.standard_normal((len(ci), C)) if C == 2 else rng.standard_normal(len(ci))
    A = mpk.Csr(rp, ci, val)
    x = rand_vec(np.random.default_rng(K), n, C, K)
    y = host(mpk.csr_spmv(A, dev(x)))
    yo = orc.spmv(rp, ci, val, x)
    assert np.array_equal(y, yo)
    assert np.all(y[lens == 0] == 0)


@pytest.mark.parametrize("name", ["rand_real", "rand_cplx"])
@pytest.mark.parametrize("K", [2, 4])
def test_spmv_transpose_bitwise(mpk, orc, name, K):
    p = case(name)
    A = mpk.Csr.from_problem(p)
    x = rand_vec(np.random.default_rng(K + 7), p.n, p.C, K)
    y = host(mpk.csr_spmv(A, dev(x), trans=True))
    yo = orc.spmv(p.row_ptr, p.col_idx, p.val, x, trans=True)
    assert np.array_equal(y, yo)


@pytest.mark.parametrize("name", ["rand_real", "rand_cplx", "conv2d", "conv2d_tail", "conv3d", "helm",
                                  "rdd"])
@pytest.mark.parametrize("kf,K", [(1, 1), (1, 2), (2, 2), (1, 3), (2, 3), (1, 4), (2, 4), (3, 3),
                                  (3, 4), (4, 4)])
def test_ilu0_apply_bitwise(mpk, orc, name, kf, K):
    p = case(name)
    A = mpk.Csr.from_problem(p)
    M = mpk.ilu0_factor(A, kf, adjoint=True)
    st, bad, f = orc.ilu0(p.row_ptr, p.col_idx, p.val, p.C, kf)
    assert st == 0
    r = rand_vec(np.random.default_rng(11 * K + kf), p.n, p.C, K)
    z = host(mpk.ilu0_apply(M, dev(r)))
    zo = orc.ilu0_apply(p.row_ptr, p.col_idx, f, r)
    assert np.array_equal(z, zo)
    zh = host(mpk.ilu0_apply(M, dev(r), conj_trans=True))
    zho = orc.ilu0_apply(p.row_ptr, p.col_idx, f, r, conj_trans=True)
    assert np.array_equal(zh, zho)


@pytest.mark.parametrize("name", ["rand_real", "rand_cplx", "conv2d_tail", "conv3d", "helm", "rdd"])
@pytest.mark.parametrize("kf,K", [(1, 2), (2, 2), (1, 4), (4, 4)])
def test_ilu0_apply_level_launches_bitwise(mpk, orc, monkeypatch, name, kf, K):
    """The one-launch-per-level sweeps (chosen by themselves for few, wide
    levels; forced here on every case) against the oracle, bit for bit."""
    monkeypatch.setenv("MPK_TRSV_MODE", "s")
    p = case(name)
    A = mpk.Csr.from_problem(p)
    M = mpk.ilu0_factor(A, kf, adjoint=True)
    st, bad, f = orc.ilu0(p.row_ptr, p.col_idx, p.val, p.C, kf)
    assert st == 0
    r = rand_vec(np.random.default_rng(7 * K + kf), p.n, p.C, K)
    assert np.array_equal(host(mpk.ilu0_apply(M, dev(r))), orc.ilu0_apply(p.row_ptr, p.col_idx,
                                                                           f, r))
    assert np.array_equal(host(mpk.ilu0_apply(M, dev(r), conj_trans=True)),
                          orc.ilu0_apply(p.row_ptr, p.col_idx, f, r, conj_trans=True))


def complex_grid2d(m, seed):
    """A complex matrix on the 5-point pattern of an m x m grid (diagonally
    dominant): the pattern of config1 with random complex values."""
    p = W.config1(m)
    rng = np.random.default_rng(seed)
    val = np.zeros((len(p.col_idx), 2))
    val[:, 0] = p.val
    val[:, 1] = 0.3 * rng.uniform(-1, 1, len(p.col_idx))
    return p.row_ptr, p.col_idx, val


@pytest.mark.parametrize("shape", ["conv3d_20", "conv2d_150", "cplx2d_70"])
@pytest.mark.parametrize("rows", [256, 1024])
@pytest.mark.parametrize("kf,K", [(1, 2), (2, 3), (1, 4)])
def test_ilu0_apply_deep_blocks_bitwise(mpk, orc, monkeypatch, shape, rows, kf, K):
    """Blocked sweeps with blocks several grid planes (or lines) deep: small
    blocks force many of them, including short ones at the grid's end, on
    3D and 2D grids and a complex system; all four sweeps (L, U and the
    adjoint pair) against the oracle, element by element."""
    monkeypatch.setenv("MPK_TRSV_BLOCK_ROWS", str(rows))
    monkeypatch.setenv("MPK_TRSV_MODE", "b")   # blocked, not the grid sweeps
    if shape == "conv3d_20":
        p = W.config2(20)
        rp, ci, val, C = p.row_ptr, p.col_idx, p.val, 1
    elif shape == "conv2d_150":
        p = W.config1(150)
        rp, ci, val, C = p.row_ptr, p.col_idx, p.val, 1
    else:
        rp, ci, val = complex_grid2d(70, 5)
        C = 2
    n = len(rp) - 1
    A = mpk.Csr(rp, ci, val)
    M = mpk.ilu0_factor(A, kf, adjoint=True)
    st, bad, f = orc.ilu0(rp, ci, val, C, kf)
    assert st == 0
    r = rand_vec(np.random.default_rng(7 * K + kf + rows), n, C, K)
    z = host(mpk.ilu0_apply(M, dev(r)))
    assert np.array_equal(z, orc.ilu0_apply(rp, ci, f, r))
    zh = host(mpk.ilu0_apply(M, dev(r), conj_trans=True))
    assert np.array_equal(zh, orc.ilu0_apply(rp, ci, f, r, conj_trans=True))


def grid_problem(shape, seed, C=1):
    """A matrix on the 7-point (3D) or 5-point (2D) stencil of a grid of the
    given shape (x fastest), random off-diagonal entries and a dominant
    diagonal; complex when C = 2."""
    rng = np.random.default_rng(seed)
    dims = len(shape)
    offs = ([(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
            if dims == 3 else [(0, -1), (-1, 0), (0, 0), (1, 0), (0, 1)])
    arr_shape = tuple(reversed(shape))
    coef = []
    for o in offs:
        if all(v == 0 for v in o):
            coef.append(None)
            continue
        c = -rng.uniform(0.1, 1.0, arr_shape)
        if C == 2:
            c = c + 1j * rng.uniform(-0.3, 0.3, arr_shape)
        coef.append(c)
    dia = sum(np.abs(c) for c in coef if c is not None) + 1.0
    coef = [dia if c is None else c for c in coef]
    rp, ci, val = W.stencil_csr(shape, offs, coef)
    return rp, ci, val


GRID_SHAPES = [(12, 12, 12), (20, 13, 9), (9, 17, 16), (33, 8, 8), (5, 3, 70), (37, 37),
               (150, 150), (64, 70), (7, 200), (130, 65)]


@pytest.mark.parametrize("shape", GRID_SHAPES)
@pytest.mark.parametrize("kf,K", [(1, 1), (1, 2), (2, 2), (1, 3), (3, 3), (2, 4), (4, 4)])
def test_ilu0_apply_grid_bitwise(mpk, orc, shape, kf, K):
    """The grid sweeps (7-point and 5-point stencils numbered x fastest,
    blocks of 8 x 8 or 64 lines, ragged last blocks) against the oracle,
    element by element: the forward L and backward U sweeps, and the
    adjoint pair (which keeps the blocked sweeps)."""
    rp, ci, val = grid_problem(shape, sum(shape) + kf)
    n = len(rp) - 1
    A = mpk.Csr(rp, ci, val)
    M = mpk.ilu0_factor(A, kf, adjoint=True)
    st, bad, f = orc.ilu0(rp, ci, val, 1, kf)
    assert st == 0
    r = rand_vec(np.random.default_rng(5 * K + kf), n, 1, K)
    assert np.array_equal(host(mpk.ilu0_apply(M, dev(r))), orc.ilu0_apply(rp, ci, f, r))
    assert np.array_equal(host(mpk.ilu0_apply(M, dev(r), conj_trans=True)),
                          orc.ilu0_apply(rp, ci, f, r, conj_trans=True))


@pytest.mark.parametrize("shape", [(10, 11, 12), (70, 70), (9, 130)])
@pytest.mark.parametrize("kf,K", [(1, 2), (2, 2), (1, 4), (4, 4)])
def test_ilu0_apply_grid_complex_bitwise(mpk, orc, shape, kf, K):
    rp, ci, val = grid_problem(shape, 3 + kf, C=2)
    n = len(rp) - 1
    A = mpk.Csr(rp, ci, val)
    M = mpk.ilu0_factor(A, kf)
    st, bad, f = orc.ilu0(rp, ci, val, 2, kf)
    assert st == 0
    r = rand_vec(np.random.default_rng(9 * K + kf), n, 2, K)
    assert np.array_equal(host(mpk.ilu0_apply(M, dev(r))), orc.ilu0_apply(rp, ci, f, r))


def test_ilu0_apply_grid_matches_blocked(mpk, orc, monkeypatch):
    """On the same 24^3 system the grid sweeps and the forced blocked sweeps
    give the same bits (and the oracle's)."""
    rp, ci, val = grid_problem((24, 24, 24), 11)
    n = len(rp) - 1
    r = rand_vec(np.random.default_rng(1), n, 1, 2)
    A = mpk.Csr(rp, ci, val)
    z_grid = host(mpk.ilu0_apply(mpk.ilu0_factor(A, 1), dev(r)))
    monkeypatch.setenv("MPK_TRSV_MODE", "b")
    z_blk = host(mpk.ilu0_apply(mpk.ilu0_factor(A, 1), dev(r)))
    st, bad, f = orc.ilu0(rp, ci, val, 1, 1)
    assert np.array_equal(z_grid, z_blk)
    assert np.array_equal(z_grid, orc.ilu0_apply(rp, ci, f, r))


@pytest.mark.parametrize("C,K", [(1, 1), (1, 2), (1, 4), (2, 2), (2, 3)])
@pytest.mark.parametrize("n", [1, 255, 256, 257, 100003])
def test_dot_within_bound(mpk, orc, C, K, n):
    rng = np.random.default_rng(n + K)
    a = rand_vec(rng, n, C, K)
    b = rand_vec(rng, n, C, K)
    d = host(mpk.dot(dev(a), dev(b)))
    do = orc.dot(a, b)
    mag = np.sum(np.abs(a[:, :, 0]).sum(1) * np.abs(b[:, :, 0]).sum(1))
    err = np.abs(d.sum(axis=-1) - do.sum(axis=-1)).max() if K == 1 else \
        max(abs(float(np.sum(d[c])) - float(np.sum(do[c]))) for c in range(C))
    # both sides are within (n + log2 n) 3 u^K of the exact value
    bound = 2 * (n + 20) * 3 * U ** K * mag
    # compare limb sums in extended arithmetic
    from fractions import Fraction as F
    for c in range(C):
        diff = abs(sum(F(v) for v in d[c]) - sum(F(v) for v in do[c]))
        assert float(diff) <= bound + 1e-300
    del err


def test_factor_errors(mpk):
    import torch
    # zero pivot: [[1, 1], [1, 1]]
    A = mpk.Csr([0, 2, 4], [0, 1, 0, 1], [1.0, 1.0, 1.0, 1.0])
    with pytest.raises(mpk.MpkError) as e:
        mpk.ilu0_factor(A, 1)
    assert e.value.status == -4 and e.value.bad_row == 1
    # missing diagonal
    A = mpk.Csr([0, 2, 3], [0, 1, 0], [1.0, 2.0, 3.0])
    with pytest.raises(mpk.MpkError) as e:
        mpk.ilu0_factor(A, 1)
    assert e.value.status == -5 and e.value.bad_row == 1
    # unsorted columns
    A = mpk.Csr([0, 2, 4], [1, 0, 0, 1], [1.0, 2.0, 3.0, 4.0])
    with pytest.raises(mpk.MpkError) as e:
        mpk.ilu0_factor(A, 1)
    assert e.value.status == -8
    # non-finite entry
    A = mpk.Csr([0, 1, 2], [0, 1], [1.0, float("nan")])
    with pytest.raises(mpk.MpkError) as e:
        mpk.ilu0_factor(A, 2)
    assert e.value.status == -7 and e.value.bad_row == 1
    torch.cuda.synchronize()


@pytest.mark.parametrize("shape", [(9, 7, 6), (40, 30)])
@pytest.mark.parametrize("kf", [1, 2])
def test_grid_factor_zero_pivot(mpk, orc, monkeypatch, shape, kf):
    """Zero pivots on a grid pattern: a row whose diagonal and lower entries
    are zero has u_ii = 0 exactly; the grid factorisation and the
    level-by-level one (forced) report the lowest such row, as the oracle."""
    rp, ci, val = grid_problem(shape, 7)
    val = val.copy()
    n = len(rp) - 1
    for k in (n // 3, n // 2):
        for q in range(rp[k], rp[k + 1]):
            if ci[q] <= k:
                val[q] = 0.0
    st, bad, f = orc.ilu0(rp, ci, val, 1, kf)
    assert st == -4 and bad == n // 3
    for mode in (None, "l"):
        if mode:
            monkeypatch.setenv("MPK_TRSV_MODE", mode)
        with pytest.raises(mpk.MpkError) as e:
            mpk.ilu0_factor(mpk.Csr(rp, ci, val), kf)
        assert e.value.status == -4 and e.value.bad_row == n // 3


def test_grid_recognition_near_grids(mpk, orc):
    """Without adjoint schedules a grid is recognised on the device; patterns
    that only look like one take the other schedules: a stencil row with one
    column moved (still sorted and in range), the last row changed, and
    broken row pointers (reported as the host's checks report them).  The
    apply agrees with the oracle bit for bit."""
    shape = (9, 8, 7)
    rp, ci, val = grid_problem(shape, 21)
    n = len(rp) - 1
    r = rand_vec(np.random.default_rng(5), n, 1, 2)
    cases = []
    moved = ci.copy()
    k = 4 * 9 * 8 + 3 * 9 + 4          # an interior row; its x + 1 entry moves to x + 2
    q = int(np.searchsorted(ci[rp[k]:rp[k + 1]], k + 1)) + rp[k]
    assert ci[q] == k + 1
    moved[q] = k + 2
    cases.append(moved)
    last = ci.copy()
    last[rp[n - 1]] = ci[rp[n - 1]] + 1      # the last row's z - 1 column shifted
    cases.append(last)
    for cc in cases:
        A = mpk.Csr(rp, cc, val)
        M = mpk.ilu0_factor(A, 1)
        st, bad, f = orc.ilu0(rp, cc, val, 1, 1)
        assert st == 0
        assert np.array_equal(host(mpk.ilu0_apply(M, dev(r))), orc.ilu0_apply(rp, cc, f, r))
    for cut in (n // 2, n):
        bad_rp = rp.copy()
        bad_rp[cut] = -5 if cut < n else rp[n] - 1
        with pytest.raises(mpk.MpkError) as e:
            mpk.ilu0_factor(mpk.Csr(bad_rp, ci, val), 1)
        assert e.value.status == -8, e.value.status


def true_relres(orc, p, x, b):
    """||b - A x|| / ||b|| from the GPU's x (any limb count), by the oracle:
    the residual components are formed exactly and rounded once, so the
    check does not depend on the precision the solve ran in."""
    return orc.true_relres(p.row_ptr, p.col_idx, p.val, b, x)


# The device stops when its own K-limb true residual passes the test; the
# exact residual differs from that by a rounding of the norms (binary64 on
# both sides), far below this margin.
RES_MARGIN = 1 + 1e-8


SOLVE_CASES = [
    # (problem, method, K, kf, tol)
    ("conv2d32", "bicgstab", 2, 1, 1e-20),
    ("conv2d", "bicgstab", 2, 1, 1e-20),
    ("conv2d", "bicgstab", 2, 2, 1e-25),
    ("conv2d", "cgs", 2, 1, 1e-20),
    ("conv2d", "bicg", 2, 1, 1e-20),
    ("conv2d", "gpbicg", 2, 1, 1e-20),
    ("conv3d", "bicgstab", 2, 1, 1e-25),
    ("conv3d", "gpbicg", 2, 2, 1e-25),
    ("conv3d", "bicg", 2, 2, 1e-25),
    ("conv3d", "cgs", 3, 1, 1e-30),
    ("conv3d", "bicgstab", 4, 2, 1e-50),
    ("conv2d", "bicgstab", 1, 1, 1e-12),
    ("conv2d_tail", "bicg", 2, 1, 1e-25),
    ("helm", "gpbicg", 2, 1, 1e-25),
    ("helm", "bicgstab", 2, 2, 1e-25),
    ("helm", "bicg", 2, 1, 1e-25),
    ("helm", "cgs", 4, 1, 1e-40),
    ("rdd", "bicgstab", 2, 1, 1e-25),
    ("rdd", "gpbicg", 3, 2, 1e-35),
    # full-precision factors: triple- and quad-word ILU(0)
    ("conv3d", "bicgstab", 3, 3, 1e-35),
    ("conv3d", "bicg", 4, 4, 1e-50),
    ("conv2d", "cgs", 4, 4, 1e-50),
    ("helm", "gpbicg", 3, 3, 1e-35),
    ("helm", "bicgstab", 4, 4, 1e-50),
    ("rdd", "gpbicg", 4, 4, 1e-50),
    ("rand_cplx", "bicg", 3, 3, 1e-35),
    # complex GPBiCG in QD: its 2x2 system's denominator falls below
    # 2^-300 near convergence (complex division with a scaled divisor)
    ("helm", "gpbicg", 4, 4, 1e-50),
    ("rand_cplx", "gpbicg", 4, 1, 1e-50),
]


@pytest.mark.parametrize("name,method,K,kf,tol", SOLVE_CASES)
def test_solve_parity(mpk, orc, name, method, K, kf, tol):
    p = case(name)
    b = orc.spmv(p.row_ptr, p.col_idx, p.val, p.x_true_limbs(K))
    ref = orc.krylov(method, p.row_ptr, p.col_idx, p.val, b, kf=kf, tol_rel=tol, max_iter=3000,
                     hist_len=3000)
    assert ref["status"] == 0, ref["status"]
    A = mpk.Csr.from_problem(p)
    x, info = mpk.krylov_solve(method, A, dev(b), fprec=kf, tol_rel=tol, max_iter=3000,
                               hist_len=3000)
    assert info["status"] == "ok", info
    rel = true_relres(orc, p, host(x), b)
    assert rel <= tol * RES_MARGIN, (rel, tol)
    assert abs(info["iters"] - ref["iters"]) <= max(3, 0.05 * ref["iters"]), (info["iters"],
                                                                             ref["iters"])
    # the recursive residual histories agree over the first passes (only the
    # inner products' reduction order differs, a u_K-level perturbation)
    h, ho = host(info["hist"]), ref["hist"]
    m = min(20, len(h), len(ho))
    assert np.allclose(h[:m], ho[:m], rtol=1e-12 if K >= 2 else 1e-6, atol=0)
    # the GPU's own report of the true residual is consistent with the recheck
    assert info["relres_true"] <= tol


@pytest.mark.parametrize("method,K,kf", [("bicgstab", 2, 1), ("bicg", 2, 1), ("gpbicg", 3, 2)])
def test_solve_parity_deep_blocks(mpk, orc, monkeypatch, method, K, kf):
    """Whole solves on blocked sweeps with blocks several planes deep (small
    blocks forced on a 20^3 grid, so sweeps cross many of them): the same
    checks as the other solve cases against the oracle."""
    monkeypatch.setenv("MPK_TRSV_BLOCK_ROWS", "256")
    monkeypatch.setenv("MPK_TRSV_MODE", "b")   # blocked, not the grid sweeps
    p = W.config2(20)
    tol = 1e-25 if K == 2 else 1e-35
    b = orc.spmv(p.row_ptr, p.col_idx, p.val, p.x_true_limbs(K))
    ref = orc.krylov(method, p.row_ptr, p.col_idx, p.val, b, kf=kf, tol_rel=tol, max_iter=3000,
                     hist_len=3000)
    assert ref["status"] == 0, ref["status"]
    A = mpk.Csr.from_problem(p)
    x, info = mpk.krylov_solve(method, A, dev(b), fprec=kf, tol_rel=tol, max_iter=3000,
                               hist_len=3000)
    assert info["status"] == "ok", info
    rel = true_relres(orc, p, host(x), b)
    assert rel <= tol * RES_MARGIN, (rel, tol)
    assert abs(info["iters"] - ref["iters"]) <= max(3, 0.05 * ref["iters"])
    h, ho = host(info["hist"]), ref["hist"]
    m = min(20, len(h), len(ho))
    assert np.allclose(h[:m], ho[:m], rtol=1e-12, atol=0)


@pytest.mark.parametrize("name,method,K,kf,tol", [("conv2d", "bicgstab", 2, 1, 1e-20),
                                                  ("helm", "gpbicg", 2, 1, 1e-25),
                                                  ("rdd", "bicg", 2, 1, 1e-25),
                                                  ("conv3d", "cgs", 3, 3, 1e-30)])
def test_solve_parity_level_launches(mpk, orc, monkeypatch, name, method, K, kf, tol):
    """Whole solves with the one-launch-per-level sweeps (graph-captured),
    with the checks of the other solve cases."""
    monkeypatch.setenv("MPK_TRSV_MODE", "s")
    p = case(name)
    b = orc.spmv(p.row_ptr, p.col_idx, p.val, p.x_true_limbs(K))
    ref = orc.krylov(method, p.row_ptr, p.col_idx, p.val, b, kf=kf, tol_rel=tol, max_iter=3000,
                     hist_len=3000)
    assert ref["status"] == 0, ref["status"]
    A = mpk.Csr.from_problem(p)
    x, info = mpk.krylov_solve(method, A, dev(b), fprec=kf, tol_rel=tol, max_iter=3000,
                               hist_len=3000)
    assert info["status"] == "ok", info
    rel = true_relres(orc, p, host(x), b)
    assert rel <= tol * RES_MARGIN, (rel, tol)
    assert abs(info["iters"] - ref["iters"]) <= max(3, 0.05 * ref["iters"])
    h, ho = host(info["hist"]), ref["hist"]
    m = min(20, len(h), len(ho))
    assert np.allclose(h[:m], ho[:m], rtol=1e-12, atol=0)


def test_solve_breakdown_and_max_iter(mpk, orc):
    A = mpk.Csr([0, 2, 4], [0, 1, 0, 1], [0.0, 1.0, 1.0, 0.0])
    b = np.zeros((2, 1, 2))
    b[0, 0, 0] = 1.0
    for m in ("cgs", "bicgstab", "gpbicg", "bicg"):
        x, info = mpk.krylov_solve(m, A, dev(b), fprec=0, tol_rel=1e-25, max_iter=10)
        ref = orc.krylov(m, [0, 2, 4], [0, 1, 0, 1], [0.0, 1.0, 1.0, 0.0], b, kf=0,
                         tol_rel=1e-25, max_iter=10)
        assert info["status"] == "breakdown", m
        assert info["iters"] == ref["iters"], m
    p = case("conv2d")
    b = orc.spmv(p.row_ptr, p.col_idx, p.val, p.x_true_limbs(2))
    A = mpk.Csr.from_problem(p)
    x, info = mpk.krylov_solve("bicgstab", A, dev(b), fprec=1, tol_rel=1e-20, max_iter=3)
    assert info["status"] == "not_converged" and info["iters"] == 3


def test_graph_and_stream_paths_agree(mpk, orc):
    p = case("conv3d")
    b = orc.spmv(p.row_ptr, p.col_idx, p.val, p.x_true_limbs(2))
    A = mpk.Csr.from_problem(p)
    x1, i1 = mpk.krylov_solve("bicgstab", A, dev(b), fprec=1, tol_rel=1e-25, max_iter=500,
                              graph=True)
    x2, i2 = mpk.krylov_solve("bicgstab", A, dev(b), fprec=1, tol_rel=1e-25, max_iter=500,
                              graph=False)
    assert i1["iters"] == i2["iters"]
    assert np.array_equal(host(x1), host(x2))


GRID_METHODS = ["bicg", "cgs", "bicgstab", "gpbicg"]
GRID_PRECS = [(2, 1e-25), (4, 1e-50)]


@pytest.fixture(scope="module")
def conv3d_grid(orc):
    """The 32^3 system and the oracle's solves of every grid case, run on
    host threads (the oracle's calls release the interpreter lock)."""
    import concurrent.futures as cf
    p = W.config2(32)
    bs = {K: orc.spmv(p.row_ptr, p.col_idx, p.val, p.x_true_limbs(K)) for K, _ in GRID_PRECS}
    keys = [(m, K, tol, kf) for m in GRID_METHODS for K, tol in GRID_PRECS for kf in (1, 2)]
    with cf.ThreadPoolExecutor(16) as ex:
        refs = list(ex.map(lambda k: orc.krylov(k[0], p.row_ptr, p.col_idx, p.val, bs[k[1]],
                                                kf=k[3], tol_rel=k[2], max_iter=3000,
                                                hist_len=3000), keys))
    return p, bs, dict(zip(keys, refs))


@pytest.mark.parametrize("method", GRID_METHODS)
@pytest.mark.parametrize("K,tol", GRID_PRECS)
@pytest.mark.parametrize("kf", [1, 2])
def test_solve_parity_conv3d_grid(mpk, orc, conv3d_grid, method, K, tol, kf):
    """The 3D convection-diffusion family (7-point upwind, Peclet 100,
    seeded wind) at 32^3: every method in DD to 1e-25 and in QD to 1e-50,
    with a binary64 and a double-word ILU(0) factor (the "_d_ILU(0)" and
    "ILU(0)" variants of Section 4), against the oracle's solve."""
    p, bs, refs = conv3d_grid
    b, ref = bs[K], refs[(method, K, tol, kf)]
    assert ref["status"] == 0, ref["status"]
    A = mpk.Csr.from_problem(p)
    x, info = mpk.krylov_solve(method, A, dev(b), fprec=kf, tol_rel=tol, max_iter=3000,
                               hist_len=3000)
    assert info["status"] == "ok", info
    rel = true_relres(orc, p, host(x), b)
    assert rel <= tol * RES_MARGIN, (rel, tol)
    assert abs(info["iters"] - ref["iters"]) <= max(3, 0.05 * ref["iters"]), (info["iters"],
                                                                             ref["iters"])
    h, ho = host(info["hist"]), ref["hist"]
    m = min(20, len(h), len(ho))
    assert np.allclose(h[:m], ho[:m], rtol=1e-12, atol=0)
