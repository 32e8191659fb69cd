"""MatrixMarket reading and writing, and the paper's right-hand side, for
the replication harness (no GPU): round trips of the repository's own
generators, symmetric / skew-symmetric / hermitian expansion against dense
matrices, added zero diagonals, rejected inputs, and x = sqrt(2) i
(sqrt(2 + 3i) i) to the working precision."""
import decimal

import numpy as np
import pytest

from paper_2504_14498_amd import mtx
from paper_2504_14498_amd import workloads as W
from paper_2504_14498_amd.replicate import paper_x


def dense(p):
    n = p.n
    D = np.zeros((n, n), dtype=complex)
    v = p.val.reshape(-1, p.C)
    for i in range(n):
        for q in range(p.row_ptr[i], p.row_ptr[i + 1]):
            D[i, p.col_idx[q]] = v[q, 0] + (1j * v[q, 1] if p.C == 2 else 0)
    return D


@pytest.mark.parametrize("prob", ["conv2d", "helm", "rdd", "rand_cplx"])
def test_round_trip(tmp_path, prob):
    p = {"conv2d": lambda: W.config1(9), "helm": lambda: W.config3(7),
         "rdd": lambda: W.random_dd(300, 4),
         "rand_cplx": lambda: W.random_pattern(80, 0.05, 3, complex_=True, dominance=1.2)}[prob]()
    f = tmp_path / "a.mtx"
    mtx.write(f, p, comment="test matrix\nsecond line")
    q = mtx.read(f)
    assert q.n == p.n and q.C == p.C
    assert np.array_equal(q.row_ptr, p.row_ptr) and np.array_equal(q.col_idx, p.col_idx)
    assert np.array_equal(q.val, p.val)        # 17 digits read back exactly
    assert q.meta["added_diagonal"] == 0


def _write(path, header, size, entries):
    with open(path, "w") as f:
        f.write(header + "\n% a comment\n" + size + "\n")
        for e in entries:
            f.write(e + "\n")


def test_symmetric_expansions(tmp_path):
    rng = np.random.default_rng(1)
    n = 6
    L = np.tril(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)), -1)
    L[np.abs(L) < 0.8] = 0
    d = rng.standard_normal(n)
    ent = [(i, j) for i in range(n) for j in range(i) if L[i, j] != 0]
    # complex symmetric (like dwg961b): A = L + L^T + diag
    f = tmp_path / "s.mtx"
    _write(f, "%%MatrixMarket matrix coordinate complex symmetric", "%d %d %d" % (n, n, len(ent) + n),
           ["%d %d %.17g %.17g" % (i + 1, j + 1, L[i, j].real, L[i, j].imag) for i, j in ent] +
           ["%d %d %.17g 0" % (i + 1, i + 1, d[i]) for i in range(n)])
    assert np.array_equal(dense(mtx.read(f)), L + L.T + np.diag(d))
    # hermitian: A = L + L^H + diag
    f = tmp_path / "h.mtx"
    _write(f, "%%MatrixMarket matrix coordinate complex hermitian", "%d %d %d" % (n, n, len(ent) + n),
           ["%d %d %.17g %.17g" % (i + 1, j + 1, L[i, j].real, L[i, j].imag) for i, j in ent] +
           ["%d %d %.17g 0" % (i + 1, i + 1, d[i]) for i in range(n)])
    assert np.array_equal(dense(mtx.read(f)), L + L.conj().T + np.diag(d))
    # real skew-symmetric: no diagonal in the file; zeros added
    f = tmp_path / "k.mtx"
    Lr = L.real
    ent = [(i, j) for i in range(n) for j in range(i) if Lr[i, j] != 0]
    _write(f, "%%MatrixMarket matrix coordinate real skew-symmetric", "%d %d %d" % (n, n, len(ent)),
           ["%d %d %.17g" % (i + 1, j + 1, Lr[i, j]) for i, j in ent])
    q = mtx.read(f)
    assert np.array_equal(dense(q).real, Lr - Lr.T)
    assert q.meta["added_diagonal"] == n
    # pattern and integer fields, unsorted entries
    f = tmp_path / "p.mtx"
    _write(f, "%%MatrixMarket matrix coordinate pattern general", "3 3 4", ["3 1", "1 1", "2 2", "3 3"])
    q = mtx.read(f)
    assert list(q.row_ptr) == [0, 1, 2, 4] and list(q.col_idx) == [0, 1, 0, 2]
    assert np.all(q.val == 1)
    f = tmp_path / "i.mtx"
    _write(f, "%%MatrixMarket matrix coordinate integer general", "2 2 3", ["2 2 -4", "1 2 7", "1 1 3"])
    assert np.array_equal(dense(mtx.read(f)).real, [[3, 7], [0, -4]])


@pytest.mark.parametrize("header,size,entries", [
    ("%%MatrixMarket matrix array real general", "2 2", ["1", "2", "3", "4"]),
    ("%%MatrixMarket matrix coordinate real general", "2 3 1", ["1 1 1"]),
    ("%%MatrixMarket matrix coordinate real general", "2 2 2", ["1 1 1", "1 1 2"]),
    ("%%MatrixMarket matrix coordinate real general", "2 2 1", ["3 1 1"]),
    ("%%MatrixMarket matrix coordinate real symmetric", "2 2 1", ["1 2 1"]),
    ("%%MatrixMarket matrix coordinate real general", "2 2 2", ["1 1 1"]),
    ("%%MatrixMarket matrix coordinate real general", "2 2 1", ["1 1 nan"]),
])
def test_rejected(tmp_path, header, size, entries):
    f = tmp_path / "bad.mtx"
    _write(f, header, size, entries)
    with pytest.raises(mtx.MtxError):
        mtx.read(f)


@pytest.mark.parametrize("C,K", [(1, 2), (1, 4), (2, 3), (2, 4)])
def test_paper_rhs_solution(C, K):
    """x_i = s i with s = sqrt(2) or sqrt(2 + 3i): the limbs sum to the
    exact value within the format's unit, and s^2 = 2 (2 + 3i)."""
    n = 50
    x = paper_x(n, C, K)
    ctx = decimal.Context(prec=150)
    u = 2.0 ** (-53 * K + 2)
    for i in (0, 1, 17, n - 1):
        comps = []
        for c in range(C):
            v = decimal.Decimal(0)
            for limb in x[i, c]:
                v = ctx.add(v, decimal.Decimal(limb))      # exact at 150 digits
            comps.append(v)
        s = [ctx.divide(v, decimal.Decimal(i + 1)) for v in comps]
        if C == 1:
            assert abs(float(ctx.subtract(ctx.multiply(s[0], s[0]), 2))) <= 4 * u
        else:
            re = ctx.subtract(ctx.multiply(s[0], s[0]), ctx.multiply(s[1], s[1]))
            im = ctx.multiply(2, ctx.multiply(s[0], s[1]))
            assert abs(float(re - 2)) <= 8 * u and abs(float(im - 3)) <= 8 * u
        # limbs are non-overlapping and decreasing
        for c in range(C):
            for k in range(K - 1):
                assert abs(x[i, c, k + 1]) <= abs(x[i, c, k]) * 2.0 ** -52
