"""Pins of the oracle's exact residual r = b - A x (the check on a solution
behind the stopping rule of Algorithm 3): against exact rational
arithmetic, on cancellations down to exact zero, across the whole binary64
exponent range, and for complex matrices."""
from fractions import Fraction as F

import numpy as np
import pytest


def limbs_value(v):
    return sum((F(float(t)) for t in v), F(0))


def exact_residual(rp, ci, val, b, x):
    """b - A x in Fractions; returns (n, C) list of Fractions."""
    n, C, _ = b.shape
    out = []
    for i in range(n):
        if C == 1:
            acc = limbs_value(b[i, 0])
            for p in range(rp[i], rp[i + 1]):
                acc -= F(float(val[p])) * limbs_value(x[ci[p], 0])
            out.append([acc])
        else:
            re, im = limbs_value(b[i, 0]), limbs_value(b[i, 1])
            for p in range(rp[i], rp[i + 1]):
                ar, ai = F(float(val[p, 0])), F(float(val[p, 1]))
                xr, xi = limbs_value(x[ci[p], 0]), limbs_value(x[ci[p], 1])
                re -= ar * xr - ai * xi
                im -= ar * xi + ai * xr
            out.append([re, im])
    return out


def random_csr(rng, n, per_row, C):
    rp, ci = [0], []
    for i in range(n):
        cols = sorted(set(rng.choice(n, size=per_row, replace=True).tolist()) | {i})
        ci.extend(cols)
        rp.append(len(ci))
    nnz = len(ci)
    val = rng.standard_normal((nnz, C)) if C == 2 else rng.standard_normal(nnz)
    return np.array(rp, np.int32), np.array(ci, np.int32), val


def limbs(rng, n, C, K, scale=1.0):
    x = np.zeros((n, C, K))
    v = scale * rng.uniform(-1, 1, (n, C))
    for k in range(K):
        x[:, :, k] = v
        v = v * rng.uniform(0.5, 1.0, (n, C)) * 2.0 ** -53
    return x


def assert_close(r, ref):
    for got, want in zip(np.asarray(r).reshape(-1), [q for row in ref for q in row]):
        if want == 0:
            assert got == 0.0
        else:
            # the conversion is within two units in the last place
            assert abs(F(float(got)) - want) <= abs(want) * F(2) ** -51, (got, float(want))


@pytest.mark.parametrize("C", [1, 2])
@pytest.mark.parametrize("kb,kx", [(1, 1), (2, 2), (2, 4), (4, 3), (3, 1)])
def test_residual_matches_exact_rationals(orc, C, kb, kx):
    rng = np.random.default_rng(10 * C + kb + 7 * kx)
    n = 25
    rp, ci, val = random_csr(rng, n, 4, C)
    b = limbs(rng, n, C, kb)
    x = limbs(rng, n, C, kx)
    r = orc.residual(rp, ci, val, b, x)
    assert_close(r, exact_residual(rp, ci, val, b, x))


@pytest.mark.parametrize("C", [1, 2])
def test_residual_of_an_exact_product_is_zero(orc, C):
    """b = A x with small integers is exact in binary64: r must be exactly
    zero, whatever the summation order; and moving b by one unit in its
    lowest limb must show up exactly."""
    rng = np.random.default_rng(3 + C)
    n = 40
    rp, ci, _ = random_csr(rng, n, 5, C)
    val = rng.integers(-9, 10, (len(ci), C)).astype(np.float64)
    if C == 1:
        val = val[:, 0]
    x = np.zeros((n, C, 2))
    x[:, :, 0] = rng.integers(-1000, 1000, (n, C))
    x[:, :, 1] = x[:, :, 0] * 2.0 ** -60   # exact, a second limb far below
    ex = exact_residual(rp, ci, val, np.zeros((n, C, 1)), x)
    # b holds -(A x) split into two limbs (hi, lo) exactly
    b = np.zeros((n, C, 2))
    for i in range(n):
        for c in range(C):
            v = -ex[i][c]
            hi = float(v)
            b[i, c, 0] = hi
            b[i, c, 1] = float(v - F(hi))
            assert F(b[i, c, 0]) + F(b[i, c, 1]) == v
    r = orc.residual(rp, ci, val, b, x)
    assert np.all(r == 0.0)
    b2 = b.copy()
    b2[7, 0, 1] += 2.0 ** -200
    r2 = orc.residual(rp, ci, val, b2, x)
    want = F(b2[7, 0, 1]) - F(b[7, 0, 1])
    assert F(float(r2[7, 0])) == want
    r2[7, 0] = 0.0
    assert np.all(r2 == 0.0)


def test_residual_across_the_exponent_range(orc):
    """Huge terms that cancel exactly next to tiny ones (subnormal limbs
    and products far below binary64's range): only the tiny part
    remains."""
    big, tiny = 2.0 ** 900, 2.0 ** -1070
    rp = np.array([0, 2, 3], np.int32)       # row 0: columns 0 and 1; row 1: column 1
    ci = np.array([0, 1, 1], np.int32)
    val = np.array([big, -big, 1.0])
    x = np.zeros((2, 1, 3))
    x[0, 0] = [1.0, 2.0 ** -80, tiny]
    x[1, 0] = [1.0, 2.0 ** -80, 0.0]
    b = np.zeros((2, 1, 2))
    b[0, 0] = [0.0, 3 * tiny]
    b[1, 0] = [1.0, 2.0 ** -80]
    r = orc.residual(rp, ci, val, b, x)
    ref = exact_residual(rp, ci, val, b, x)
    # row 0: 3 tiny - big * tiny (the leading limbs' products cancel)
    assert ref[0][0] == 3 * F(tiny) - F(big) * F(tiny)
    assert_close(r, ref)
    assert r[1, 0] == 0.0


def test_true_relres_definition(orc):
    """true_relres is ||b - A x|| / ||b|| in the 2-norm, with both
    vectors from the exact residual."""
    rng = np.random.default_rng(5)
    n = 30
    rp, ci, val = random_csr(rng, n, 3, 1)
    b = limbs(rng, n, 1, 2)
    x = limbs(rng, n, 1, 2)
    ex = exact_residual(rp, ci, val, b, x)
    nr = np.sqrt(sum(float(q[0]) ** 2 for q in ex))
    nb = np.sqrt(sum(float(limbs_value(b[i, 0])) ** 2 for i in range(n)))
    assert abs(orc.true_relres(rp, ci, val, b, x) - nr / nb) <= 1e-14 * nr / nb
