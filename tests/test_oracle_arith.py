"""Pins for the oracle's multi-component arithmetic (not GPU).

The paper fixes the formats (DD, TD, QD: 2, 3, 4 binary64 components,
Section 2) but not the algorithms.  These tests check the oracle against
exact rational arithmetic: error-free transforms must be exact, double-word
operations must meet the error bounds proved by Joldes, Muller and Popescu
(ACM TOMS 2017) for the algorithms used, and the truncated expansions for
TD/QD must stay within a small multiple of u^K."""
from fractions import Fraction as F

import numpy as np
import pytest

U = 2.0 ** -53


def fr(x):
    return sum(F(float(v)) for v in np.asarray(x).reshape(-1))


def rand_mp(rng, orc, K, scale=1.0):
    t = [rng.uniform(-1, 1) * scale]
    for _ in range(K + 1):
        t.append(t[-1] * rng.uniform(-1, 1) * 2.0 ** -53)
    return orc.renorm(np.array(t), K)


ADVERSARIAL = [
    (1.0, 2.0 ** -53), (1.0, -2.0 ** -54), (1e308, 1e292), (3.0, -3.0), (5e-324, 5e-324),
    (2.0 ** -1022, -2.0 ** -1074), (1.0 + 2.0 ** -52, -1.0), (0.1, 0.2), (1e16, 1.0),
    (-7.5, 2.0 ** 60), (0.0, -0.0),
]


def test_two_sum_exact(orc):
    rng = np.random.default_rng(0)
    pairs = list(ADVERSARIAL)
    for _ in range(2000):
        a = rng.standard_normal() * 10.0 ** rng.integers(-30, 30)
        b = rng.standard_normal() * 10.0 ** rng.integers(-30, 30)
        pairs.append((a, b))
    for a, b in pairs:
        s, e = orc.two_sum(a, b)
        assert F(s) + F(e) == F(a) + F(b)
        assert s == a + b


def test_two_prod_exact(orc):
    rng = np.random.default_rng(1)
    # TwoProd is exact only without underflow: |a b| >= 2^-969 (or a b == 0 exactly)
    pairs = [(a, b) for a, b in ADVERSARIAL
             if abs(a * b) < 1e300 and (a == 0 or b == 0 or abs(a * b) > 2.0 ** -960)]
    for _ in range(2000):
        pairs.append((rng.standard_normal() * 10.0 ** rng.integers(-100, 100),
                      rng.standard_normal() * 10.0 ** rng.integers(-100, 100)))
    for a, b in pairs:
        p, e = orc.two_prod(a, b)
        assert F(p) + F(e) == F(a) * F(b)


@pytest.mark.parametrize("m,K", [(2, 2), (3, 3), (4, 4), (3, 4), (1, 3)])
def test_renorm_exact_when_no_truncation(orc, m, K):
    rng = np.random.default_rng(m * 10 + K)
    for _ in range(500):
        t = rng.standard_normal(m) * 10.0 ** rng.integers(-20, 20, size=m)
        z = orc.renorm(t, K)
        assert fr(z) == fr(t)


# Proven relative error bounds of the double-word algorithms (units of u^2).
DW_BOUNDS = {"add": 3.0, "mul_fp": 2.0, "mul": 4.0, "div_fp": 3.0, "div": 15.0}
# Measured-constant bounds for the truncated expansions (units of u^K); the
# measured maxima are about 1.4 (add), 1.2 (mul), 0.7 (div).
EX_BOUNDS = {"add": 4.0, "mul_fp": 4.0, "mul": 4.0, "div_fp": 4.0, "div": 4.0}


@pytest.mark.parametrize("K", [2, 3, 4])
def test_ops_error_bounds(orc, K):
    rng = np.random.default_rng(100 + K)
    B = DW_BOUNDS if K == 2 else EX_BOUNDS
    unit = U ** K
    worst = dict.fromkeys(B, 0.0)
    for trial in range(1500):
        x = rand_mp(rng, orc, K)
        y = rand_mp(rng, orc, K, float(rng.choice([1.0, 1e-9, 1e9, 1e-200])))
        if trial % 4 == 0:
            y = -x.copy()
            y[-1] *= 1 + rng.uniform(-1e-3, 1e-3)
            y = orc.renorm(y, K)
        ex = fr(x) + fr(y)
        z = orc.add(x, y)
        if ex != 0:
            worst["add"] = max(worst["add"], float(abs(fr(z) - ex) / abs(ex)))
        y = rand_mp(rng, orc, K, float(rng.choice([1.0, 1e-9, 1e9])))
        ex = fr(x) * fr(y)
        worst["mul"] = max(worst["mul"], float(abs(fr(orc.mul(x, y)) - ex) / abs(ex)))
        a = rng.uniform(-1, 1) * 10.0 ** rng.integers(-5, 5)
        ex = fr(x) * F(a)
        worst["mul_fp"] = max(worst["mul_fp"], float(abs(fr(orc.mul_fp(x, a)) - ex) / abs(ex)))
        ex = fr(x) / fr(y)
        worst["div"] = max(worst["div"], float(abs(fr(orc.div_k(x, y)) - ex) / abs(ex)))
        ex = fr(x) / F(a)
        worst["div_fp"] = max(worst["div_fp"],
                              float(abs(fr(orc.div_k(x, np.array([a]))) - ex) / abs(ex)))
    for k, bound in B.items():
        assert worst[k] <= bound * unit * (1 + 1e-6), (k, worst[k] / unit)


@pytest.mark.parametrize("K", [3, 4])
def test_mixed_factor_products(orc, K):
    """A double-word factor times a K-limb vector value, and the division by
    a double-word pivot (mixed precision ILU(0) substitutions, Section 3)."""
    rng = np.random.default_rng(7 + K)
    for _ in range(500):
        x = rand_mp(rng, orc, K)
        f = rand_mp(rng, orc, 2, 3.0)
        ex = fr(x) * fr(f)
        assert abs(fr(orc.mul_k(x, f)) - ex) <= 4 * U ** K * abs(ex)
        ex = fr(x) / fr(f)
        assert abs(fr(orc.div_k(x, f)) - ex) <= 4 * U ** K * abs(ex)


def test_k1_is_binary64(orc):
    rng = np.random.default_rng(3)
    for _ in range(200):
        a, b = rng.standard_normal(2)
        assert orc.add([a], [b])[0] == a + b
        assert orc.mul([a], [b])[0] == a * b
        assert orc.div_k([a], [b])[0] == a / b


@pytest.mark.parametrize("K", [1, 2, 4])
def test_complex_mul_div(orc, K):
    """Complex product and quotient (x conj(d) / |d|^2) against exact Gaussian
    rationals; the quotient is checked componentwise against |x|/|d|."""
    rng = np.random.default_rng(20 + K)
    tol = 8 * U ** K
    for _ in range(300):
        s = np.stack([rand_mp(rng, orc, K), rand_mp(rng, orc, K)])
        x = np.stack([rand_mp(rng, orc, K), rand_mp(rng, orc, K)])
        sr, si, xr, xi = fr(s[0]), fr(s[1]), fr(x[0]), fr(x[1])
        z = orc.cmul(s, x)
        er, ei = sr * xr - si * xi, sr * xi + si * xr
        mag = (abs(sr) + abs(si)) * (abs(xr) + abs(xi))
        assert abs(fr(z[0]) - er) <= tol * mag
        assert abs(fr(z[1]) - ei) <= tol * mag
        q = orc.cdiv(x, s)
        d2 = sr * sr + si * si
        qr, qi = (xr * sr + xi * si) / d2, (xi * sr - xr * si) / d2
        qmag = (abs(xr) + abs(xi)) * (abs(sr) + abs(si)) / d2
        assert abs(fr(q[0]) - qr) <= 4 * tol * qmag
        assert abs(fr(q[1]) - qi) <= 4 * tol * qmag


@pytest.mark.parametrize("K", [2, 3, 4])
def test_complex_div_outside_the_squared_range(orc, K):
    """x / d for denominators far from 1 (|d| ~ 2^-700 .. 2^700, where |d|^2
    leaves the binary64 range): the quotient equals the exact Gaussian
    rational quotient within the same bound as near 1, and equals, bit for
    bit, the quotient of the same operands brought near 1 by powers of two
    (multiplying by a power of two is exact in binary64)."""
    rng = np.random.default_rng(40 + K)
    tol = 32 * U ** K
    for shift_d, shift_x in [(-700, -700), (-600, -650), (-400, 0), (500, 480), (700, 700),
                             (-350, -300), (310, 330), (200, 150), (-250, -260)]:
        for _ in range(40):
            s = np.stack([rand_mp(rng, orc, K), rand_mp(rng, orc, K)])
            x = np.stack([rand_mp(rng, orc, K), rand_mp(rng, orc, K)])
            q1 = orc.cdiv(x, s)
            q = orc.cdiv(np.ldexp(x, shift_x), np.ldexp(s, shift_d))
            assert np.all(np.isfinite(q))
            assert np.array_equal(q, np.ldexp(q1, shift_x - shift_d))
            sr, si = fr(np.ldexp(s[0], shift_d)), fr(np.ldexp(s[1], shift_d))
            xr, xi = fr(np.ldexp(x[0], shift_x)), fr(np.ldexp(x[1], shift_x))
            d2 = sr * sr + si * si
            qr, qi = (xr * sr + xi * si) / d2, (xi * sr - xr * si) / d2
            qmag = (abs(xr) + abs(xi)) * (abs(sr) + abs(si)) / d2
            assert abs(fr(q[0]) - qr) <= tol * qmag
            assert abs(fr(q[1]) - qi) <= tol * qmag
