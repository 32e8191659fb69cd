"""Pins of the learned-correction oracle (oracle/gnn.py) against things that
do not come from it: a library bfloat16 conversion, hand-computed features,
a brute-force per-edge evaluation of the network, central finite
differences, the exact LU of a no-fill matrix, dense matrix products and a
library Adam."""
import numpy as np
import pytest

from oracle import gnn


def tiny_pattern(n, seed, density=0.35):
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < density
    np.fill_diagonal(mask, True)
    val = rng.standard_normal((n, n))
    off = np.where(mask, np.abs(val), 0.0)
    np.fill_diagonal(off, 0.0)
    val[np.arange(n), np.arange(n)] = 1.5 * off.sum(1) + 1.0
    rows, cols = np.nonzero(mask)
    rp = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(mask.sum(1), out=rp[1:])
    return rp, cols.astype(np.int32), val[rows, cols].copy()


def random_theta(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return (scale * rng.standard_normal(gnn.NPARAM)).astype(np.float32).astype(np.float64)


def plain_factor(rp, ci, val):
    import oracle
    st, bad, f = oracle.ilu0(rp, ci, val.reshape(-1, 1), 1, 1)
    assert st == 0
    return f.reshape(-1)


def test_param_count():
    assert gnn.NPARAM == 2 * (32 * 4 + 32) + 3 * (32 * 96 + 32 + 32 * 64 + 32) + 96 + 1


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 65504.0, 3e38,
                         1e-40, -1e-42, np.inf, -np.inf]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = gnn.bf16(x)
    assert np.array_equal(got, ref)
    assert np.isnan(gnn.bf16(np.array([np.nan]))[0])


def test_features_by_hand():
    # 3x3: row 0 = [4, -1, 0], row 1 = [-2, 5, -1], row 2 = [0, -1, 3]
    rp = np.array([0, 2, 5, 7], dtype=np.int32)
    ci = np.array([0, 1, 0, 1, 2, 1, 2], dtype=np.int32)
    val = np.array([4.0, -1.0, -2.0, 5.0, -1.0, -1.0, 3.0])
    f = plain_factor(rp, ci, val)
    # ILU(0) by hand (tridiagonal: exact LU): u00 = 4, l10 = -0.5, u11 = 5 - 0.5 = 4.5,
    # l21 = -1/4.5, u22 = 3 - 1/4.5
    assert np.allclose(f, [4.0, -1.0, -0.5, 4.5, -1.0, -1 / 4.5, 3 - 1 / 4.5], rtol=1e-15)
    x, y = gnn.features(rp, ci, val, f)
    f32 = lambda a: np.float64(np.float32(a))
    assert np.array_equal(x[1], [f32(np.log(5.0)), f32(3.0 / 5.0), f32(np.log(4.5 / 5.0)),
                                 f32(3 / 8)])
    assert np.array_equal(x[2], [f32(np.log(3.0)), f32(1 / 3), f32(np.log((3 - 1 / 4.5) / 3)),
                                 f32(2 / 8)])
    # edge (1,0): lower, feature = l_10;  edge (1,2): upper, u_12 / |a_11|
    assert np.array_equal(y[2], [f32(-2 / 5), f32(-0.5), 1.0, 0.0])
    assert np.array_equal(y[3], [1.0, f32(4.5 / 5), 0.0, 0.0])
    assert np.array_equal(y[4], [f32(-1 / 5), f32(-1 / 5), 0.0, 1.0])


def brute_forward(theta, rp, ci, x, y, bf16_acts):
    """The network evaluated one node and one edge at a time with Python
    loops, from the definition in the oracle's docstring."""
    P = gnn.unpack(theta)
    R = gnn.bf16 if bf16_acts else (lambda a: np.asarray(a, dtype=np.float64))
    n = len(rp) - 1
    edges = [(i, int(ci[q])) for i in range(n) for q in range(rp[i], rp[i + 1])]
    relu = lambda v: np.maximum(v, 0)
    h = [R(relu(P["Wn"] @ x[i] + P["bn"])) for i in range(n)]
    e = [R(relu(P["We"] @ y[q] + P["be"])) for q in range(len(edges))]
    for l in range(3):
        Wm = gnn.bf16(P["Wm%d" % l]) if bf16_acts else P["Wm%d" % l]
        Wu = gnn.bf16(P["Wu%d" % l]) if bf16_acts else P["Wu%d" % l]
        m = []
        for q, (i, j) in enumerate(edges):
            m.append(R(relu(Wm[:, :32] @ h[i] + Wm[:, 32:64] @ h[j] + Wm[:, 64:] @ e[q]
                            + P["bm%d" % l])))
        hn = []
        for i in range(n):
            qs = [q for q, (a, _) in enumerate(edges) if a == i]
            s = np.zeros(32)
            for q in qs:
                s = s + m[q]
            g = R(s / len(qs))
            u = Wu[:, :32] @ h[i] + Wu[:, 32:] @ g + P["bu%d" % l]
            hn.append(R(h[i] + relu(u)))
        e = [R(e[q] + m[q]) for q in range(len(edges))]
        h = hn
    return np.array([P["wd"][:32] @ h[i] + P["wd"][32:64] @ h[j] + P["wd"][64:] @ e[q]
                     + P["bd"][0] for q, (i, j) in enumerate(edges)])


@pytest.mark.parametrize("bf", [False, True])
def test_forward_vs_brute_force(bf):
    rp, ci, val = tiny_pattern(9, 3)
    f = plain_factor(rp, ci, val)
    x, y = gnn.features(rp, ci, val, f)
    th = random_theta(4)
    d, _ = gnn.forward(th, rp, ci, x, y, bf16_acts=bf)
    ref = brute_forward(th, rp, ci, x, y, bf)
    assert np.allclose(d, ref, rtol=1e-12, atol=1e-12)
    assert np.std(d) > 1e-3


def test_backward_vs_finite_differences():
    rp, ci, val = tiny_pattern(8, 5)
    f = plain_factor(rp, ci, val)
    x, y = gnn.features(rp, ci, val, f)
    th = random_theta(6)
    rng = np.random.default_rng(7)
    gd = rng.standard_normal(len(ci))
    _, S = gnn.forward(th, rp, ci, x, y, bf16_acts=False)
    g = gnn.backward(th, S, gd)
    obj = lambda t: gd @ gnn.forward(t, rp, ci, x, y, bf16_acts=False)[0]
    eps = 1e-6
    # every parameter of the encoders, decoder and one layer, plus random directions
    P = gnn.unpack(np.arange(gnn.NPARAM, dtype=np.float64))
    idx = np.concatenate([P["Wn"].ravel(), P["bn"], P["We"].ravel(), P["Wm1"].ravel()[::37],
                          P["bu2"], P["wd"], P["bd"]]).astype(int)
    for k in idx:
        t1, t2 = th.copy(), th.copy()
        t1[k] += eps
        t2[k] -= eps
        fd = (obj(t1) - obj(t2)) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])
    for _ in range(5):
        v = rng.standard_normal(gnn.NPARAM)
        fd = (obj(th + eps * v) - obj(th - eps * v)) / (2 * eps)
        assert abs(fd - g @ v) <= 1e-6 * max(1.0, abs(fd))


def test_backward_from_stored_activations_equals_forward_state():
    """backward() started from the stored bfloat16 activations alone (the
    state a device keeps) gives the same gradient as from the forward's
    full state: its masks only need the signs of m, R(relu(u)), h0, e0."""
    rp, ci, val = tiny_pattern(30, 8, density=0.2)
    f = plain_factor(rp, ci, val)
    x, y = gnn.features(rp, ci, val, f)
    th = random_theta(9)
    gd = np.random.default_rng(10).standard_normal(len(ci))
    _, S = gnn.forward(th, rp, ci, x, y, bf16_acts=True)
    L = S["layers"]
    relu = lambda a: np.maximum(a, 0.0)
    h = [l["h"] for l in L] + [S["h"]]
    e = [l["e"] for l in L] + [S["e"]]
    m = [l["m"] for l in L]
    g = [l["g"] for l in L]
    r = [gnn.bf16(relu(l["u"])) for l in L]
    assert all(np.any(v == 0) and np.any(v > 0) for v in r + m)
    saved = gnn.saved_from(th, rp, ci, x, y, h, e, m, g, r)
    assert np.array_equal(gnn.backward(th, saved, gd), gnn.backward(th, S, gd))


def tridiag(n, seed):
    rng = np.random.default_rng(seed)
    rp = [0]
    ci, val = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                ci.append(j)
                val.append(4.0 + rng.random() if i == j else -1.0 + 0.5 * rng.random())
        rp.append(len(ci))
    return np.array(rp, dtype=np.int32), np.array(ci, dtype=np.int32), np.array(val)


def test_loss_zero_on_exact_lu():
    rp, ci, val = tridiag(40, 1)
    f = plain_factor(rp, ci, val)
    W = np.random.default_rng(2).standard_normal((3, 40))
    loss, g = gnn.factor_loss(rp, ci, val, f, np.zeros(len(ci)), W)
    assert loss < 1e-28
    assert np.max(np.abs(g)) < 1e-13


def dense(rp, ci, v, n):
    M = np.zeros((n, n))
    for i in range(n):
        M[i, ci[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    return M


def test_loss_vs_dense_products_and_fd():
    rp, ci, val = tiny_pattern(12, 9, density=0.3)
    n = 12
    f = plain_factor(rp, ci, val)
    rng = np.random.default_rng(3)
    delta = 0.3 * rng.standard_normal(len(ci))
    W = rng.standard_normal((4, n))
    loss, g = gnn.factor_loss(rp, ci, val, f, delta, W)
    v = gnn.corrected(rp, ci, f, delta)
    F = dense(rp, ci, v, n)
    Lm = np.tril(F, -1) + np.eye(n)
    Um = np.triu(F)
    A = dense(rp, ci, val, n)
    ref = np.mean([np.sum((A @ w - Lm @ Um @ w) ** 2) / np.sum((A @ w) ** 2) for w in W])
    assert abs(loss - ref) <= 1e-13 * ref
    assert loss > 1e-4
    # the sparse pattern and the dense matrices agree at delta = 0 on the ILU identity:
    # (L U)_ij = a_ij on the pattern
    F0 = dense(rp, ci, f, n)
    LU0 = (np.tril(F0, -1) + np.eye(n)) @ np.triu(F0)
    mask = dense(rp, ci, np.ones(len(ci)), n) > 0
    assert np.allclose(LU0[mask], A[mask], rtol=1e-13, atol=1e-13)
    eps = 1e-6
    for k in range(len(ci)):
        d1, d2 = delta.copy(), delta.copy()
        d1[k] += eps
        d2[k] -= eps
        fd = (gnn.factor_loss(rp, ci, val, f, d1, W)[0] -
              gnn.factor_loss(rp, ci, val, f, d2, W)[0]) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(fd), 1e-3), (k, fd, g[k])


def test_correction_formula_and_guards():
    rp, ci, val = tiny_pattern(10, 11)
    f = plain_factor(rp, ci, val)
    E = len(ci)
    G = gnn.Graph(rp, ci)
    isd = G.row == G.col
    fb, v = gnn.correct(rp, ci, f, np.zeros(E))
    assert fb == 0 and np.array_equal(v, f)
    d = np.full(E, 0.7)
    fb, v = gnn.correct(rp, ci, f, d)
    assert fb == 0
    assert np.allclose(v[isd], f[isd] * np.exp(0.7), rtol=1e-15)
    assert np.allclose(v[~isd], f[~isd] * (1 + 0.5 * np.tanh(0.7)), rtol=1e-15)
    assert np.all(np.sign(v[isd]) == np.sign(f[isd]))
    # off-diagonals stay within [v/2, 3v/2] however large delta is
    fb, v = gnn.correct(rp, ci, f, np.where(isd, 0.0, 1e6))
    assert fb == 0 and np.allclose(v[~isd], 1.5 * f[~isd])
    for bad in (np.nan, np.inf, 18.5, -18.5):
        dd = np.zeros(E)
        dd[np.flatnonzero(isd)[3]] = bad
        fb, v = gnn.correct(rp, ci, f, dd)
        assert fb == 1 and np.array_equal(v, f)
    dd = np.zeros(E)
    dd[np.flatnonzero(isd)[3]] = 18.0          # exp(18) = 6.6e7: accepted
    assert gnn.correct(rp, ci, f, dd)[0] == 0
    dd = np.zeros(E)
    dd[np.flatnonzero(~isd)[0]] = np.nan
    assert gnn.correct(rp, ci, f, dd)[0] == 1


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    th = rng.standard_normal(50)
    p = torch.nn.Parameter(torch.tensor(th.copy()))
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    for step in range(1, 7):
        g = rng.standard_normal(50)
        p.grad = torch.tensor(g.copy())
        opt.step()
        th, m, v = gnn.adam(th, g, m, v, step, lr=3e-3)
        assert np.allclose(th, p.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_end_to_end_gradient_vs_fd():
    rp, ci, val = tiny_pattern(10, 13, density=0.3)
    f = plain_factor(rp, ci, val)
    x, y = gnn.features(rp, ci, val, f)
    W = np.random.default_rng(1).standard_normal((3, 10))
    th = random_theta(8, scale=0.2)

    def obj(t):
        d, S = gnn.forward(t, rp, ci, x, y, bf16_acts=False)
        return gnn.factor_loss(rp, ci, val, f, d, W)[0], d, S

    L0, d, S = obj(th)
    gd = gnn.factor_loss(rp, ci, val, f, d, W)[1]
    g = gnn.backward(th, S, gd)
    rng = np.random.default_rng(2)
    eps = 1e-6
    for _ in range(4):
        v = rng.standard_normal(gnn.NPARAM)
        fd = (obj(th + eps * v)[0] - obj(th - eps * v)[0]) / (2 * eps)
        assert abs(fd - g @ v) <= 1e-6 * max(abs(fd), 1e-3)
