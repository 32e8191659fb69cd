"""GPU parity of the learned ILU(0) correction against the CPU oracle
(oracle/gnn.py): network forward and backward (bfloat16 activations,
float32 weights), the float64 factor loss and its gradient, Adam, the
guarded correction, and solves with a supplied factor."""
import numpy as np
import pytest

from paper_2504_14498_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_14498_amd import mpk as m
    m.library()
    return m


@pytest.fixture(scope="module")
def gnn():
    from oracle import gnn as g
    return g


def dev(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def host(t):
    return t.detach().cpu().numpy()


def problem(name):
    if name == "lognormal23":      # ragged tiles: n = 529
        return W.config5(3, m=23)
    if name == "lognormal64":
        return W.config5(7, m=64)
    if name == "random37":
        return W.random_pattern(37, 0.15, 5, dominance=1.5)
    raise KeyError(name)


def theta(seed, gnn, scale=0.25):
    rng = np.random.default_rng(seed)
    return (scale * rng.standard_normal(gnn.NPARAM)).astype(np.float32)


def setup(mpk, orc, p):
    val = p.val.reshape(-1)
    A = mpk.Csr(p.row_ptr, p.col_idx, val)
    M = mpk.ilu0_factor(A, fprec=1, vprec=2)
    G = mpk.GnnGraph(A, M)
    st, bad, f = orc.ilu0(p.row_ptr, p.col_idx, val.reshape(-1, 1), 1, 1)
    assert st == 0
    return A, M, G, val, f.reshape(-1)


def rel_err(got, ref):
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def cosine(a, b):
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


NAMES = ["random37", "lognormal23", "lognormal64"]


@pytest.mark.parametrize("name", NAMES)
def test_forward_matches_oracle(mpk, orc, gnn, name):
    p = problem(name)
    A, M, G, val, f = setup(mpk, orc, p)
    th = theta(11, gnn)
    delta, _ = mpk.gnn_forward(G, dev(th))
    x, y = gnn.features(p.row_ptr, p.col_idx, val, f)
    ref, _ = gnn.forward(th.astype(np.float64), p.row_ptr, p.col_idx, x, y, bf16_acts=True)
    got = host(delta).astype(np.float64)
    assert np.all(np.isfinite(got))
    # float32 accumulation against float64, with the same bf16 storage points
    assert rel_err(got, ref) <= 1e-3, rel_err(got, ref)
    assert cosine(got, ref) >= 0.999
    assert np.std(ref) > 1e-3


def test_initial_parameters_predict_zero(mpk, orc, gnn):
    p = problem("lognormal23")
    A, M, G, val, f = setup(mpk, orc, p)
    th = mpk.gnn_init(5)
    assert th.numel() == gnn.NPARAM
    delta, _ = mpk.gnn_forward(G, th)
    assert np.array_equal(host(delta), np.zeros(A.nnz, dtype=np.float32))
    # weights bounded by 1/sqrt(fan_in), biases zero
    P = gnn.unpack(host(th).astype(np.float64))
    assert np.all(np.abs(P["Wm0"]) <= 1 / np.sqrt(96)) and np.any(P["Wm0"] != 0)
    assert np.all(P["bm0"] == 0) and np.all(P["wd"] == 0)


def device_activations(mpk, G, ws, gnn):
    """The activations the device's last forward stored (bfloat16), as
    float64 arrays: h and e for every layer boundary, m, g and r per
    layer."""
    def get(which, layer):
        u = host(mpk.gnn_saved(G, ws, which, layer)).view(np.uint16).astype(np.uint32)
        return (u << 16).view(np.float32).astype(np.float64)
    L = gnn.LAYERS
    return ([get("h", l) for l in range(L + 1)], [get("e", l) for l in range(L + 1)],
            [get("m", l) for l in range(L)], [get("g", l) for l in range(L)],
            [get("r", l) for l in range(L)])


@pytest.mark.parametrize("name", NAMES)
def test_backward_matches_oracle(mpk, orc, gnn, name):
    """The device's parameter gradient against the oracle's float64
    backward started from the activations the device itself stored, so
    both differentiate the same bfloat16 values: relative norm error at
    most 1e-3 and cosine at least 0.999, overall and per parameter group.
    The stored activations are themselves the oracle forward's, up to
    values that float32 accumulation moved across a bfloat16 rounding
    boundary."""
    p = problem(name)
    A, M, G, val, f = setup(mpk, orc, p)
    th = theta(12, gnn)
    gd = np.random.default_rng(3).standard_normal(A.nnz).astype(np.float32)
    delta, ws = mpk.gnn_forward(G, dev(th))
    dp = host(mpk.gnn_backward(G, dev(th), dev(gd), ws)).astype(np.float64)
    x, y = gnn.features(p.row_ptr, p.col_idx, val, f)
    h, e, m, g, r = device_activations(mpk, G, ws, gnn)
    # the stored activations follow the oracle's forward (same storage
    # points), apart from rounding-boundary crossings
    _, S = gnn.forward(th.astype(np.float64), p.row_ptr, p.col_idx, x, y, bf16_acts=True)
    assert rel_err(h[gnn.LAYERS], S["h"]) <= 1e-2
    assert rel_err(e[gnn.LAYERS], S["e"]) <= 1e-2
    saved = gnn.saved_from(th.astype(np.float64), p.row_ptr, p.col_idx, x, y, h, e, m, g, r)
    ref = gnn.backward(th.astype(np.float64), saved, gd.astype(np.float64))
    assert rel_err(dp, ref) <= 1e-3, rel_err(dp, ref)
    assert cosine(dp, ref) >= 0.999
    Pg, Pr = gnn.unpack(dp), gnn.unpack(ref)
    for k in Pr:
        if np.linalg.norm(Pr[k]) > 1e-6 * np.linalg.norm(ref):
            err = rel_err(Pg[k].ravel(), Pr[k].ravel())
            assert err <= 1e-3, (k, err)
            assert cosine(Pg[k].ravel(), Pr[k].ravel()) >= 0.999, k


@pytest.mark.parametrize("name", NAMES)
def test_factor_loss_matches_oracle(mpk, orc, gnn, name):
    p = problem(name)
    A, M, G, val, f = setup(mpk, orc, p)
    rng = np.random.default_rng(21)
    delta = (0.3 * rng.standard_normal(A.nnz)).astype(np.float32)
    probes = rng.standard_normal((3, A.n))
    loss, gd, _ = mpk.gnn_factor_loss(G, M, dev(delta), dev(probes))
    ref_loss, ref_gd = gnn.factor_loss(p.row_ptr, p.col_idx, val, f,
                                       delta.astype(np.float64), probes)
    assert abs(float(host(loss)) - ref_loss) <= 1e-12 * ref_loss
    got = host(gd).astype(np.float64)
    assert np.max(np.abs(got - ref_gd)) <= 1e-6 * np.max(np.abs(ref_gd))
    # no gradient requested: same loss
    loss2, none, _ = mpk.gnn_factor_loss(G, M, dev(delta), dev(probes), grad=False)
    assert none is None and float(host(loss2)) == float(host(loss))


def test_factor_loss_zero_on_exact_lu(mpk, orc):
    # tridiagonal: ILU(0) is the exact LU, so delta = 0 leaves nothing
    n = 300
    rp = np.concatenate([[0], np.cumsum([2] + [3] * (n - 2) + [2])]).astype(np.int32)
    ci, val = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                ci.append(j)
                val.append(3.0 if i == j else -1.0 - 0.001 * i)
    A = mpk.Csr(rp, np.array(ci, dtype=np.int32), np.array(val))
    M = mpk.ilu0_factor(A, fprec=1, vprec=2)
    G = mpk.GnnGraph(A, M)
    probes = np.random.default_rng(1).standard_normal((2, n))
    loss, gd, _ = mpk.gnn_factor_loss(G, M, dev(np.zeros(A.nnz, np.float32)), dev(probes))
    assert float(host(loss)) < 1e-28
    assert np.max(np.abs(host(gd))) < 1e-12


def test_adam_matches_oracle(mpk, gnn):
    rng = np.random.default_rng(4)
    n = 1000
    th = rng.standard_normal(n).astype(np.float32)
    p, m, v = dev(th), dev(np.zeros(n, np.float32)), dev(np.zeros(n, np.float32))
    rt, rm, rv = th.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in range(1, 6):
        g = rng.standard_normal(n).astype(np.float32)
        mpk.gnn_adam(p, dev(g), m, v, step, lr=1e-2)
        rt, rm, rv = gnn.adam(rt, g.astype(np.float64), rm, rv, step, lr=1e-2)
    assert np.max(np.abs(host(p) - rt)) <= 1e-5 * max(1.0, np.max(np.abs(rt)))


@pytest.mark.parametrize("name", ["lognormal23", "lognormal64"])
def test_correction_matches_oracle(mpk, orc, gnn, name):
    p = problem(name)
    A, M, G, val, f = setup(mpk, orc, p)
    rng = np.random.default_rng(5)
    delta = (0.4 * rng.standard_normal(A.nnz)).astype(np.float32)
    assert mpk.ilu0_correct(M, dev(delta)) is False
    fb, fc = gnn.correct(p.row_ptr, p.col_idx, f, delta.astype(np.float64))
    assert fb == 0
    r = rng.standard_normal((A.n, 1, 2))
    r[:, :, 1] *= 1e-17
    got = host(mpk.ilu0_apply(M, dev(r)))
    ref = orc.ilu0_apply(p.row_ptr, p.col_idx, fc.reshape(-1, 1, 1), r)
    # exp and tanh may differ by an ulp between the device and numpy
    err = np.max(np.abs(got[:, 0, 0] - ref[:, 0, 0])) / np.max(np.abs(ref[:, 0, 0]))
    assert err <= 1e-12, err


@pytest.mark.parametrize("bad", ["nan_offdiag", "inf_diag", "big_pivot", "tiny_pivot"])
def test_correction_guards_keep_plain_factor(mpk, orc, bad):
    p = problem("lognormal23")
    A, M, G, val, f = setup(mpk, orc, p)
    M_ref = mpk.ilu0_factor(A, fprec=1, vprec=2)
    rows = np.repeat(np.arange(A.n), np.diff(p.row_ptr))
    dpos = np.flatnonzero(rows == p.col_idx)
    opos = np.flatnonzero(rows != p.col_idx)
    delta = np.full(A.nnz, 0.01, dtype=np.float32)
    if bad == "nan_offdiag":
        delta[opos[7]] = np.nan
    elif bad == "inf_diag":
        delta[dpos[3]] = np.inf
    elif bad == "big_pivot":
        delta[dpos[-1]] = 18.5        # exp(18.5) > 1e8
    else:
        delta[dpos[0]] = -18.5
    assert mpk.ilu0_correct(M, dev(delta)) is True
    r = np.random.default_rng(2).standard_normal((A.n, 1, 2))
    a = host(mpk.ilu0_apply(M, dev(r)))
    b = host(mpk.ilu0_apply(M_ref, dev(r)))
    assert np.array_equal(a, b)
    # just inside the bound is accepted
    ok = np.zeros(A.nnz, dtype=np.float32)
    ok[dpos[0]] = 18.0
    assert mpk.ilu0_correct(M, dev(ok)) is False


def test_precond_solve_equals_plain_solve(mpk, orc):
    p = problem("lognormal64")
    A = mpk.Csr.from_problem(p)
    import torch
    xt = torch.as_tensor(p.x_true_limbs(2)).cuda()
    b = mpk.csr_spmv(A, xt)
    M = mpk.ilu0_factor(A, fprec=1, vprec=2)
    x1, i1 = mpk.krylov_solve("bicgstab", A, b, fprec=1, tol_rel=1e-25, max_iter=3000)
    x2, i2 = mpk.krylov_solve_precond("bicgstab", A, M, b, tol_rel=1e-25, max_iter=3000)
    assert i1["status"] == i2["status"] == "ok"
    assert i1["iters"] == i2["iters"]
    assert np.array_equal(host(x1), host(x2))
    # wrong factor / precision declarations are rejected before any work
    M1 = mpk.ilu0_factor(A, fprec=1, vprec=1)
    with pytest.raises(mpk.MpkError):
        mpk.krylov_solve_precond("bicgstab", A, M1, b)
    with pytest.raises(mpk.MpkError):
        mpk.krylov_solve_precond("bicg", A, M, b)


def test_solve_with_corrected_factor_matches_oracle(mpk, orc, gnn):
    p = problem("lognormal64")
    A, M, G, val, f = setup(mpk, orc, p)
    rng = np.random.default_rng(8)
    delta = (0.1 * rng.standard_normal(A.nnz)).astype(np.float32)
    assert mpk.ilu0_correct(M, dev(delta)) is False
    fb, fc = gnn.correct(p.row_ptr, p.col_idx, f, delta.astype(np.float64))
    bh = orc.spmv(p.row_ptr, p.col_idx, val.reshape(-1, 1), p.x_true_limbs(2))
    x, info = mpk.krylov_solve_precond("bicgstab", A, M, dev(bh), tol_rel=1e-25, max_iter=3000)
    ref = orc.krylov("bicgstab", p.row_ptr, p.col_idx, val.reshape(-1, 1), bh, kf=1,
                     tol_rel=1e-25, max_iter=3000, factor=fc)
    assert ref["status"] == 0 and info["status"] == "ok"
    assert abs(info["iters"] - ref["iters"]) <= 1
    assert info["relres_true"] < 1e-25
    err = np.max(np.abs(host(x)[:, 0, 0] - p.x_true))
    assert err < 1e-20


def test_short_training_lowers_the_loss(mpk):
    from paper_2504_14498_amd import learned
    insts = [learned.Instance(W.config5(s, m=32)) for s in range(4)]
    tr = learned.Trainer(seed=1, lr=3e-3)
    before = [float(tr.loss(i)) for i in insts]
    for epoch in range(15):
        for inst in insts:
            tr.step(inst)
    after = [float(tr.loss(i)) for i in insts]
    assert np.all(np.isfinite(after))
    assert np.mean(after) < 0.9 * np.mean(before), (before, after)


def test_trained_network_gains_over_plain_ilu0(mpk):
    """Train on 32 small lognormal systems (64^2), then solve 8 held-out
    ones to 1e-25 with the learned and the plain factor.  The plain method
    is the judge: the learned factor must not need more passes at the
    median, every solve must converge, and the fallback rule must hold."""
    from paper_2504_14498_amd import learned
    train = [learned.Instance(W.config5(s, m=64), seed=s) for s in range(32)]
    tr = learned.Trainer(seed=1, lr=2e-3)
    for epoch in range(4):
        for inst in train:
            tr.step(inst)
    plain_train = [learned.solve_plain(i.A, i.b)[1]["iters"] for i in train[:8]]
    cap = learned.iteration_cap(plain_train)
    ratios = []
    for s in range(8):
        inst = learned.Instance(W.config5(100_000 + s, m=64), probes=False)
        _, ip = learned.solve_plain(inst.A, inst.b)
        _, il = learned.solve_learned(inst.A, inst.b, tr.params, cap)
        assert ip["status"] == "ok" and il["status"] == "ok"
        assert il["relres_true"] < 1e-25
        if il["fallback"] is None:
            assert il["iters_total"] <= cap
        ratios.append(il["iters_total"] / ip["iters"])
    print("learned/plain pass ratios on held-out systems:", np.round(ratios, 3))
    assert np.median(ratios) < 1.0, ratios
