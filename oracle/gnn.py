"""CPU oracle of the learned correction to the ILU(0) factor.

TEST INFRASTRUCTURE ONLY: plain float64 numpy, written from the definition
below; only the tests, ``__graft_entry__.smoke()`` and the CPU baseline of
``bench.py`` may use it.  It shares no code with the HIP path.

The paper has no learned part; this is the network the library defines on
top of the paper's ILU(0) (Alg. 1) and its Krylov methods, stated once here
and once (independently) in the HIP kernels:

Graph.  Nodes are the rows i of A, edges the stored entries q = (i, j) of A
in CSR order (the diagonal included), so the network's output has exactly
the ILU(0) pattern.  ``row[q] = i``, ``col[q] = j``, ``deg[i]`` = stored
entries of row i.

Inputs (computed in float64, handed to the network as float32):
  node i:  [log|a_ii|, sum_{j!=i}|a_ij| / |a_ii|, log(|u_ii| / |a_ii|), deg_i / 8]
  edge q:  [a_ij / |a_ii|, (l_ij if j < i else u_ij / |a_ii|), [j < i], [j > i]]
where l, u are the plain binary64 ILU(0) factor values (Alg. 1).

Network (hidden width 32, three message-passing layers):
  h0_i = R(relu(Wn x_i + bn)),  e0_q = R(relu(We y_q + be))
  layer l:  z_q   = Wm_l [h_i; h_j; e_q] + bm_l            (Wm rounded to bf16)
            m_q   = R(relu(z_q))
            g_i   = R((sum_{q in row i} m_q) / deg_i)
            u_i   = Wu_l [h_i; g_i] + bu_l                 (Wu rounded to bf16)
            h_i  <- R(h_i + relu(u_i)),   e_q <- R(e_q + m_q)
  delta_q = wd . [h_i; h_j; e_q] + bd                     (float32 weights)
R() is round-to-nearest-even to bfloat16 (the stored activation type); the
oracle applies it in float64 when ``bf16=True``.  Backward treats R as the
identity and uses the forward's rounded weights and activations.

Correction of the binary64 factor: u_ii <- u_ii exp(delta_ii) (sign kept,
never zero), every other value v <- v (1 + tanh(delta_q) / 2).  Guards: a
non-finite delta or corrected value, or a pivot ratio exp(delta_ii) outside
[1e-8, 1e8], rejects the whole correction (the plain factor is kept).

Training loss on probe vectors w_p (normalised residuals of the plain
method): L = mean_p ||A w_p - L~ U~ w_p||^2 / ||A w_p||^2 with L~ unit lower
and U~ upper from the corrected values: a sparse-product (SpMV-shaped)
measure of how far the factor is from A on the directions the iteration
actually meets; it needs no triangular solve.

Parameter vector (float32, this order, row-major matrices [out][in]):
  Wn[32][4], bn[32], We[32][4], be[32],
  3 x (Wm[32][96], bm[32], Wu[32][64], bu[32]),
  wd[96], bd[1]                                     -> 15969 values.
"""
import numpy as np

HID = 32
LAYERS = 3
FN = 4
FE = 4
C_OFF = 0.5
PIVOT_MIN, PIVOT_MAX = 1e-8, 1e8


def _shapes():
    s = [("Wn", (HID, FN)), ("bn", (HID,)), ("We", (HID, FE)), ("be", (HID,))]
    for l in range(LAYERS):
        s += [("Wm%d" % l, (HID, 3 * HID)), ("bm%d" % l, (HID,)),
              ("Wu%d" % l, (HID, 2 * HID)), ("bu%d" % l, (HID,))]
    s += [("wd", (3 * HID,)), ("bd", (1,))]
    return s


SHAPES = _shapes()
NPARAM = sum(int(np.prod(sh)) for _, sh in SHAPES)


def unpack(theta):
    """Flat parameter vector -> dict of float64 arrays (views copied)."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (NPARAM,)
    out, o = {}, 0
    for name, sh in SHAPES:
        k = int(np.prod(sh))
        out[name] = theta[o:o + k].reshape(sh).copy()
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def bf16(x):
    """Round float64 values to the nearest bfloat16 (ties to even), returned
    as float64.  Values are first rounded to float32, as the device holds
    float32 before it stores bfloat16."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    nan = np.isnan(a)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, r)


class Graph:
    """Edge lists of a CSR pattern."""

    def __init__(self, rp, ci):
        self.rp = np.asarray(rp, dtype=np.int64)
        self.ci = np.asarray(ci, dtype=np.int64)
        self.n = len(self.rp) - 1
        self.E = len(self.ci)
        self.deg = np.diff(self.rp).astype(np.float64)
        self.row = np.repeat(np.arange(self.n), np.diff(self.rp))
        self.col = self.ci

    def row_sum(self, v):
        """sum over the edges of each row (edges in CSR order)."""
        out = np.zeros((self.n,) + v.shape[1:])
        np.add.at(out, self.row, v)
        return out

    def col_sum(self, v):
        """sum over the edges that point at each node (column j)."""
        out = np.zeros((self.n,) + v.shape[1:])
        np.add.at(out, self.col, v)
        return out


def features(rp, ci, val, f):
    """Node [n, 4] and edge [E, 4] inputs (float32 values as float64) from
    A's values and the plain ILU(0) factor f (both in A's pattern)."""
    G = Graph(rp, ci)
    val = np.asarray(val, dtype=np.float64).reshape(-1)
    f = np.asarray(f, dtype=np.float64).reshape(-1)
    isd = G.row == G.col
    if np.count_nonzero(isd) != G.n:
        raise ValueError("every diagonal entry must be stored")
    dpos = np.flatnonzero(isd)
    dpos = dpos[np.argsort(G.row[dpos])]
    aii = np.abs(val[dpos])
    uii = np.abs(f[dpos])
    off = G.row_sum(np.where(isd, 0.0, np.abs(val)))
    x = np.stack([np.log(aii), off / aii, np.log(uii / aii), G.deg / 8.0], axis=1)
    lower = G.col < G.row
    upper = G.col > G.row
    ya = val / aii[G.row]
    yf = np.where(lower, f, f / aii[G.row])
    y = np.stack([ya, yf, lower.astype(np.float64), upper.astype(np.float64)], axis=1)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    return f32(x), f32(y)


def forward(theta, rp, ci, x, y, bf16_acts=True):
    """delta[E] and the saved state for backward."""
    P = unpack(theta)
    G = Graph(rp, ci)
    R = bf16 if bf16_acts else (lambda a: np.asarray(a, dtype=np.float64))
    Wr = bf16 if bf16_acts else (lambda a: a)
    relu = lambda a: np.maximum(a, 0.0)
    pre_n = x @ P["Wn"].T + P["bn"]
    pre_e = y @ P["We"].T + P["be"]
    h = R(relu(pre_n))
    e = R(relu(pre_e))
    saved = {"G": G, "x": x, "y": y, "pre_n": pre_n, "pre_e": pre_e, "layers": []}
    for l in range(LAYERS):
        Wm, Wu = Wr(P["Wm%d" % l]), Wr(P["Wu%d" % l])
        X = np.concatenate([h[G.row], h[G.col], e], axis=1)
        z = X @ Wm.T + P["bm%d" % l]
        m = R(relu(z))
        g = R(G.row_sum(m) / G.deg[:, None])
        U = np.concatenate([h, g], axis=1) @ Wu.T + P["bu%d" % l]
        saved["layers"].append({"h": h, "e": e, "z": z, "m": m, "g": g, "u": U,
                                "Wm": Wm, "Wu": Wu})
        h = R(h + relu(U))
        e = R(e + m)
    Xd = np.concatenate([h[G.row], h[G.col], e], axis=1)
    delta = Xd @ P["wd"] + P["bd"][0]
    saved["h"], saved["e"], saved["Xd"] = h, e, Xd
    return delta, saved


def saved_from(theta, rp, ci, x, y, h, e, m, g, r):
    """The saved state backward() needs, built from given stored
    activations instead of a forward pass: h, e (LAYERS + 1 arrays each:
    encoder outputs, then after each layer), m, g and r (LAYERS arrays: the
    messages, the row means and R(relu(u)) of each layer).  backward() uses
    z, u, pre_n and pre_e only through their signs, and those are the signs
    of m, r, h[0] and e[0] (bfloat16 keeps float32's exponent range, so R()
    maps no positive value to zero)."""
    P = unpack(theta)
    G = Graph(rp, ci)
    saved = {"G": G, "x": x, "y": y, "pre_n": h[0], "pre_e": e[0], "layers": []}
    for l in range(LAYERS):
        saved["layers"].append({"h": h[l], "e": e[l], "z": m[l], "m": m[l], "g": g[l],
                                "u": r[l], "Wm": bf16(P["Wm%d" % l]),
                                "Wu": bf16(P["Wu%d" % l])})
    saved["h"], saved["e"] = h[LAYERS], e[LAYERS]
    saved["Xd"] = np.concatenate([h[LAYERS][G.row], h[LAYERS][G.col], e[LAYERS]], axis=1)
    return saved


def backward(theta, saved, gdelta):
    """Gradient of sum_q gdelta_q delta_q with respect to theta (float64)."""
    P = unpack(theta)
    G = saved["G"]
    gdelta = np.asarray(gdelta, dtype=np.float64)
    D = {name: np.zeros(sh) for name, sh in SHAPES}
    D["wd"] = saved["Xd"].T @ gdelta
    D["bd"] = np.array([gdelta.sum()])
    dX = np.outer(gdelta, P["wd"])
    dh = G.row_sum(dX[:, :HID]) + G.col_sum(dX[:, HID:2 * HID])
    de = dX[:, 2 * HID:]
    for l in reversed(range(LAYERS)):
        S = saved["layers"][l]
        h, e, z, m, g, U = S["h"], S["e"], S["z"], S["m"], S["g"], S["u"]
        dU = dh * (U > 0)
        D["Wu%d" % l] = dU.T @ np.concatenate([h, g], axis=1)
        D["bu%d" % l] = dU.sum(axis=0)
        dXu = dU @ S["Wu"]
        dh_new = dh + dXu[:, :HID]
        dg = dXu[:, HID:]
        dm = de + (dg / G.deg[:, None])[G.row]
        dz = dm * (z > 0)
        X = np.concatenate([h[G.row], h[G.col], e], axis=1)
        D["Wm%d" % l] = dz.T @ X
        D["bm%d" % l] = dz.sum(axis=0)
        dXm = dz @ S["Wm"]
        dh_new = dh_new + G.row_sum(dXm[:, :HID]) + G.col_sum(dXm[:, HID:2 * HID])
        de = de + dXm[:, 2 * HID:]
        dh = dh_new
    dzn = dh * (saved["pre_n"] > 0)
    dze = de * (saved["pre_e"] > 0)
    D["Wn"] = dzn.T @ saved["x"]
    D["bn"] = dzn.sum(axis=0)
    D["We"] = dze.T @ saved["y"]
    D["be"] = dze.sum(axis=0)
    return pack(D)


def corrected(rp, ci, f, delta):
    """Corrected factor values (no guards)."""
    G = Graph(rp, ci)
    f = np.asarray(f, dtype=np.float64).reshape(-1)
    delta = np.asarray(delta, dtype=np.float64)
    isd = G.row == G.col
    with np.errstate(over="ignore", invalid="ignore"):
        return np.where(isd, f * np.exp(delta), f * (1.0 + C_OFF * np.tanh(delta)))


def correct(rp, ci, f, delta):
    """(fell_back, values): the guarded correction."""
    G = Graph(rp, ci)
    f = np.asarray(f, dtype=np.float64).reshape(-1)
    delta = np.asarray(delta, dtype=np.float64)
    isd = G.row == G.col
    v = corrected(rp, ci, f, delta)
    with np.errstate(over="ignore", invalid="ignore"):
        ratio = np.exp(delta[isd])
    bad = (not np.all(np.isfinite(delta))) or (not np.all(np.isfinite(v))) or \
        np.any(ratio < PIVOT_MIN) or np.any(ratio > PIVOT_MAX)
    return (1, f.copy()) if bad else (0, v)


def _lu_products(G, v, w):
    """y = U~ w, z = L~ y with L~ unit lower, U~ upper from values v."""
    lower = G.col < G.row
    y = np.zeros(G.n)
    np.add.at(y, G.row[~lower], v[~lower] * w[G.col[~lower]])
    z = y.copy()
    np.add.at(z, G.row[lower], v[lower] * y[G.col[lower]])
    return y, z


def factor_loss(rp, ci, val, f, delta, probes):
    """(loss, dloss/ddelta) of the probe loss above, in float64."""
    G = Graph(rp, ci)
    val = np.asarray(val, dtype=np.float64).reshape(-1)
    f = np.asarray(f, dtype=np.float64).reshape(-1)
    delta = np.asarray(delta, dtype=np.float64)
    probes = np.atleast_2d(np.asarray(probes, dtype=np.float64))
    isd = G.row == G.col
    lower = G.col < G.row
    v = corrected(rp, ci, f, delta)
    th = np.tanh(delta)
    dv_dd = np.where(isd, v, f * C_OFF * (1.0 - th * th))
    P = len(probes)
    loss = 0.0
    gv = np.zeros(G.E)
    for w in probes:
        Aw = np.zeros(G.n)
        np.add.at(Aw, G.row, val * w[G.col])
        y, z = _lu_products(G, v, w)
        e = Aw - z
        s = Aw @ Aw
        loss += (e @ e) / s
        gz = -2.0 * e / (s * P)
        # dz/dl_ij = y_j (row i);  dL/dy = L~^T gz;  dy/du_ij = w_j (row i)
        gy = gz.copy()
        np.add.at(gy, G.col[lower], v[lower] * gz[G.row[lower]])
        gv += np.where(lower, gz[G.row] * y[G.col], gy[G.row] * w[G.col])
    return loss / P, gv * dv_dd


def adam(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, Alg. 1, with bias correction)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
