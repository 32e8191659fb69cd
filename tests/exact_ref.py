"""Exact rational (Gaussian-rational for complex) reference arithmetic used
to pin the oracle.  Test helper only: it is not the oracle and shares no
code with it or with the HIP path."""
from fractions import Fraction as F

import numpy as np


class Q:
    """Gaussian rational re + i im with Fraction parts."""
    __slots__ = ("re", "im")

    def __init__(self, re=0, im=0):
        self.re = F(re)
        self.im = F(im)

    def __add__(self, o):
        o = _q(o)
        return Q(self.re + o.re, self.im + o.im)

    __radd__ = __add__

    def __sub__(self, o):
        o = _q(o)
        return Q(self.re - o.re, self.im - o.im)

    def __rsub__(self, o):
        return _q(o) - self

    def __neg__(self):
        return Q(-self.re, -self.im)

    def __mul__(self, o):
        o = _q(o)
        return Q(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    __rmul__ = __mul__

    def __truediv__(self, o):
        o = _q(o)
        d = o.re * o.re + o.im * o.im
        n = self * o.conj()
        return Q(n.re / d, n.im / d)

    def __rtruediv__(self, o):
        return _q(o) / self

    def conj(self):
        return Q(self.re, -self.im)

    def is_zero(self):
        return self.re == 0 and self.im == 0

    def __eq__(self, o):
        o = _q(o)
        return self.re == o.re and self.im == o.im

    def __hash__(self):
        return hash((self.re, self.im))

    def abs2(self):
        return self.re * self.re + self.im * self.im

    def __complex__(self):
        return complex(float(self.re), float(self.im))

    def __repr__(self):
        return "Q(%s, %s)" % (self.re, self.im)


def _q(o):
    if isinstance(o, Q):
        return o
    if isinstance(o, complex):
        return Q(F(o.real), F(o.imag))
    return Q(o, 0)


def limbs_to_q(x):
    """(C, K) float limbs -> Q (exact sum of limbs)."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        return Q(sum(F(v) for v in x), 0)
    re = sum(F(v) for v in x[0])
    im = sum(F(v) for v in x[1]) if x.shape[0] > 1 else F(0)
    return Q(re, im)


def vec_to_q(x):
    """(n, C, K) float array -> list of Q."""
    return [limbs_to_q(x[i]) for i in range(x.shape[0])]


def csr_to_dense_q(rp, ci, val, n, C):
    """Dense list-of-lists of Q (None where not stored)."""
    A = [[None] * n for _ in range(n)]
    val = np.asarray(val, dtype=np.float64).reshape(-1, C)
    for i in range(n):
        for p in range(rp[i], rp[i + 1]):
            re = F(val[p, 0])
            im = F(val[p, 1]) if C == 2 else F(0)
            A[i][ci[p]] = Q(re, im)
    return A


def matvec(A, x):
    n = len(x)
    return [sum((A[i][j] * x[j] for j in range(n) if A[i][j] is not None), Q()) for i in range(n)]


def matvec_h(A, x):
    n = len(x)
    return [sum((A[j][i].conj() * x[j] for j in range(n) if A[j][i] is not None), Q())
            for i in range(n)]


def dot(a, b):
    return sum((ai.conj() * bi for ai, bi in zip(a, b)), Q())


def ilu0_literal(A):
    """Algorithm 1 taken literally (KIJ, structural nonzeros), exact."""
    n = len(A)
    W = [[A[i][j] for j in range(n)] for i in range(n)]
    L = [[Q(1) if i == j else None for j in range(n)] for i in range(n)]
    U = [[None] * n for _ in range(n)]
    for k in range(n):
        ukk = W[k][k]
        if ukk is None or ukk.is_zero():
            continue
        U[k][k] = ukk
        for i in range(k + 1, n):
            if W[i][k] is None:
                continue
            L[i][k] = W[i][k] / ukk
            for j in range(k + 1, n):
                if W[k][j] is not None and W[i][j] is not None:
                    W[i][j] = W[i][j] - L[i][k] * W[k][j]
        for j in range(k + 1, n):
            if W[k][j] is not None:
                U[k][j] = W[k][j]
    return L, U


def lu_solve(L, U, r):
    n = len(r)
    y = [None] * n
    for i in range(n):
        s = r[i]
        for j in range(i):
            if L[i][j] is not None:
                s = s - L[i][j] * y[j]
        y[i] = s
    z = [None] * n
    for i in range(n - 1, -1, -1):
        s = y[i]
        for j in range(i + 1, n):
            if U[i][j] is not None:
                s = s - U[i][j] * z[j]
        z[i] = s / U[i][i]
    return z


def lu_solve_h(L, U, r):
    """(L U)^{-H} r = L^{-H} U^{-H} r."""
    n = len(r)
    w = [None] * n
    for i in range(n):
        s = r[i]
        for j in range(i):
            if U[j][i] is not None:
                s = s - U[j][i].conj() * w[j]
        w[i] = s / U[i][i].conj()
    z = [None] * n
    for i in range(n - 1, -1, -1):
        s = w[i]
        for j in range(i + 1, n):
            if L[j][i] is not None:
                s = s - L[j][i].conj() * z[j]
        z[i] = s
    return z


def _axpy(x, a, y):
    return [xi + a * yi for xi, yi in zip(x, y)]


def _is_zero_vec(v):
    return all(vi.is_zero() for vi in v)


def bicg(A, b, passes, M=None):
    """Algorithm 3 (preconditioned BiCG), exact.  Returns per-pass dicts."""
    n = len(b)
    P = (lambda v: lu_solve(*M, v)) if M else (lambda v: list(v))
    PH = (lambda v: lu_solve_h(*M, v)) if M else (lambda v: list(v))
    x = [Q() for _ in range(n)]
    r = list(b)
    rt = list(r)
    z, zt = P(r), PH(rt)
    p, pt = list(z), list(zt)
    rho = dot(zt, r)
    out = []
    for _ in range(passes):
        q = matvec(A, p)
        qt = matvec_h(A, pt)
        d = dot(pt, q)
        if d.is_zero():
            break
        alpha = rho / d
        x = _axpy(x, alpha, p)
        r = _axpy(r, -alpha, q)
        rt = _axpy(rt, -alpha.conj(), qt)
        out.append({"alpha": alpha, "x": x, "r": r})
        if _is_zero_vec(r):
            break
        z, zt = P(r), PH(rt)
        rho_new = dot(zt, r)
        beta = rho_new / rho
        out[-1]["beta"] = beta
        p = _axpy(z, beta, p)
        pt = _axpy(zt, beta.conj(), pt)
        rho = rho_new
    return out


def cgs(A, b, passes, M=None):
    n = len(b)
    P = (lambda v: lu_solve(*M, v)) if M else (lambda v: list(v))
    x = [Q() for _ in range(n)]
    r = list(b)
    rt = list(r)
    out = []
    q = p = None
    rho_old = None
    for k in range(1, passes + 1):
        rho = dot(rt, r)
        if rho.is_zero():
            break
        if k == 1:
            u = list(r)
            p = list(u)
        else:
            beta = rho / rho_old
            out[-1]["beta"] = beta
            u = _axpy(r, beta, q)
            p = _axpy(u, beta, _axpy(q, beta, p))
        ph = P(p)
        v = matvec(A, ph)
        sigma = dot(rt, v)
        if sigma.is_zero():
            break
        alpha = rho / sigma
        q = _axpy(u, -alpha, v)
        uh = P([a + c for a, c in zip(u, q)])
        x = _axpy(x, alpha, uh)
        r = _axpy(r, -alpha, matvec(A, uh))
        out.append({"alpha": alpha, "x": x, "r": r})
        if _is_zero_vec(r):
            break
        rho_old = rho
    return out


def bicgstab(A, b, passes, M=None):
    n = len(b)
    P = (lambda v: lu_solve(*M, v)) if M else (lambda v: list(v))
    x = [Q() for _ in range(n)]
    r = list(b)
    rt = list(r)
    out = []
    p = v = None
    rho_old = alpha = omega = None
    for k in range(1, passes + 1):
        rho = dot(rt, r)
        if rho.is_zero():
            break
        if k == 1:
            p = list(r)
        else:
            beta = (rho / rho_old) * (alpha / omega)
            out[-1]["beta"] = beta
            p = _axpy(r, beta, _axpy(p, -omega, v))
        ph = P(p)
        v = matvec(A, ph)
        sigma = dot(rt, v)
        if sigma.is_zero():
            break
        alpha = rho / sigma
        s = _axpy(r, -alpha, v)
        if _is_zero_vec(s):
            x = _axpy(x, alpha, ph)
            out.append({"alpha": alpha, "x": x, "r": s, "omega": Q()})
            break
        sh = P(s)
        t = matvec(A, sh)
        omega = dot(t, s) / dot(t, t)
        x = _axpy(_axpy(x, alpha, ph), omega, sh)
        r = _axpy(s, -omega, t)
        out.append({"alpha": alpha, "omega": omega, "x": x, "r": r})
        if _is_zero_vec(r) or omega.is_zero():
            break
        rho_old = rho
    return out


def gpbicg(A, b, passes, M=None, force_eta_zero=False):
    n = len(b)
    P = (lambda v: lu_solve(*M, v)) if M else (lambda v: list(v))
    zero = [Q() for _ in range(n)]
    x = list(zero)
    r = list(b)
    rt = list(r)
    beta = Q()
    told, w, u, p = list(zero), list(zero), list(zero), list(zero)
    phold, thold, zh = list(zero), list(zero), list(zero)
    rho = dot(rt, r)
    out = []
    for k in range(1, passes + 1):
        p = _axpy(r, beta, [a - c for a, c in zip(p, u)])
        ph = P(p)
        q = matvec(A, ph)
        sig = dot(rt, q)
        if sig.is_zero():
            break
        alpha = rho / sig
        y = _axpy(_axpy([a - c for a, c in zip(told, r)], -alpha, w), alpha, q)
        t = _axpy(r, -alpha, q)
        if _is_zero_vec(t):
            # exact termination inside the pass: x + alpha p^ solves A x = b
            x = _axpy(x, alpha, ph)
            out.append({"alpha": alpha, "zeta": Q(), "eta": Q(), "x": x, "r": t})
            break
        th = P(t)
        s = matvec(A, th)
        ss, st_ = dot(s, s), dot(s, t)
        if k == 1 or force_eta_zero:
            zeta, eta = st_ / ss, Q()
        else:
            yy, sy, ys, yt = dot(y, y), dot(s, y), dot(y, s), dot(y, t)
            den = ss * yy - sy * ys
            zeta = (yy * st_ - sy * yt) / den
            eta = (ss * yt - ys * st_) / den
        tmp = _axpy([a - c for a, c in zip(told, r)], beta, u)
        u = [zeta * a + eta * c for a, c in zip(q, tmp)]
        vh = _axpy(_axpy(_axpy(zh, -alpha, thold), -(alpha * beta), phold), alpha, ph)
        zh = [zeta * a + eta * c for a, c in zip(th, vh)]
        x = [a + c for a, c in zip(_axpy(x, alpha, ph), zh)]
        r = _axpy(_axpy(t, -eta, y), -zeta, s)
        out.append({"alpha": alpha, "zeta": zeta, "eta": eta, "x": x, "r": r})
        if _is_zero_vec(r) or zeta.is_zero():
            break
        rho_new = dot(rt, r)
        beta = (alpha / zeta) * (rho_new / rho)
        out[-1]["beta"] = beta
        w = _axpy(s, beta, q)
        told, phold, thold = t, ph, th
        rho = rho_new
    return out


def cg(A, b, passes):
    """Textbook conjugate gradients (Hestenes-Stiefel), exact."""
    n = len(b)
    x = [Q() for _ in range(n)]
    r = list(b)
    p = list(r)
    rr = dot(r, r)
    out = []
    for _ in range(passes):
        q = matvec(A, p)
        alpha = rr / dot(p, q)
        x = _axpy(x, alpha, p)
        r = _axpy(r, -alpha, q)
        out.append({"alpha": alpha, "x": x, "r": r})
        rr_new = dot(r, r)
        if rr_new.is_zero():
            break
        p = _axpy(r, rr_new / rr, p)
        rr = rr_new
    return out
