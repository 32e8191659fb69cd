"""Seeded synthetic inputs: sparse matrices in CSR and exact solutions.

This module only builds problems (matrix entries, x_true); it holds none of
the solver's arithmetic, so the HIP path and the oracle can both use it.
All randomness comes from numpy's PCG64 generator with the stated seeds.

CSR layout: row_ptr int32[n+1], col_idx int32[nnz] (ascending, unique per
row, the diagonal always stored), val float64[nnz] (real) or
float64[nnz, 2] ((re, im), complex).  Grid unknowns are numbered in natural
lexicographic order, x fastest; Dirichlet boundary values are eliminated.

The paper measured on two SuiteSparse matrices (mcfe, dwg961b; Section 4)
that are not available here; these generators stand in for them with the
shapes of the workloads the method is benchmarked on: convection-diffusion
stencils (real, nonsymmetric), a complex shifted Helmholtz stencil, random
diagonally dominant systems of uneven size, and a variable-coefficient
convection-diffusion family.
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    name: str
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray          # (nnz,) real or (nnz, 2) complex
    x_true: np.ndarray       # (n,) real or (n, 2) complex, binary64
    meta: dict = field(default_factory=dict)

    @property
    def C(self):
        return 2 if self.val.ndim == 2 else 1

    @property
    def nnz(self):
        return int(self.row_ptr[-1])

    def val_flat(self):
        return np.ascontiguousarray(self.val, dtype=np.float64).reshape(-1)

    def x_true_limbs(self, K):
        """x_true as a (n, C, K) multi-limb array (lower limbs zero)."""
        x = np.zeros((self.n, self.C, K))
        x[:, :, 0] = self.x_true.reshape(self.n, self.C)
        return x


def stencil_csr(shape, offsets, coeffs):
    """CSR of a constant- or variable-coefficient stencil on a grid.

    shape: grid dims (nx, ny[, nz]), x fastest.  offsets: list of integer
    tuples, ordered so that their linear offsets ascend.  coeffs: list of
    scalars or per-point arrays (grid shape, possibly complex) per offset.
    Entries that fall outside the grid are dropped (Dirichlet elimination).
    """
    shape = tuple(shape)
    dims = len(shape)
    n = int(np.prod(shape))
    strides = [1]
    for d in range(1, dims):
        strides.append(strides[-1] * shape[d - 1])
    lin = [sum(o[d] * strides[d] for d in range(dims)) for o in offsets]
    assert all(lin[i] < lin[i + 1] for i in range(len(lin) - 1)), "offsets must ascend"
    # grid coordinates in x-fastest order; arrays are indexed [..., y, x]
    coords = np.meshgrid(*[np.arange(s, dtype=np.int64) for s in shape], indexing="ij")
    coords = [c.transpose(tuple(range(dims - 1, -1, -1))).reshape(-1) for c in coords]
    idx = np.arange(n, dtype=np.int64)
    is_complex = any(np.iscomplexobj(c) for c in coeffs)
    cols = np.empty((n, len(offsets)), dtype=np.int64)
    vals = np.empty((n, len(offsets)), dtype=np.complex128 if is_complex else np.float64)
    valid = np.ones((n, len(offsets)), dtype=bool)
    for k, (o, c) in enumerate(zip(offsets, coeffs)):
        ok = np.ones(n, dtype=bool)
        for d in range(dims):
            ok &= (coords[d] + o[d] >= 0) & (coords[d] + o[d] < shape[d])
        valid[:, k] = ok
        cols[:, k] = idx + lin[k]
        if np.isscalar(c):
            vals[:, k] = c
        else:
            vals[:, k] = np.asarray(c).transpose(tuple(range(dims - 1, -1, -1))).reshape(-1)
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = cols[valid].astype(np.int32)
    v = vals[valid]
    if is_complex:
        val = np.stack([v.real, v.imag], axis=1).astype(np.float64)
    else:
        val = v.astype(np.float64)
    assert row_ptr[-1] < 2**31
    return row_ptr.astype(np.int32), col_idx, np.ascontiguousarray(val)


def _upwind_coeffs(wind, h, dims):
    """Coefficients of h^2 * (-Laplace u + w . grad u), first-order upwind.

    Returns (diag, minus[d], plus[d]) with minus the coefficient of the
    neighbour at -e_d and plus that at +e_d."""
    diag = 2.0 * dims + h * sum(abs(w) for w in wind)
    minus = [-1.0 - h * max(w, 0.0) for w in wind]
    plus = [-1.0 - h * max(-w, 0.0) for w in wind]
    return diag, minus, plus


def convdiff2d(m, wind, name="convdiff2d"):
    """5-point upwind convection-diffusion on an m x m interior grid."""
    h = 1.0 / (m + 1)
    diag, mi, pl = _upwind_coeffs(wind, h, 2)
    offs = [(0, -1), (-1, 0), (0, 0), (1, 0), (0, 1)]
    coef = [mi[1], mi[0], diag, pl[0], pl[1]]
    rp, ci, val = stencil_csr((m, m), offs, coef)
    return rp, ci, val


def convdiff3d(m, wind):
    """7-point upwind convection-diffusion on an m^3 interior grid."""
    h = 1.0 / (m + 1)
    diag, mi, pl = _upwind_coeffs(wind, h, 3)
    offs = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    coef = [mi[2], mi[1], mi[0], diag, pl[0], pl[1], pl[2]]
    return stencil_csr((m, m, m), offs, coef)


def config1(m=32):
    """Real nonsymmetric 2D convection-diffusion, 5-point upwind, 32 x 32,
    Peclet 10 (wind 10 (1, 1)/sqrt(2)); b = A * ones."""
    w = 10.0 / np.sqrt(2.0)
    rp, ci, val = convdiff2d(m, (w, w))
    n = m * m
    return Problem("convdiff2d_%d_pe10" % m, n, rp, ci, val, np.ones(n),
                   {"tol": 1e-20, "max_iter": 2000, "method": "bicgstab", "kf": 1,
                    "grid": (m, m)})


def config2(m=128, seed=2504, xseed=2505):
    """Real 3D convection-diffusion, 7-point upwind, m^3 (m = 128: n =
    2,097,152, nnz = 14,581,760), Peclet 100 with a seeded random wind
    direction; x_true ~ U(-1, 1)."""
    g = np.random.Generator(np.random.PCG64(seed)).standard_normal(3)
    wind = 100.0 * g / np.linalg.norm(g)
    rp, ci, val = convdiff3d(m, tuple(wind))
    n = m ** 3
    x = np.random.Generator(np.random.PCG64(xseed)).uniform(-1.0, 1.0, n)
    return Problem("convdiff3d_%d_pe100" % m, n, rp, ci, val, x,
                   {"tol": 1e-25, "max_iter": min(3 * n, 10000), "method": "bicgstab",
                    "kf": 1, "wind": wind.tolist(), "grid": (m, m, m)})


def config3(m=1024, k=20.0, xseed=2506):
    """Complex shifted Helmholtz, 9-point Mehrstellen stencil (h^2-scaled,
    (1/6)[-1 -4 -1; -4 20 -4; -1 -4 -1]) minus (1 + 0.5i)(kh)^2 I on an
    m x m grid (m = 1024: n = 1,048,576, nnz = 9,424,900); x_true with
    re, im ~ U(-1, 1)."""
    h = 1.0 / (m + 1)
    shift = (1.0 + 0.5j) * (k * h) ** 2
    a, b, c = -1.0 / 6.0, -4.0 / 6.0, 20.0 / 6.0
    offs = [(-1, -1), (0, -1), (1, -1), (-1, 0), (0, 0), (1, 0), (-1, 1), (0, 1), (1, 1)]
    coef = [a, b, a, b, c - shift, b, a, b, a]
    rp, ci, val = stencil_csr((m, m), offs, coef)
    n = m * m
    rng = np.random.Generator(np.random.PCG64(xseed))
    x = np.stack([rng.uniform(-1.0, 1.0, n), rng.uniform(-1.0, 1.0, n)], axis=1)
    return Problem("helmholtz2d_%d_k%g" % (m, k), n, rp, ci, val, x,
                   {"tol": 1e-25, "max_iter": 10000, "method": "gpbicg", "kf": 1,
                    "grid": (m, m)})


def random_dd(n, seed, mmin=7, mmax=30, dmin=1.05, dmax=2.0):
    """Random nonsymmetric sparse system: each row stores m_i ~ U{mmin..mmax}
    entries including the diagonal; the m_i - 1 off-diagonal columns are
    distinct and uniform on [0, n) minus {i}, values N(0, 1); the diagonal
    is d_i * sum |a_ij| with d_i ~ U(dmin, dmax); x_true ~ U(-1, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = rng.integers(mmin, mmax + 1, size=n)
    k = np.minimum(m - 1, n - 1)
    tot = int(k.sum())
    rows = np.repeat(np.arange(n, dtype=np.int64), k)
    # draw columns on [0, n-1) and shift past the diagonal, redraw duplicates
    cols = rng.integers(0, n - 1, size=tot)
    cols = cols + (cols >= rows)
    while True:
        key = rows * n + cols
        order = np.argsort(key)
        ks = key[order]
        dup = np.zeros(tot, dtype=bool)
        dup[order[1:]] = ks[1:] == ks[:-1]
        nd = int(dup.sum())
        if nd == 0:
            break
        c = rng.integers(0, n - 1, size=nd)
        cols[dup] = c + (c >= rows[dup])
    offv = rng.standard_normal(tot)
    d = rng.uniform(dmin, dmax, size=n)
    absum = np.bincount(rows, weights=np.abs(offv), minlength=n)
    diag = d * absum
    diag[diag == 0.0] = 1.0
    # merge the (already row-grouped) off-diagonal entries, sorted by key,
    # with the diagonal: one sort of the combined row-major key
    ks = ks  # sorted off-diagonal keys from the last duplicate check
    offs = offv[order]
    dkey = np.arange(n, dtype=np.int64) * (n + 1)
    pos = np.searchsorted(ks, dkey)
    allk = np.insert(ks, pos, dkey)
    allv = np.insert(offs, pos, diag)
    ci = (allk % n).astype(np.int32)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(k + 1, out=rp[1:])
    x = rng.uniform(-1.0, 1.0, n)
    return Problem("random_dd_%d_s%d" % (n, seed), n, rp.astype(np.int32), ci, allv, x,
                   {"tol": 1e-25, "max_iter": 10000, "method": "bicgstab", "kf": 1})


def config4_sizes(nsys=512, base_seed=4_000_000, nmin=2000, nmax=200000):
    """Sizes of the batched workload: system s has n_s ~ U{nmin..nmax} drawn
    from its own seed base_seed + s."""
    return [int(np.random.Generator(np.random.PCG64(base_seed + s)).integers(nmin, nmax + 1))
            for s in range(nsys)]


def config4_system(s, base_seed=4_000_000, nmin=2000, nmax=200000):
    """System s of the batched workload (512 random diagonally dominant
    nonsymmetric systems of uneven size)."""
    n = config4_sizes(1, base_seed + s, nmin, nmax)[0]
    p = random_dd(n, (base_seed + s) * 7 + 1)
    p.name = "batched_sys%d_n%d" % (s, n)
    return p


def random_pattern(n, density, seed, complex_=False, dominance=None, symmetric_pattern=False):
    """Small random sparse matrix with every diagonal stored, for tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = rng.random((n, n)) < density
    if symmetric_pattern:
        mask |= mask.T
    np.fill_diagonal(mask, True)
    re = rng.standard_normal((n, n))
    im = rng.standard_normal((n, n)) if complex_ else np.zeros((n, n))
    if dominance is not None:
        off = np.where(mask, np.abs(re + 1j * im), 0.0)
        np.fill_diagonal(off, 0.0)
        re[np.arange(n), np.arange(n)] = dominance * off.sum(axis=1) + 1.0
        im[np.arange(n), np.arange(n)] = 0.0
    rows, cols = np.nonzero(mask)
    rp = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(mask.sum(axis=1), out=rp[1:])
    ci = cols.astype(np.int32)
    if complex_:
        val = np.stack([re[rows, cols], im[rows, cols]], axis=1)
    else:
        val = re[rows, cols].copy()
    x = rng.uniform(-1, 1, (n, 2) if complex_ else n)
    return Problem("random_%d_s%d" % (n, seed), n, rp, ci, val, x)


def lognormal_field(m, ell, seed, sigma=1.0, pad=2):
    """Unit-variance Gaussian random field with squared-exponential
    covariance (correlation length ell on the unit square), by spectral
    synthesis on a periodic (pad*m)^2 grid cropped to m x m; returns
    exp(sigma * g)."""
    N = pad * m
    rng = np.random.Generator(np.random.PCG64(seed))
    k = np.fft.fftfreq(N, d=1.0 / (N / (m + 1)))  # wavenumbers for spacing h
    kx, ky = np.meshgrid(k, k, indexing="ij")
    # spectral density of exp(-r^2 / (2 ell^2)) in 2D
    S = 2 * np.pi * ell ** 2 * np.exp(-2 * (np.pi ** 2) * (ell ** 2) * (kx ** 2 + ky ** 2))
    noise = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    g = np.fft.ifft2(noise * np.sqrt(S)).real
    g = g[:m, :m]
    g = (g - g.mean()) / (g.std() + 1e-300)
    return np.exp(sigma * g)


def config5(seed, m=512, ell=0.05):
    """Variable-coefficient 2D convection-diffusion on an m x m grid: 5-point
    finite volumes, diffusivity exp(g) (lognormal, sigma 1, correlation
    length ell) with harmonic-mean face values, first-order upwind
    convection with Peclet ~ U(1, 1000) at a random angle."""
    rng = np.random.Generator(np.random.PCG64(10_000_019 + seed))
    kap = lognormal_field(m, ell, seed)
    pe = rng.uniform(1.0, 1000.0)
    th = rng.uniform(0.0, 2 * np.pi)
    wx, wy = pe * np.cos(th), pe * np.sin(th)
    h = 1.0 / (m + 1)
    # face diffusivities (harmonic mean); boundary faces use the cell value
    kx_face = np.empty((m, m + 1))
    ky_face = np.empty((m + 1, m))
    k_ = kap  # indexed [y, x]
    kx_face[:, 1:m] = 2 * k_[:, :-1] * k_[:, 1:] / (k_[:, :-1] + k_[:, 1:])
    kx_face[:, 0] = k_[:, 0]
    kx_face[:, m] = k_[:, -1]
    ky_face[1:m, :] = 2 * k_[:-1, :] * k_[1:, :] / (k_[:-1, :] + k_[1:, :])
    ky_face[0, :] = k_[0, :]
    ky_face[m, :] = k_[-1, :]
    west = -kx_face[:, :m] - h * max(wx, 0.0)
    east = -kx_face[:, 1:] - h * max(-wx, 0.0)
    south = -ky_face[:m, :] - h * max(wy, 0.0)
    north = -ky_face[1:, :] - h * max(-wy, 0.0)
    diag = (kx_face[:, :m] + kx_face[:, 1:] + ky_face[:m, :] + ky_face[1:, :]
            + h * (abs(wx) + abs(wy)))
    # arrays are [y, x]; stencil_csr wants per-point arrays in grid shape (x, y)
    T = lambda a: a.T
    offs = [(0, -1), (-1, 0), (0, 0), (1, 0), (0, 1)]
    rp, ci, val = stencil_csr((m, m), offs, [T(south), T(west), T(diag), T(east), T(north)])
    n = m * m
    x = np.random.Generator(np.random.PCG64(20_000_003 + seed)).uniform(-1, 1, n)
    return Problem("lognormal_convdiff_%d_s%d" % (m, seed), n, rp, ci, val, x,
                   {"tol": 1e-25, "max_iter": 10000, "method": "bicgstab", "kf": 1,
                    "peclet": pe, "angle": th, "grid": (m, m)})


CONFIGS = {1: config1, 2: config2, 3: config3}
