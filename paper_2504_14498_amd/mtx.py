"""MatrixMarket coordinate files to and from the CSR layout of the library.

The paper measures on two SuiteSparse matrices, a real nonsymmetric and a
complex symmetric one (Section 4); SuiteSparse distributes them as
MatrixMarket files.  This reader takes the coordinate format with real,
integer, complex or pattern values and general, symmetric, skew-symmetric
or hermitian storage, and returns a Problem (workloads.Problem) in the
library's CSR layout: rows in the file's order (no reordering: any
reordering would change ILU(0)), columns ascending and unique per row, the
diagonal stored (an explicit zero is added where the file has none, so
that a missing diagonal is reported by ILU(0) as a zero pivot rather than
rejected by the pattern check), binary64 values, (re, im) pairs when
complex.  Duplicate entries are rejected, not summed.

File format: a header line "%%MatrixMarket matrix coordinate <field>
<symmetry>", comment lines starting with "%", a size line "m n nnz", then
one entry per line, "i j value" (1-based; complex: "i j re im"; pattern:
"i j").
"""
import numpy as np

from .workloads import Problem

FIELDS = ("real", "integer", "complex", "pattern")
SYMMETRIES = ("general", "symmetric", "skew-symmetric", "hermitian")


class MtxError(ValueError):
    pass


def _header(line):
    parts = line.strip().lower().split()
    if len(parts) != 5 or parts[0] != "%%matrixmarket" or parts[1] != "matrix":
        raise MtxError("not a MatrixMarket matrix header: %r" % line.strip())
    if parts[2] != "coordinate":
        raise MtxError("only the coordinate format is supported, got %r" % parts[2])
    if parts[3] not in FIELDS or parts[4] not in SYMMETRIES:
        raise MtxError("unsupported field/symmetry %r %r" % (parts[3], parts[4]))
    if parts[4] == "hermitian" and parts[3] != "complex":
        raise MtxError("hermitian storage needs complex values")
    return parts[3], parts[4]


def read(path, name=None):
    """Problem with the matrix of a MatrixMarket file (x_true all zero:
    the caller chooses its right-hand side)."""
    with open(path, "r") as f:
        first = f.readline()
        field, sym = _header(first)
        line = f.readline()
        while line and (line.startswith("%") or not line.strip()):
            line = f.readline()
        dims = line.split()
        if len(dims) != 3:
            raise MtxError("bad size line %r" % line.strip())
        m, n, nz = (int(v) for v in dims)
        if m != n or n <= 0:
            raise MtxError("the matrix must be square and non-empty (%d x %d)" % (m, n))
        ncol = {"pattern": 2, "complex": 4}.get(field, 3)
        data = np.loadtxt(f, dtype=np.float64, ndmin=2, comments="%") if nz > 0 else \
            np.zeros((0, ncol))
    if data.shape != (nz, ncol):
        raise MtxError("expected %d entries of %d fields, found %s" % (nz, ncol, data.shape))
    i = data[:, 0].astype(np.int64) - 1
    j = data[:, 1].astype(np.int64) - 1
    if np.any((i < 0) | (i >= n) | (j < 0) | (j >= n)) or \
            np.any(data[:, 0] != np.floor(data[:, 0])) or np.any(data[:, 1] != np.floor(data[:, 1])):
        raise MtxError("entry indices out of range")
    C = 2 if field == "complex" else 1
    if field == "pattern":
        v = np.ones((nz, 1))
    elif field == "complex":
        v = data[:, 2:4].copy()
    else:
        v = data[:, 2:3].copy()
    if sym != "general":
        if np.any(i < j):
            raise MtxError("symmetric storage must list the lower triangle only")
        off = i != j
        vt = v[off].copy()
        if sym == "skew-symmetric":
            if np.any(~off):
                raise MtxError("a skew-symmetric matrix has no diagonal entries")
            vt = -vt
        elif sym == "hermitian":
            vt[:, 1] = -vt[:, 1]
            if np.any(v[~off, 1] != 0):
                raise MtxError("a hermitian matrix has a real diagonal")
        i, j, v = (np.concatenate([i, j[off]]), np.concatenate([j, i[off]]),
                   np.concatenate([v, vt]))
    # add an explicit zero diagonal where none is stored
    has_diag = np.zeros(n, dtype=bool)
    has_diag[i[i == j]] = True
    miss = np.nonzero(~has_diag)[0]
    if len(miss):
        i = np.concatenate([i, miss])
        j = np.concatenate([j, miss])
        v = np.concatenate([v, np.zeros((len(miss), v.shape[1]))])
    order = np.lexsort((j, i))
    i, j, v = i[order], j[order], v[order]
    dup = (i[1:] == i[:-1]) & (j[1:] == j[:-1])
    if np.any(dup):
        k = int(np.nonzero(dup)[0][0])
        raise MtxError("duplicate entry (%d, %d)" % (i[k] + 1, j[k] + 1))
    if not np.all(np.isfinite(v)):
        raise MtxError("non-finite value")
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, i + 1, 1)
    rp = np.cumsum(rp)
    if rp[-1] >= 2 ** 31:
        raise MtxError("more than 2^31 - 1 stored entries")
    val = v.reshape(-1) if C == 1 else np.ascontiguousarray(v)
    x0 = np.zeros(n) if C == 1 else np.zeros((n, 2))
    return Problem(name or str(path), n, rp.astype(np.int32), j.astype(np.int32),
                   np.ascontiguousarray(val, dtype=np.float64), x0,
                   meta={"field": field, "symmetry": sym, "file_entries": nz,
                         "added_diagonal": len(miss)})


def write(path, p, comment=None):
    """Write a Problem's matrix as a general coordinate file (17
    significant digits, which read back to the same binary64 values)."""
    C = p.C
    rows = np.repeat(np.arange(p.n), np.diff(p.row_ptr)) + 1
    cols = p.col_idx.astype(np.int64) + 1
    with open(path, "w") as f:
        f.write("%%%%MatrixMarket matrix coordinate %s general\n" % ("complex" if C == 2 else "real"))
        if comment:
            for line in comment.splitlines():
                f.write("%% %s\n" % line)
        f.write("%d %d %d\n" % (p.n, p.n, p.nnz))
        if C == 1:
            for r, c, v in zip(rows, cols, p.val.reshape(-1)):
                f.write("%d %d %.17g\n" % (r, c, v))
        else:
            for r, c, v in zip(rows, cols, p.val.reshape(-1, 2)):
                f.write("%d %d %.17g %.17g\n" % (r, c, v[0], v[1]))
