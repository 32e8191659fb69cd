"""The paper's experiment on user-supplied matrices: every method with and
without ILU(0), in every multi-component precision, with the two factor
variants, on MatrixMarket files (Section 4, Tables 1, 2 and 4).

    python -m paper_2504_14498_amd.replicate mcfe.mtx dwg961b.mtx [--json out.json]

Per matrix and precision (DD, TD, QD) and method (BiCG, CGS, BiCGSTAB,
GPBiCG), three variants, named as in the paper's tables:
  <method>            no preconditioner (SpMV with binary64 A)
  <method>_ILU(0)     ILU(0) factor computed and stored in the working
                      precision from A promoted exactly
  <method>_d_ILU(0)   ILU(0) factor computed and stored in binary64
The mixed-precision SpMV (binary64 A times a multi-component vector) is the
only SpMV of this library, so the paper's "_d" SpMV variant of the
unpreconditioned methods is the unpreconditioned row itself.

Problem setup as in Section 4: x = sqrt(2) [1 ... n]^T for a real matrix and
sqrt(2 + 3i) [1 ... n]^T for a complex one (principal square root), formed
exactly and rounded once to the working precision's limbs; b = A x by the
library's SpMV in that precision; x0 = 0; stop when ||r|| < eps_r ||r0|| +
eps_a with eps_r = 1e-13, eps_a = 1e-100 (then confirmed on the true
residual), at most 3n passes.

Reported per run, as the tables' columns: [1] passes, [2] seconds (setup,
factorisation and iterations; G18 of the reading notes), [3] ms per pass;
and per matrix, precision and method the per-pass time ratios of Table 4:
ILU(0) / no preconditioner, _d_ILU(0) / no preconditioner, ILU(0) /
_d_ILU(0).  Every step runs in the HIP library; this module orders the
calls and formats the report.
"""
import argparse
import decimal
import json
import sys
import time

import numpy as np

from . import mtx

METHODS = ("bicg", "cgs", "bicgstab", "gpbicg")
METHOD_NAMES = {"bicg": "BiCG", "cgs": "CGS", "bicgstab": "BiCGSTAB", "gpbicg": "GPBiCG"}
PRECS = {2: "DD", 3: "TD", 4: "QD"}
EPS_R, EPS_A = 1e-13, 1e-100


def _limbs(v, K, ctx):
    """Round an exact real (decimal.Decimal at high precision) to K binary64
    limbs, each the nearest binary64 to what the earlier ones leave."""
    out = []
    for _ in range(K):
        d = float(v)
        out.append(d)
        v = ctx.subtract(v, decimal.Decimal(d))
    return out


def paper_x(n, C, K):
    """x_i = s i (i = 1..n) with s = sqrt(2) (real) or sqrt(2 + 3i)
    (complex, principal branch), computed with 120 significant digits and
    rounded to K limbs per component: float64 (n, C, K)."""
    ctx = decimal.Context(prec=120)
    two = decimal.Decimal(2)
    if C == 1:
        parts = [ctx.sqrt(two)]
    else:
        mod = ctx.sqrt(decimal.Decimal(13))          # |2 + 3i|
        re = ctx.sqrt(ctx.divide(ctx.add(mod, two), two))
        im = ctx.sqrt(ctx.divide(ctx.subtract(mod, two), two))
        parts = [re, im]
    x = np.zeros((n, C, K))
    for c, s in enumerate(parts):
        for i in range(n):
            x[i, c, :] = _limbs(ctx.multiply(s, decimal.Decimal(i + 1)), K, ctx)
    return x


def run_matrix(p, precs=(2, 3, 4), methods=METHODS, max_iter=None, note=None, rhs=None,
               keep_x=False):
    """All variants on one problem; returns a list of run records.  rhs:
    optional function (K) -> b as a (n, C, K) host array, instead of A x
    by the library's SpMV; keep_x: keep each run's solution (host) in its
    record."""
    import torch

    from . import mpk
    A = mpk.Csr.from_problem(p)
    max_iter = max_iter or 3 * p.n
    runs = []
    for K in precs:
        xt = torch.as_tensor(paper_x(p.n, p.C, K)).cuda()
        b = mpk.csr_spmv(A, xt) if rhs is None else torch.as_tensor(rhs(K)).cuda()
        for m in methods:
            for variant, fp in (("", 0), ("_ILU(0)", K), ("_d_ILU(0)", 1)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, info = mpk.krylov_solve(m, A, b, fprec=fp, tol_rel=EPS_R, tol_abs=EPS_A,
                                           max_iter=max_iter)
                torch.cuda.synchronize()
                sec = time.perf_counter() - t0
                rec = {"matrix": p.name, "n": p.n, "nnz": p.nnz, "complex": p.C == 2,
                       "prec": PRECS[K], "K": K, "method": m,
                       "variant": METHOD_NAMES[m] + variant, "fprec": fp,
                       "status": info["status"], "iters": info["iters"], "seconds": sec,
                       "ms_per_iter": 1e3 * sec / max(info["iters"], 1),
                       "relres_true": info["relres_true"],
                       "err_vs_x": float(torch.max(torch.abs(x[:, :, 0] - xt[:, :, 0])).item())}
                if keep_x:
                    rec["x"] = x.cpu().numpy()
                runs.append(rec)
                if note:
                    note("%s %s %s: %s, %d passes, %.3f s" % (p.name, PRECS[K], rec["variant"],
                                                            rec["status"], rec["iters"], sec))
    return runs


def ratios(runs):
    """Table 4: per-pass time ratios for each (matrix, precision, method)."""
    by = {}
    for r in runs:
        kind = "0" if r["fprec"] == 0 else ("d" if r["fprec"] == 1 else "w")
        by.setdefault((r["matrix"], r["prec"], r["method"]), {})[kind] = r["ms_per_iter"]
    out = []
    for (mat, prec, m), t in sorted(by.items()):
        if not {"0", "w", "d"} <= set(t):
            continue
        out.append({"matrix": mat, "prec": prec, "method": METHOD_NAMES[m],
                    "ILU(0)/plain": t["w"] / t["0"], "ILU(0)_d/plain": t["d"] / t["0"],
                    "ILU(0)/ILU(0)_d": t["w"] / t["d"]})
    return out


def table(runs):
    """Text table in the layout of Tables 1 and 2: one row per variant,
    columns [1] [2] [3] per precision."""
    precs = sorted({r["prec"] for r in runs}, key=lambda s: "DD TD QD".index(s))
    lines = []
    for mat in sorted({r["matrix"] for r in runs}):
        rs = [r for r in runs if r["matrix"] == mat]
        lines.append("%s (n = %d, nnz = %d%s)" % (mat, rs[0]["n"], rs[0]["nnz"],
                                                  ", complex" if rs[0]["complex"] else ""))
        head = "%-20s" % "" + "".join("  %8s [1] %9s [2] %9s [3]" % (p, "s", "ms") for p in precs)
        lines.append(head)
        variants = []
        for r in rs:
            if r["variant"] not in variants:
                variants.append(r["variant"])
        for v in variants:
            row = "%-20s" % v
            for p in precs:
                r = next((r for r in rs if r["variant"] == v and r["prec"] == p), None)
                if r is None:
                    row += " " * 36
                    continue
                it = "%d%s" % (r["iters"], "" if r["status"] == "ok" else "*")
                row += "  %12s %13.3f %13.3f" % (it, r["seconds"], r["ms_per_iter"])
            lines.append(row)
        lines.append("(* not converged: max_iter reached or breakdown)")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("files", nargs="+", help="MatrixMarket coordinate files")
    ap.add_argument("--precs", default="2,3,4", help="limb counts (2 = DD, 3 = TD, 4 = QD)")
    ap.add_argument("--methods", default=",".join(METHODS))
    ap.add_argument("--max-iter", type=int, default=None, help="default 3n")
    ap.add_argument("--json", default=None, help="write every run and the ratios here")
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    note = lambda m: print("[replicate] " + m, file=sys.stderr, flush=True)
    runs = []
    for f in args.files:
        p = mtx.read(f)
        runs += run_matrix(p, tuple(int(k) for k in args.precs.split(",")),
                           tuple(args.methods.split(",")), args.max_iter, note)
    print(table(runs))
    rat = ratios(runs)
    print("\nPer-pass time ratios (Table 4 layout)")
    for r in rat:
        print("%-12s %s %-9s ILU(0)/plain %8.1f  ILU(0)_d/plain %8.1f  ILU(0)/ILU(0)_d %5.2f" %
              (r["matrix"][-12:], r["prec"], r["method"], r["ILU(0)/plain"], r["ILU(0)_d/plain"],
               r["ILU(0)/ILU(0)_d"]))
    if args.json:
        with open(args.json, "w") as fh:
            json.dump({"runs": runs, "ratios": rat}, fh, indent=1)


if __name__ == "__main__":
    main()
