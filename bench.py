"""Benchmark: double-double time-to-solution at relative residual 1e-25.

Workload (one "step" = one complete solve, inputs resident in HBM): the
real 3D convection-diffusion system on a 128^3 grid (7-point upwind
stencil, Peclet 100, seeded wind direction; n = 2,097,152, nnz =
14,581,760), b = A x_true with x_true ~ U(-1, 1), solved by ILU(0)-
preconditioned BiCGSTAB in double-double with a binary64 ILU(0) factor,
to a true relative residual of 1e-25.  A step covers the whole path:
pattern checks, level analysis, ILU(0) factorisation, the iterations and
the true-residual confirmation.

Besides the JSON line's time-to-solution, the run measures the two kernel
families of the hot path with HIP events on the stream they run on: the
DD SpMV (y = A x) and the ILU(0) apply (forward + backward sweep), and
reports their algorithmic GB/s against the 8 TB/s HBM peak.  The CPU
baseline runs the oracle (single-threaded C) for a bounded number of
passes of the same solve and scales it to a time-to-solution.

Unless --no-extras, the same run also reports: the multicolour variant on
the same system (a different preconditioner, labelled as such), the SpMV
on random rows with the lanes-per-row sweep, the 512-system batched solve
(and 16 large systems, one workgroup each against teams of workgroups),
and the learned correction against plain ILU(0).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def spmv_bytes(n, nnz, C, K):
    """Algorithmic bytes of one SpMV: values + column indices once, row
    pointers once, x read once, y written once."""
    return nnz * (8 * C + 4) + 4 * (n + 1) + 2 * n * 8 * C * K


def apply_bytes(n, nnz, C, K, KF):
    """Algorithmic bytes of one ILU(0) apply (forward + backward sweep):
    factor values and column indices once (the diagonal once), the two
    sweeps' row pointers and level orders, r read, y written and read,
    z written."""
    off = nnz - n
    return (off * (8 * C * KF + 4) + n * 8 * C * KF + 2 * 4 * (n + 1) + 2 * 4 * n
            + 4 * n * 8 * C * K)


def time_events(fn, reps, stream):
    """Mean duration of fn over reps back-to-back launches (HIP events on
    the stream the kernels run on)."""
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        fn()
        start.record(stream)
        for _ in range(reps):
            fn()
        stop.record(stream)
    stop.synchronize()
    return start.elapsed_time(stop) / reps


def time_events_cold(fn, reps, stream, flush):
    """Mean duration of fn when a buffer larger than the 256 MiB Infinity
    Cache has been read just before each launch, so that its inputs come
    from HBM rather than from the cache (read, not written: no dirty lines
    are left to be written back during the timed launch)."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    sink = torch.empty(1, dtype=flush.dtype, device=flush.device)
    with torch.cuda.stream(stream):
        fn()
        for a, b in evs:
            torch.sum(flush, dim=0, keepdim=True, out=sink)
            a.record(stream)
            fn()
            b.record(stream)
    evs[-1][1].synchronize()
    return sum(a.elapsed_time(b) for a, b in evs) / reps


def kernel_sources_digest():
    """Digest of the sources of the measured kernels: hardware-counter
    traffic recorded for another version of them is not reported."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hpp", "mp.hpp", "internal.hpp", "ops.hip", "apply.hpp", "analysis.cpp"):
        with open(os.path.join(ROOT, "paper_2504_14498_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(p, b, iters_gpu, passes):
    """Oracle (plain sequential C) on a bounded sample: ILU(0) + `passes`
    BiCGSTAB passes of the same system; scaled to the GPU's iteration
    count to give a projected time-to-solution."""
    import oracle
    t0 = time.perf_counter()
    st, bad, f = oracle.ilu0(p.row_ptr, p.col_idx, p.val, 1, 1)
    t1 = time.perf_counter()
    res = oracle.krylov("bicgstab", p.row_ptr, p.col_idx, p.val, b, kf=1, tol_rel=1e-25,
                        max_iter=passes)
    t2 = time.perf_counter()
    per_pass = (t2 - t1 - (t1 - t0)) / max(res["iters"], 1)
    projected = (t1 - t0) + per_pass * iters_gpu
    return {"value": projected, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": "ILU(0) factor + %d BiCGSTAB-DD passes on the full %d-row system "
                      "(%.1f s measured), scaled to %d passes" % (res["iters"], p.n, t2 - t0,
                                                                  iters_gpu),
            "measured_s": t2 - t0, "per_pass_s": per_pass}


def _gen_system(q):
    from paper_2504_14498_amd import workloads as W
    p = W.config4_system(q)
    return p.n, p.row_ptr, p.col_idx, p.val, p.x_true


# vector streams of one BiCGSTAB pass beyond its two SpMVs and two applies
# (loads and stores of n-element vectors by the update and inner-product
# kernels)
BICGSTAB_VECTOR_STREAMS = 17


def batched_bytes(ns, nnzs, iters, K=2, KF=1):
    """Algorithmic bytes of the batched solve: per system the ILU(0)
    factorisation (A's values and indices read, the factor written) and,
    per pass, two SpMVs, two ILU(0) applies and the vector streams."""
    tot = 0
    for n, nnz, it in zip(ns, nnzs, iters):
        fac = nnz * (8 + 4) + 4 * (n + 1) + nnz * 8 * KF
        per = (2 * spmv_bytes(n, nnz, 1, K) + 2 * apply_bytes(n, nnz, 1, K, KF)
               + BICGSTAB_VECTOR_STREAMS * n * 8 * K)
        tot += fac + it * per
    return tot


def measure_batched(nsys, warmup, steps, seq_sample, note):
    """512 random nonsymmetric systems (n ~ U{2000..200000}, 7-30 entries per
    row, diagonal dominance U(1.05, 2)) solved by ILU(0)-BiCGSTAB in DD to
    1e-25 in one persistent launch; compared with the same systems solved
    one after another on the single-system path (a sample, scaled by nnz)."""
    import concurrent.futures as cf
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as pool:
        systems = list(pool.map(_gen_system, range(nsys)))
    tgen = time.perf_counter() - t0
    import torch

    from paper_2504_14498_amd import mpk
    torch.cuda.set_device(0)
    note("generated %d systems in %.1f s: sum n = %d, sum nnz = %d" %
         (len(systems), tgen, sum(s[0] for s in systems), sum(len(s[2]) for s in systems)))
    mats, bs = [], []
    for n, rp, ci, val, x in systems:
        A = mpk.Csr(rp, ci, val)
        xt = torch.zeros((n, 1, 2), dtype=torch.float64, device="cuda")
        xt[:, 0, 0] = torch.as_tensor(x, device="cuda")
        mats.append(A)
        bs.append(mpk.csr_spmv(A, xt))
        if len(mats) % 128 == 0:
            note("uploaded %d systems: %.1f s" % (len(mats), time.perf_counter() - t0))
    del systems
    torch.cuda.synchronize()
    note("uploaded, b = A x_true computed: %.1f s" % (time.perf_counter() - t0))
    ws = None
    for w in range(max(warmup, 1)):   # the first call also autotunes the schedule
        a = time.perf_counter()
        xs, infos, st, ws = mpk.krylov_solve_batched(mats, bs, fprec=1, tol_rel=1e-25,
                                                     max_iter=10000, workspace=ws)
        note("batched warmup %d (%s): %s, %.3f s" %
             (w, "with autotune" if w == 0 else "tuned", st, time.perf_counter() - a))
    times = []
    for _ in range(steps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        xs, infos, st, ws = mpk.krylov_solve_batched(mats, bs, fprec=1, tol_rel=1e-25,
                                                     max_iter=10000, workspace=ws)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - a)
        note("batched solve: %s %.3f s" % (st, times[-1]))
    iters = [i["iters"] for i in infos]
    ok = sum(i["status"] == "ok" for i in infos)
    samp = list(range(0, len(mats), max(1, len(mats) // seq_sample)))[:seq_sample]
    tseq = 0.0
    nnz_s = 0
    for q in samp:
        torch.cuda.synchronize()
        a = time.perf_counter()
        x, info = mpk.krylov_solve("bicgstab", mats[q], bs[q], fprec=1, tol_rel=1e-25,
                                   max_iter=10000)
        torch.cuda.synchronize()
        tseq += time.perf_counter() - a
        nnz_s += mats[q].nnz
    tot_nnz = sum(A.nnz for A in mats)
    seq_proj = tseq * tot_nnz / max(nnz_s, 1)
    med = sorted(times)[len(times) // 2]
    nbytes = batched_bytes([A.n for A in mats], [A.nnz for A in mats], iters)
    gbs = nbytes / med / 1e9
    return {"workload": "batched_random_dd nsys=%d (n ~ U{2000..200000}, 7-30 entries/row, "
                        "BiCGSTAB-DD, ILU(0)-D, 1e-25)" % len(mats),
            "sum_n": sum(A.n for A in mats), "sum_nnz": tot_nnz,
            "launch_s": med, "solves_per_s": len(mats) / med, "converged": ok,
            "iters_median": sorted(iters)[len(iters) // 2], "iters_max": max(iters),
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes": nbytes},
            "sequential": {"sample_systems": len(samp), "sample_s": tseq,
                           "projected_s": seq_proj, "speedup": seq_proj / med}}


def measure_batched_few(nsys, nrows, note):
    """Fewer systems than workgroups (nsys random systems of nrows rows each,
    as in the batched workload): one workgroup per system against the tuned
    schedule, which gives each system a team of workgroups on one XCD.  The
    solutions must agree bit for bit."""
    import concurrent.futures as cf
    import torch

    from paper_2504_14498_amd import mpk
    from paper_2504_14498_amd import workloads as W
    with cf.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as pool:
        probs = list(pool.map(lambda q: W.random_dd(nrows, 7_000_000 + q), range(nsys)))
    mats, bs = [], []
    for p in probs:
        A = mpk.Csr.from_problem(p)
        xt = torch.zeros((p.n, 1, 2), dtype=torch.float64, device="cuda")
        xt[:, 0, 0] = torch.as_tensor(p.x_true, device="cuda")
        mats.append(A)
        bs.append(mpk.csr_spmv(A, xt))
    del probs
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    res, xs_of = {}, {}
    ws = None
    for name, sched in (("one_workgroup_per_system", "grid=%d,order=lpt" % cus),
                        ("tuned", None)):
        for rep in range(2):   # the first tuned call also autotunes
            torch.cuda.synchronize()
            a = time.perf_counter()
            xs, infos, st, ws = mpk.krylov_solve_batched(mats, bs, fprec=1, tol_rel=1e-25,
                                                         max_iter=10000, schedule=sched,
                                                         workspace=ws)
            torch.cuda.synchronize()
            dt = time.perf_counter() - a
        res[name] = {"launch_s": dt, "status": st,
                     "iters_max": max(i["iters"] for i in infos)}
        xs_of[name] = xs
        note("batched, %d x %d rows, %s: %s %.3f s" % (nsys, nrows, name, st, dt))
    same = all(torch.equal(u, v) for u, v in zip(xs_of["one_workgroup_per_system"],
                                                 xs_of["tuned"]))
    return {"workload": "batched_random_dd nsys=%d n=%d (7-30 entries/row, BiCGSTAB-DD, "
                        "ILU(0)-D, 1e-25)" % (nsys, nrows),
            **res, "speedup_tuned": res["one_workgroup_per_system"]["launch_s"] /
            res["tuned"]["launch_s"], "bitwise_equal": same}


def measure_spmv_rows(reps, note):
    """SpMV (DD vectors) on one system of the batched workload (random
    columns, 7-30 entries per row): one lane per row against the vector
    layouts (2-16 lanes per row), each timed with its inputs coming from
    HBM, and the lanes the library's tuner picks."""
    import torch

    from paper_2504_14498_amd import mpk
    from paper_2504_14498_amd import workloads as W
    p = W.config4_system(0)
    A = mpk.Csr.from_problem(p)
    K = 2
    x = torch.rand((p.n, 1, K), dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    s = torch.cuda.Stream()
    flush = torch.empty(512 << 17, dtype=torch.float64, device="cuda").zero_()
    sb = spmv_bytes(p.n, p.nnz, 1, K)
    cold = {}
    for lanes in (1, 2, 4, 8, 16):
        mpk.spmv_set_lanes(A, lanes)
        cold[lanes] = time_events_cold(lambda: mpk.csr_spmv(A, x, y, stream=s), reps, s, flush)
    mpk.spmv_set_lanes(A, 0)
    tuned, _ = mpk.spmv_tune(A, x, y, stream=s)
    del flush
    note("spmv random rows: " + " ".join("%d:%.4f ms" % (l, t) for l, t in cold.items()) +
         ", tuner picks %d" % tuned)
    return {"workload": "random nonsymmetric n=%d nnz=%d (7-30 entries/row), DD vectors"
                        % (p.n, p.nnz),
            "bytes": sb, "note": "cold: a 512 MiB buffer read before each launch",
            "cold_ms_by_lanes": {str(l): t for l, t in cold.items()},
            "cold_gbs_by_lanes": {str(l): sb / (t * 1e-3) / 1e9 for l, t in cold.items()},
            "tuned_lanes": tuned, "tuned_cold_ms": cold[tuned],
            "speedup_tuned_vs_1": cold[1] / cold[tuned]}


def measure_multicolor(p, A, b, tol, max_iter, reps, natural_s, note):
    """The multicolour variant on the headline system (a different
    preconditioner, beyond the paper's method): rows ordered by a greedy
    colouring of A + A^T, B = P A P^T, BiCGSTAB-DD on B y = P b with a
    binary64 ILU(0) of B, x = P^T y.  Time-to-solution covers the ordering,
    the permutations, the factorisation and the passes."""
    import torch

    from paper_2504_14498_amd import mpk
    x, info = mpk.krylov_solve_multicolor("bicgstab", A, b, fprec=1, tol_rel=tol,
                                          max_iter=max_iter)   # warm-up
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = mpk.krylov_solve_multicolor("bicgstab", A, b, fprec=1, tol_rel=tol,
                                              max_iter=max_iter)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    tts = sorted(times)[1]
    B = info["B"]
    M = mpk.ilu0_factor(B, 1, vprec=2)
    s = torch.cuda.Stream()
    bp = mpk.vec_permute(b, info["perm"])
    z = torch.empty_like(bp)
    apply_ms = time_events(lambda: mpk.ilu0_apply(M, bp, z, stream=s), reps, s)
    flush = torch.empty(512 << 17, dtype=torch.float64, device="cuda").zero_()
    apply_cold = time_events_cold(lambda: mpk.ilu0_apply(M, bp, z, stream=s), reps, s, flush)
    del flush
    ab = apply_bytes(p.n, p.nnz, 1, 2, 1)
    note("multicolour variant: %s, %d colours, %d passes, %.1f ms (natural ordering %.1f ms), "
         "apply %.4f ms" % (info["status"], info["ncolors"], info["iters"], tts * 1e3,
                            natural_s * 1e3, apply_ms))
    return {"variant": "multicolour ILU(0): greedy colouring of A + A^T in natural order, "
                       "B = P A P^T, ILU(0) of B (a different preconditioner from the paper's)",
            "status": info["status"], "ncolors": info["ncolors"], "iters": info["iters"],
            "relres_true": info["relres_true"], "time_to_solution_s": tts,
            "vs_natural_ordering": natural_s / tts, "setup_ms": info["setup_ms"],
            "solve_ms": info["solve_ms"], "ms_per_iter": info["solve_ms"] / max(info["iters"], 1),
            "ilu0_apply": {"ms": apply_ms, "gbs": ab / (apply_ms * 1e-3) / 1e9,
                           "frac": ab / (apply_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                           "cold_ms": apply_cold,
                           "cold_gbs": ab / (apply_cold * 1e-3) / 1e9, "bytes": ab}}


def bench_batched(args):
    note = lambda m: print("[bench] " + m, file=sys.stderr, flush=True)
    r = measure_batched(args.nsys, args.warmup, args.steps, args.seq_sample, note)
    out = {"metric": "batched DD time-to-solution at rel. residual 1e-25 (ILU(0)-BiCGSTAB, "
                     "one persistent launch)",
           "value": r["launch_s"], "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": r["launch_s"] * 1e3, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "dd (2 x f64)",
           "data": "synthetic (seeded random diagonally dominant systems)",
           "config": {"workload": r["workload"]}, "batched": r}
    print(json.dumps(out))


PARAMS_FILE = os.path.join(ROOT, "paper_2504_14498_amd", "learned_params.npz")


def load_params(path):
    """Kept network parameters and their training record (plain arrays,
    loaded without unpickling)."""
    saved = np.load(path, allow_pickle=False)
    return saved["params"].astype(np.float32), json.loads(str(saved["train_info"]))


def train_learned(args, note):
    """Train the network on method-generated lognormal convection-diffusion
    systems (streamed: each is factored, probed and used for one step) and
    keep the parameters that the plain method judges best on a validation
    split.  Returns (params on the device, training record)."""
    import concurrent.futures as cf

    import torch

    from paper_2504_14498_amd import learned as LR
    from paper_2504_14498_amd import workloads as W
    m, ntrain, nval = args.lgrid, args.ntrain, args.nval
    gen = lambda s: W.config5(s, m=m)
    pool = cf.ThreadPoolExecutor(min(16, os.cpu_count() or 1))
    val_seeds = list(range(ntrain - nval, ntrain))     # never trained on
    val = []
    for p in pool.map(gen, val_seeds):
        A = LR.mpk.Csr.from_problem(p)
        b = LR.mpk.csr_spmv(A, torch.as_tensor(p.x_true_limbs(2)).cuda())
        val.append((A, b))
    val_plain = [LR.solve_plain(A, b)[1]["iters"] for A, b in val]
    cap = LR.iteration_cap(val_plain)
    note("validation: %d systems, plain iterations %s, cap %d" % (nval, val_plain, cap))
    tr = LR.Trainer(seed=args.seed, lr=args.lr)
    best = (1.0, tr.params.clone(), 0)     # delta = 0 is the plain factor
    losses = []
    t_train = time.perf_counter()
    ntr = ntrain - nval
    for k, p in enumerate(pool.map(gen, range(ntr))):
        inst = LR.Instance(p, seed=k)
        losses.append(float(tr.step(inst)))
        del inst
        if (k + 1) % 50 == 0:
            note("step %d: mean loss of the last 50 %.4e" % (k + 1, np.mean(losses[-50:])))
        if (k + 1) % args.val_every == 0 or k + 1 == ntr:
            r = LR.validation_ratio(tr.params, val, val_plain, cap)
            if r < best[0]:
                best = (r, tr.params.clone(), k + 1)
            note("step %d: validation iteration ratio %.3f (best %.3f at %d)"
                 % (k + 1, r, best[0], best[2]))
    pool.shutdown()
    info = {"seconds": time.perf_counter() - t_train, "steps": len(losses), "lr": args.lr,
            "seed": args.seed, "grid": m, "train_seeds": [0, ntr - 1],
            "validation_seeds": [val_seeds[0], val_seeds[-1]], "kept_step": best[2],
            "validation_ratio": best[0], "validation_plain_iters": val_plain, "cap": cap,
            "loss_first_100": float(np.mean(losses[:100])) if losses else None,
            "loss_last_100": float(np.mean(losses[-100:])) if losses else None}
    return best[1], info


def evaluate_learned(params, cap, m, ntest, note):
    """DD BiCGSTAB time-to-solution at 1e-25 over held-out systems (seeds
    100000 + q), learned (factor + network + correction + solve, fallbacks
    included) against plain ILU(0) on the same GPU."""
    import concurrent.futures as cf

    import torch

    from paper_2504_14498_amd import learned as LR
    from paper_2504_14498_amd import workloads as W
    params = torch.as_tensor(params).cuda()
    gen = lambda s: W.config5(s, m=m)
    rows = []
    with cf.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as pool:
        for q, p in enumerate(pool.map(gen, range(100_000, 100_000 + ntest))):
            A = LR.mpk.Csr.from_problem(p)
            b = LR.mpk.csr_spmv(A, torch.as_tensor(p.x_true_limbs(2)).cuda())
            _, ip = LR.solve_plain(A, b)
            _, il = LR.solve_learned(A, b, params, cap)
            rows.append((ip["iters"], ip["tts_s"], il["iters_total"], il["tts_s"], il["fallback"],
                         ip["status"], il["status"], il["relres_true"]))
            if (q + 1) % 8 == 0:
                note("learned test %d/%d: plain %d it %.3f s, learned %d it %.3f s" %
                     (q + 1, ntest, rows[-1][0], rows[-1][1], rows[-1][2], rows[-1][3]))
    r = np.array([row[:4] for row in rows], dtype=np.float64)
    return {"workload": "lognormal_convdiff %dx%d (n = %d), BiCGSTAB-DD to 1e-25, held-out "
                        "seeds 100000..%d" % (m, m, m * m, 100_000 + ntest - 1),
            "test_systems": ntest, "cap": cap,
            "plain": {"tts_s_quartiles": LR.quartiles(r[:, 1]),
                      "iters_quartiles": LR.quartiles(r[:, 0])},
            "learned": {"tts_s_quartiles": LR.quartiles(r[:, 3]),
                        "iters_quartiles": LR.quartiles(r[:, 2]),
                        "fallbacks": sum(row[4] is not None for row in rows)},
            "median_ratio": {"tts": float(np.median(r[:, 3] / r[:, 1])),
                             "iters": float(np.median(r[:, 2] / r[:, 0]))},
            "both_converged": sum(row[5] == "ok" and row[6] == "ok" for row in rows),
            "max_learned_relres_true": max(row[7] for row in rows)}


def bench_learned(args):
    """The learned workload on its own: train (or load) the parameters, then
    compare learned and plain over the held-out systems."""
    import torch
    torch.cuda.set_device(0)
    note = lambda m: print("[bench] " + m, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    if args.load_params:
        params, info = load_params(args.load_params)
        note("loaded parameters from %s (trained %d steps, kept step %d)" %
             (args.load_params, info["steps"], info["kept_step"]))
    else:
        params, info = train_learned(args, note)
        params = params.cpu().numpy()
    if args.save_params:
        np.savez(args.save_params, params=params, train_info=np.array(json.dumps(info)))
        note("saved parameters to %s" % args.save_params)
    if args.ntest == 0:
        print(json.dumps({"training": info}))
        return
    r = evaluate_learned(params, info["cap"], args.lgrid, args.ntest, note)
    med_l = r["learned"]["tts_s_quartiles"][1]
    out = {"metric": "DD time-to-solution at rel. residual 1e-25, learned vs plain ILU(0) "
                     "(BiCGSTAB, lognormal convection-diffusion)",
           "value": med_l, "unit": "s", "n_gpus": 1, "steps": args.ntest, "warmup": 0,
           "ms_per_step": med_l * 1e3, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "dd (2 x f64), network bf16/f32",
           "data": "synthetic (seeded lognormal-coefficient convection-diffusion)",
           "config": {"workload": r["workload"]}, "learned": r, "training": info,
           "total_s": time.perf_counter() - t0}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--reps", type=int, default=20, help="event-timed kernel launches")
    ap.add_argument("--cpu-passes", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", type=int, default=1)
    ap.add_argument("--kernels-only", action="store_true",
                    help="run only SpMV, ILU(0) apply and a calibration copy (counter runs)")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--workload", default="convdiff3d",
                    choices=["convdiff3d", "batched", "learned"])
    ap.add_argument("--lgrid", type=int, default=512, help="grid of the learned workload")
    ap.add_argument("--ntrain", type=int, default=2000)
    ap.add_argument("--nval", type=int, default=16)
    ap.add_argument("--ntest", type=int, default=200)
    ap.add_argument("--val-every", type=int, default=250)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--save-params", default=None, help="learned workload: save the kept parameters (.npz)")
    ap.add_argument("--load-params", default=None, help="learned workload: skip training, load (.npz)")
    ap.add_argument("--nsys", type=int, default=512)
    ap.add_argument("--seq-sample", type=int, default=8)
    ap.add_argument("--learned-ntest", type=int, default=24,
                    help="held-out systems of the learned comparison in the default run")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline solve only (no batched and learned comparisons)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU path "
              "(--gpus 1); multi-GPU sharding is a design note, not implemented.",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "learned":
        return bench_learned(args)

    import torch

    from paper_2504_14498_amd import mpk
    from paper_2504_14498_amd import workloads as W

    torch.cuda.set_device(0)
    p = W.config2(args.grid)
    K, KF, C = 2, 1, 1
    tol = 1e-25
    max_iter = p.meta["max_iter"]
    A = mpk.Csr.from_problem(p)
    xt = torch.as_tensor(p.x_true_limbs(K)).cuda()
    b = mpk.csr_spmv(A, xt)          # b = A x_true in DD, on the GPU
    torch.cuda.synchronize()

    ws = None
    info = None

    def note(msg):
        print("[bench] " + msg, file=sys.stderr, flush=True)

    note("problem %s: n=%d nnz=%d" % (p.name, p.n, p.nnz))
    if args.kernels_only:
        # for hardware-counter runs: the two hot operations alone, plus a
        # plain device copy of known size whose counters calibrate theirs
        M = mpk.ilu0_factor(A, KF, vprec=K)
        y = torch.empty_like(b)
        z = torch.empty_like(b)
        src = torch.ones(args.copy_mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(args.reps):
            mpk.csr_spmv(A, b, y)
            mpk.ilu0_apply(M, b, z)
            dst.copy_(src)
        torch.cuda.synchronize()
        note("kernels only: %d x (spmv, ilu0 apply, copy of %d MiB)" % (args.reps, args.copy_mib))
        return
    for _ in range(args.warmup):
        x, info = mpk.krylov_solve("bicgstab", A, b, fprec=KF, tol_rel=tol, max_iter=max_iter,
                                   workspace=ws, graph=bool(args.graph))
        ws = info["workspace"]
        note("warmup solve: %s iters=%d setup=%.1f ms solve=%.1f ms" %
             (info["status"], info["iters"], info["setup_ms"], info["solve_ms"]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        x, info = mpk.krylov_solve("bicgstab", A, b, fprec=KF, tol_rel=tol, max_iter=max_iter,
                                   workspace=ws, graph=bool(args.graph))
        ws = info["workspace"]
        infos.append(info)
        note("timed solve: %s iters=%d setup=%.1f ms solve=%.1f ms" %
             (info["status"], info["iters"], info["setup_ms"], info["solve_ms"]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    info = infos[-1]
    if info["status"] != "ok":
        print("solve did not converge: %s" % info, file=sys.stderr)
        sys.exit(1)
    iters = info["iters"]

    # live per-kernel timing on the stream the kernels run on
    s = torch.cuda.Stream()
    y = torch.empty_like(b)
    spmv_ms = time_events(lambda: mpk.csr_spmv(A, b, y, stream=s), args.reps, s)
    M = mpk.ilu0_factor(A, KF, vprec=K)
    z = torch.empty_like(b)
    apply_ms = time_events(lambda: mpk.ilu0_apply(M, b, z, stream=s), args.reps, s)
    sb = spmv_bytes(p.n, p.nnz, C, K)
    ab = apply_bytes(p.n, p.nnz, C, K, KF)
    spmv_gbs = sb / (spmv_ms * 1e-3) / 1e9
    apply_gbs = ab / (apply_ms * 1e-3) / 1e9
    dominant = "ilu0_apply" if apply_ms >= spmv_ms else "spmv"
    dom_gbs, dom_bytes = (apply_gbs, ab) if dominant == "ilu0_apply" else (spmv_gbs, sb)
    # the same kernels with their inputs coming from HBM: a buffer larger
    # than the Infinity Cache is read before each launch
    flush = torch.empty(512 << 17, dtype=torch.float64, device="cuda").zero_()
    spmv_cold = time_events_cold(lambda: mpk.csr_spmv(A, b, y, stream=s), args.reps, s, flush)
    apply_cold = time_events_cold(lambda: mpk.ilu0_apply(M, b, z, stream=s), args.reps, s, flush)
    del flush
    # HBM traffic per launch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs
    # recorded in profiles/traffic.json, only if they were taken on these
    # kernel sources
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        try:
            tr = json.load(open(tpath))
            if (tr.get("kernel") == dominant and tr.get("grid") == args.grid
                    and tr.get("sources") == kernel_sources_digest()):
                traffic = tr.get("bytes_per_launch")
        except Exception:
            traffic = None

    note("spmv %.4f ms (%.0f GB/s), ilu0 apply %.4f ms (%.0f GB/s)" %
         (spmv_ms, spmv_gbs, apply_ms, apply_gbs))
    cpu = None
    if not args.no_cpu_baseline:
        note("cpu baseline: oracle, %d passes" % args.cpu_passes)
        bh = b.cpu().numpy()
        cpu = cpu_baseline(p, bh, iters, args.cpu_passes)

    out = {
        "metric": "DD time-to-solution at rel. residual 1e-25 (ILU(0)-BiCGSTAB)",
        "value": ms_per_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "dd (2 x f64)",
        "data": "synthetic (seeded 7-point upwind convection-diffusion, x_true ~ U(-1,1))",
        "config": {"workload": "convdiff3d_%d_pe100 BiCGSTAB-DD ILU(0)-D tol 1e-25" % args.grid,
                   "n": p.n, "nnz": p.nnz, "method": "bicgstab", "vector_prec": "DD",
                   "factor_prec": "D", "tol": tol},
        "solves_per_s": 1e3 / ms_per_step,
        "iters": iters,
        "relres_true": info["relres_true"],
        "setup_ms": info["setup_ms"],
        "solve_ms": info["solve_ms"],
        "ms_per_iter": info["solve_ms"] / max(iters, 1),
        "spmv": {"ms": spmv_ms, "gbs": spmv_gbs, "bytes": sb, "frac": spmv_gbs / HBM_PEAK_GBS,
                 "note": "ms/gbs: back to back, the 250 MB working set can stay in the "
                         "256 MiB Infinity Cache; cold_*: a 512 MiB buffer read before each "
                         "launch",
                 "cold_ms": spmv_cold, "cold_gbs": sb / (spmv_cold * 1e-3) / 1e9,
                 "cold_frac": sb / (spmv_cold * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "ilu0_apply": {"ms": apply_ms, "gbs": apply_gbs, "bytes": ab,
                       "frac": apply_gbs / HBM_PEAK_GBS,
                       "cold_ms": apply_cold, "cold_gbs": ab / (apply_cold * 1e-3) / 1e9},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": dom_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom_gbs / HBM_PEAK_GBS,
                     "traffic": traffic, "traffic_source": "profiles/traffic.json (rocprofv3 "
                     "FETCH_SIZE, WRITE_SIZE; null unless taken on these kernel sources)",
                     "algorithmic_bytes": dom_bytes},
        "cpu_baseline": cpu,
    }
    if not args.no_extras:
        del M, y, z, ws, x
        torch.cuda.empty_cache()
        out["multicolour"] = measure_multicolor(p, A, b, tol, max_iter, args.reps,
                                                ms_per_step / 1e3, note)
    del A, b, xt
    torch.cuda.empty_cache()
    if not args.no_extras:
        # the batched and learned forms of the metric, on the same GPU
        out["spmv_random_rows"] = measure_spmv_rows(args.reps, note)
        torch.cuda.empty_cache()
        out["batched"] = measure_batched(args.nsys, 1, 1, args.seq_sample, note)
        torch.cuda.empty_cache()
        out["batched"]["few_large_systems"] = measure_batched_few(16, 200000, note)
        torch.cuda.empty_cache()
        if os.path.exists(PARAMS_FILE):
            params, tinfo = load_params(PARAMS_FILE)
            lr = evaluate_learned(params, tinfo["cap"], tinfo["grid"], args.learned_ntest, note)
            lr["training"] = {k: tinfo[k] for k in ("seconds", "steps", "kept_step", "seed",
                                                   "lr", "validation_ratio", "cap")}
            lr["params_file"] = os.path.relpath(PARAMS_FILE, ROOT)
            out["learned"] = lr
        else:
            out["learned"] = None
            note("no kept parameters at %s: learned comparison skipped" % PARAMS_FILE)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
