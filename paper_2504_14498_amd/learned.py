"""Learned correction to the binary64 ILU(0) factor: training data from the
method itself, the training loop and the guarded learned solve.

Every numerical step runs in the HIP library (network forward/backward,
factor loss, Adam, correction, factorisation and solves); this module only
orders the calls.  The paper has no learned part; the network and its
loss are defined in include/mpk.h.

Training data of one system: A, b, its plain ILU(0) factor and probe
vectors: the normalised residuals r_k / ||r_k|| of the plain method at a
few points of a restarted run (the method's own residual history), plus a
few seeded Gaussian directions.  The residual probes pull the factor
towards A on the slowly converging directions; the random ones keep it
close to A everywhere else (without them the loss keeps falling while
some systems stop converging).
"""
import math
import time

import numpy as np
import torch

from . import mpk

PROBE_SEGMENTS = (4, 4, 8, 16)   # restarted plain BiCGSTAB passes between probes
RANDOM_PROBES = 8                # plus this many seeded Gaussian directions


def residual(A, b, x):
    """b - A x in double-word on the device (the library's residual), as
    its leading float64 limb."""
    return mpk.csr_residual(A, b, x)[:, 0, 0]


class Instance:
    """One system on the device with what training or solving needs."""

    def __init__(self, problem, probes=True, segments=PROBE_SEGMENTS, nrandom=RANDOM_PROBES,
                 seed=0):
        p = problem
        self.name = p.name
        self.A = mpk.Csr.from_problem(p)
        xt = torch.as_tensor(p.x_true_limbs(2)).cuda()
        self.b = mpk.csr_spmv(self.A, xt)
        self.M = mpk.ilu0_factor(self.A, fprec=1, vprec=2)
        self.G = mpk.GnnGraph(self.A, self.M)
        self.probes = None
        if probes:
            P = self._probes(segments)
            if nrandom:
                R = np.random.Generator(np.random.PCG64(77_000_000 + seed)).standard_normal(
                    (nrandom, self.A.n))
                R /= np.linalg.norm(R, axis=1, keepdims=True)
                P = torch.cat([P, torch.as_tensor(R, device=P.device)])
            self.probes = P.contiguous()

    def _probes(self, segments):
        A, b = self.A, self.b
        x = torch.zeros_like(b)
        rows = []
        ws = None
        for k in segments:
            x, info = mpk.krylov_solve_precond("bicgstab", A, self.M, b, x0=x, tol_rel=1e-25,
                                               max_iter=k, workspace=ws)
            ws = info["workspace"]
            r = residual(A, b, x)
            nr = torch.linalg.vector_norm(r)
            if not torch.isfinite(nr) or nr == 0:
                break
            rows.append(r / nr)
            if info["status"] == "ok":
                break
        if not rows:
            return torch.zeros((0, A.n), dtype=torch.float64, device=b.device)
        return torch.stack(rows).contiguous()


class Trainer:
    """Adam on the factor loss, one system per step."""

    def __init__(self, seed=0, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, device="cuda"):
        self.params = mpk.gnn_init(seed, device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step_count = 0
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps
        self._ws = None
        self._lws = None

    def _gnn_ws(self, A):
        need = mpk.library().mpk_gnn_workspace_bytes(mpk.ctypes.byref(A.c))
        if self._ws is None or self._ws[2] < need:
            self._ws = mpk.gnn_workspace(A)
        return self._ws

    def loss(self, inst, params=None):
        """Factor loss of the current (or given) parameters on inst."""
        params = self.params if params is None else params
        delta, _ = mpk.gnn_forward(inst.G, params, workspace=self._gnn_ws(inst.A))
        loss, _, self._lws = mpk.gnn_factor_loss(inst.G, inst.M, delta, inst.probes, grad=False,
                                                 workspace=self._lws)
        return loss

    def step(self, inst):
        """One training step on inst; returns the loss before the update."""
        ws = self._gnn_ws(inst.A)
        delta, _ = mpk.gnn_forward(inst.G, self.params, workspace=ws)
        loss, gd, self._lws = mpk.gnn_factor_loss(inst.G, inst.M, delta, inst.probes,
                                                  workspace=self._lws)
        grad = mpk.gnn_backward(inst.G, self.params, gd, ws)
        self.step_count += 1
        mpk.gnn_adam(self.params, grad, self.m, self.v, self.step_count, self.lr, self.beta1,
                     self.beta2, self.eps)
        return loss


def solve_plain(A, b, tol=1e-25, max_iter=10000):
    """Plain ILU(0)-BiCGSTAB in DD (factor and solve)."""
    t0 = time.perf_counter()
    x, info = mpk.krylov_solve("bicgstab", A, b, fprec=1, tol_rel=tol, max_iter=max_iter)
    torch.cuda.synchronize()
    info = dict(info)
    info["tts_s"] = time.perf_counter() - t0
    return x, info


def solve_learned(A, b, params, iter_cap, tol=1e-25, max_iter=10000):
    """Factor, predict and apply the correction, solve; fall back to plain
    ILU(0) (counted in the time) if the guards reject the correction or the
    learned solve has not converged within iter_cap passes."""
    t0 = time.perf_counter()
    M = mpk.ilu0_factor(A, fprec=1, vprec=2)
    G = mpk.GnnGraph(A, M)
    delta, _ = mpk.gnn_forward(G, params)
    rejected = mpk.ilu0_correct(M, delta)
    spent = 0
    if not rejected:
        x, info = mpk.krylov_solve_precond("bicgstab", A, M, b, tol_rel=tol,
                                           max_iter=int(iter_cap))
        spent = info["iters"]
        if info["status"] == "ok":
            torch.cuda.synchronize()
            info = dict(info)
            info.update(tts_s=time.perf_counter() - t0, fallback=None, iters_total=spent)
            return x, info
    del M, G
    x, info = mpk.krylov_solve("bicgstab", A, b, fprec=1, tol_rel=tol, max_iter=max_iter)
    torch.cuda.synchronize()
    info = dict(info)
    info.update(tts_s=time.perf_counter() - t0,
                fallback="guard" if rejected else "iteration cap",
                iters_total=spent + info["iters"])
    return x, info


def iteration_cap(plain_iters, factor=1.5):
    """The learned solve's budget: factor x the plain method's count,
    estimated from systems of the training distribution (their largest
    plain count)."""
    return int(math.ceil(factor * max(plain_iters)))


def validation_ratio(params, systems, plain_iters, cap):
    """Median over held-out training-distribution systems of learned /
    plain iterations (fallbacks counted): the method itself judges which
    parameters to keep."""
    r = [solve_learned(A, b, params, cap)[1]["iters_total"] / max(pi, 1)
         for (A, b), pi in zip(systems, plain_iters)]
    return float(np.median(r))


def quartiles(v):
    v = np.asarray(v, dtype=np.float64)
    return [float(np.percentile(v, q)) for q in (25, 50, 75)]
