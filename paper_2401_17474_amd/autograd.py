"""Differentiable least-squares solve built on the library's Kaczmarz solvers.

``RKASolve.apply(A, b, opts)`` returns x = argmin ||A x - b|| (the
least-squares problem of arXiv 2401.17474, Eq. (2)), computed by the
refinement sweeps of ``rka_refine_solve`` with the residual projected onto
range(A) (so x is the least-squares solution itself, not a point on RKA's
convergence horizon).  Its backward is implicit: for an upstream gradient
g = dL/dx,

    z      = the minimum-norm solution of A^T z = g      (= dL/db)
             -- Kaczmarz on the columns of A started from zero, which
             converges to the minimum-norm solution (Sec. 2.1), refined, in
             FP64 arithmetic over the stored A;
    lambda = the solution of A lambda = z                 (consistent: z lies
             in range(A)), by RKA, refined;
    dL/dA  = r lambda^T - z x^T  with r = b - A x          (rka_lsq_grad_A).

Every step runs in the library's kernels through the C ABI; this module only
sequences the calls.  The forward and the two backward solves draw their
rows from independent streams (seeds seed, seed + 1, seed + 2).  The forward
makes one plan of A and one of A^T (row norms and running sums, Eq. (4)),
which the backward's solves reuse.
"""
from __future__ import annotations

from dataclasses import dataclass

from . import Plan, gemv, lsq_grad_A, refine_solve, transpose


@dataclass
class SolveOpts:
    q: int = 16                 # inner workers
    alpha: float = 1.0          # inner relaxation (alpha* of Eq. (6) converges fastest)
    inner_iters: int = 2000     # iterations of each inner solve
    range_iters: int = 2000     # iterations of each column solve in the forward
    sweeps: int = 4             # refinement sweeps of each solve
    tol: float = 0.0            # stop a solve early once its residual measure <= tol
    accumulate: int = 1         # inner arithmetic: 1 = FP32 (narrow storage), 0 = FP64
    seed: int = 1


def _torch():
    import torch
    return torch


def _solve(P, rhs, o: SolveOpts, seed, Pt=None, range_iters=0, acc=None):
    """Refined solve on the plan P's matrix (Pt: plan of its transpose, for
    the range projection)."""
    if acc is None:
        acc = o.accumulate
    if P.A.dtype == _torch().float64:
        acc = 0
    x, info = refine_solve(None, rhs, plan=P, plan_t=Pt, method=0, q=o.q, accumulate=acc,
                           alpha=o.alpha, inner_iters=o.inner_iters, range_iters=range_iters,
                           range_q=o.q, range_alpha=o.alpha, max_sweeps=o.sweeps, tol=o.tol,
                           seed=seed)
    return x, info


class RKASolve(_torch().autograd.Function):
    """x = argmin ||A x - b||; A (m x n, float64 or float32, m >= n, full column
    rank) and b (float64) on the GPU.  Gradients: dA in A's dtype, db float64."""

    @staticmethod
    def forward(ctx, A, b, opts=None):
        o = opts or SolveOpts()
        At = transpose(A)
        PA, PT = Plan(A), Plan(At)
        x, info = _solve(PA, b, o, o.seed, Pt=PT, range_iters=o.range_iters)
        ctx.save_for_backward(A, At, b, x)
        ctx.plans = (PA, PT)
        ctx.opts = o
        ctx.forward_info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        torch = _torch()
        A, At, b, x = ctx.saved_tensors
        PA, PT = ctx.plans
        o = ctx.opts
        g = gx.to(torch.float64).contiguous()
        # min-norm A^T z = g.  Always FP64 arithmetic: rounding errors of the
        # updates land mostly in null(A^T), which the residual g - A^T z
        # cannot see, so refinement would never remove binary32 ones.
        z, _ = _solve(PT, g, o, o.seed + 1, acc=0)
        lam, _ = _solve(PA, z, o, o.seed + 2)          # A lambda = z
        r = gemv(A, x, c=b, gamma=-1.0)                # r = b - A x
        dA = lsq_grad_A(r, lam, z, x, dtype=A.dtype if A.dtype == torch.float64
                        else torch.float32)
        return dA, z, None


def lsq_solve(A, b, opts: SolveOpts | None = None):
    """Differentiable least-squares solve (see RKASolve)."""
    torch = _torch()
    if A.dtype not in (torch.float64, torch.float32):
        raise TypeError("the differentiable solve takes float64 or float32 A")
    return RKASolve.apply(A, b, opts)
