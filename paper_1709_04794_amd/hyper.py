"""Hold-out loss of the FSDA ratings as a differentiable function of (log beta, alpha).

``HoldoutLoss.apply(log_beta, alpha, objective)`` returns the loss per shift
H_s = 1/2 ||X_ho w_s - y_ho||^2 / n_ho, w_s the solution for beta_s =
exp(log_beta_s) on the operator with weight alpha.  Its backward pass is the
adjoint method: one batched solve A(beta_s) lambda_s = dH_s/dw_s for all
shifts (fsda_solve_columns), then dH_s/dlog beta_s = -beta_s <lambda_s, w_s> and
dH_s/dalpha = -<X lambda_s, [L - (P_l - 1_l 1_l^T/l)] X w_s>
(fsda_hypergradient).

``HoldoutLossBatch.apply(log_beta, alpha, objective)`` does the same for many
targets at once (each with its own training labeled set and held-out rows):
the forward solve is fsda_multishift_solve_batch, the loss [ntarget, S] comes
from fsda_holdout_batch, and the backward pass solves the ntarget x S adjoint
systems with fsda_solve_columns_batch and forms the gradient with
fsda_hypergradient_batch; the gradient in log beta_s sums over the targets.

Every step runs in the library's kernels; this module only moves arguments.
A forward or adjoint solve that stops short of its tolerance raises
``NotConverged`` instead of returning a gradient of an unconverged iterate.
"""
from __future__ import annotations

import numpy as np

from . import Operator, OK


class NotConverged(RuntimeError):
    """A solve behind the loss or its gradient did not reach its tolerance."""


def _require(status: int, relres, rtol: float, what: str) -> None:
    worst = float(np.max(relres)) if np.size(relres) else 0.0
    if status != OK or not np.isfinite(worst):
        raise NotConverged("%s: status %d, worst true relative residual %.3e (rtol %.1e)" % (what, status, worst, rtol))


class Objective:
    """The fixed parts of the objective: the problem (X, S, labeled set), the
    held-out rows and their targets, and the solve tolerance.  Operators are
    built per alpha and cached."""

    def __init__(self, pb, ho_idx, ho_y, rtol: float = 1e-10, maxit: int = 100000, device: str = "cuda"):
        import torch
        self.pb = pb
        self.rtol, self.maxit = float(rtol), int(maxit)
        self.ho_idx = torch.as_tensor(np.ascontiguousarray(ho_idx, dtype=np.int32)).to(device)
        self.ho_y = torch.as_tensor(np.ascontiguousarray(ho_y, dtype=np.float64)).to(device)
        self._ops = {}

    def operator(self, alpha: float) -> Operator:
        a = float(alpha)
        if a not in self._ops:
            self._ops[a] = Operator.from_problem(self.pb, alpha=a, max_shifts=64)
        return self._ops[a]


class BatchObjective(Objective):
    """Many targets over one X and graph: ``train`` is a list of (lab_idx,
    lab_y) pairs (each target's training labels), ``heldout`` a list of
    (ho_idx, ho_y) pairs (its held-out rows and +-1 targets), as made by
    ``synth.holdout_splits``."""

    def __init__(self, pb, train, heldout, rtol: float = 1e-10, maxit: int = 100000, device: str = "cuda"):
        import torch
        if len(train) != len(heldout):
            raise ValueError("one held-out set per target")
        self.pb = pb
        self.rtol, self.maxit = float(rtol), int(maxit)
        self.train = [(np.ascontiguousarray(i, dtype=np.int32), np.ascontiguousarray(y, dtype=np.int8))
                      for i, y in train]
        self.heldout = [(torch.as_tensor(np.ascontiguousarray(i, dtype=np.int32)).to(device),
                         torch.as_tensor(np.ascontiguousarray(y, dtype=np.float64)).to(device)) for i, y in heldout]
        self._ops = {}


def _torch_functions():
    import torch

    class HoldoutLoss(torch.autograd.Function):
        @staticmethod
        def forward(ctx, log_beta, alpha, objective):
            betas = torch.exp(log_beta.detach()).cpu().numpy().astype(np.float64)
            op = objective.operator(float(alpha))
            W, iters, relres, st = op.solve(betas, rtol=objective.rtol, maxit=objective.maxit)
            _require(st, relres, objective.rtol, "forward solve")
            loss, G = op.holdout(W, objective.ho_idx, objective.ho_y, gradient=True)
            ctx.objective, ctx.alpha, ctx.betas = objective, float(alpha), betas
            ctx.W, ctx.G = W, G
            return torch.as_tensor(loss, dtype=log_beta.dtype, device=log_beta.device)

        @staticmethod
        def backward(ctx, grad_out):
            op = ctx.objective.operator(ctx.alpha)
            Lam, iters, relres, st = op.solve_columns(ctx.G, ctx.betas, rtol=ctx.objective.rtol,
                                                      maxit=ctx.objective.maxit)
            _require(st, relres, ctx.objective.rtol, "adjoint solve")
            dlb, da = op.hypergradient(ctx.W, Lam, ctx.betas)
            g = grad_out.detach().cpu().numpy()
            grad_lb = torch.as_tensor(g * dlb, dtype=grad_out.dtype, device=grad_out.device)
            grad_a = torch.as_tensor(float((g * da).sum()), dtype=grad_out.dtype, device=grad_out.device)
            return grad_lb, grad_a, None

    class HoldoutLossBatch(torch.autograd.Function):
        @staticmethod
        def forward(ctx, log_beta, alpha, objective):
            betas = torch.exp(log_beta.detach()).cpu().numpy().astype(np.float64)
            op = objective.operator(float(alpha))
            W, iters, relres, st = op.solve_batch(objective.train, betas, rtol=objective.rtol, maxit=objective.maxit)
            _require(st, relres, objective.rtol, "forward solve")
            loss, G = op.holdout_batch(W, objective.heldout, gradient=True)
            ctx.objective, ctx.alpha, ctx.betas = objective, float(alpha), betas
            ctx.W, ctx.G = W, G
            return torch.as_tensor(loss, dtype=log_beta.dtype, device=log_beta.device)

        @staticmethod
        def backward(ctx, grad_out):
            obj = ctx.objective
            op = obj.operator(ctx.alpha)
            Lam, iters, relres, st = op.solve_columns_batch(obj.train, ctx.betas, ctx.G, rtol=obj.rtol,
                                                            maxit=obj.maxit)
            _require(st, relres, obj.rtol, "adjoint solve")
            dlb, da = op.hypergradient_batch(obj.train, ctx.W, Lam, ctx.betas)
            g = grad_out.detach().cpu().numpy()
            grad_lb = torch.as_tensor((g * dlb).sum(axis=0), dtype=grad_out.dtype, device=grad_out.device)
            grad_a = torch.as_tensor(float((g * da).sum()), dtype=grad_out.dtype, device=grad_out.device)
            return grad_lb, grad_a, None

    return HoldoutLoss, HoldoutLossBatch


HoldoutLoss = HoldoutLossBatch = None
try:  # torch is a dependency of the binding; keep the import lazy-tolerant for docs tools
    HoldoutLoss, HoldoutLossBatch = _torch_functions()
except ImportError:  # pragma: no cover
    pass
