"""Differentiable hypergraph ranking solve and adaptive weight learning.

``HypergraphSolve`` is a ``torch.autograd.Function``: forward solves
(I + L(w)/lam) F = Y with the library's CG; backward returns d/dw through the
hand-written adjoint (one more CG on the symmetric operator plus the
edge contraction Gamma_e) and d/dY = M^-1 dl/dF.

``learn_weights`` runs the alternating scheme of the paper's section 2 (solve
for F with w fixed, then update w with F fixed) as projected gradient descent
on the simplex {w >= 0, 1'w = 1} of eq. (4), for the objective
tr(F'LF) + lam ||F - Y||^2 + mu ||w||^2.
"""
from __future__ import annotations

import torch

from . import hgl


class HypergraphSolve(torch.autograd.Function):
    """F = HypergraphSolve.apply(w, Y, handle, lam, tol, mode)."""

    @staticmethod
    def forward(ctx, w, Y, handle, lam, tol=1e-6, mode="f32"):
        hgl.set_weights(handle, w.detach().contiguous())
        F, iters, rel, st = hgl.cg_solve(handle, lam, Y.detach().contiguous(), mode=mode, tol=tol)
        if st != 0:
            raise RuntimeError(f"forward solve did not converge (status {st})")
        ctx.handle, ctx.lam, ctx.tol, ctx.mode = handle, lam, tol, mode
        ctx.save_for_backward(w, F)
        return F

    @staticmethod
    def backward(ctx, grad_F):
        w, F = ctx.saved_tensors
        hgl.set_weights(ctx.handle, w.detach().contiguous())
        g, Z, _, _ = hgl.weight_grad(ctx.handle, ctx.lam, F, G=grad_F.contiguous().to(F.dtype),
                                     mode=ctx.mode, tol=ctx.tol, want_z=True)
        grad_w = g if ctx.needs_input_grad[0] else None
        grad_Y = Z if ctx.needs_input_grad[1] else None
        return grad_w, grad_Y, None, None, None, None


def learn_weights(handle, Y: torch.Tensor, lam: float, mu: float, steps: int, w0: torch.Tensor,
                  eta: float | None = None, tol: float = 1e-6, mode: str = "f32", history: bool = False,
                  rr_period: int = 0, rule: str = "projection"):
    """Descent on the simplex for the adaptive-weight objective.  rule
    "projection": w <- Proj(w - eta g); "active_set": the steepest-descent
    step on the Lagrangian of eq. 5 with its active constraints
    (hgl.active_set_step, the step shortened to stay feasible).  eta None: fixed step 0.5 ||w0||_inf / ||g0 - mean(g0)||_inf
    chosen at step 0.  rr_period: periodic residual replacement of the
    forward solves (0: only at the claim checks, which verify every column's
    FP64 residual anyway).  Returns (w, per-step records)."""
    w = w0.clone()
    recs = []
    for t in range(steps):
        hgl.set_weights(handle, w)
        F, iters, rel, st = hgl.cg_solve(handle, lam, Y, mode=mode, tol=tol, rr_period=rr_period)
        g, _, ait, _ = hgl.weight_grad(handle, lam, F, Y=Y, mu=mu, mode=mode, tol=tol)
        if eta is None:
            gc = g - g.mean()
            eta = float(0.5 * w.abs().max() / gc.abs().max().clamp_min(1e-300))
        info = None
        if rule == "projection":
            w = hgl.project_simplex(w - eta * g)
        elif rule == "active_set":
            w, info, _ = hgl.active_set_step(w, g, eta)
        else:
            raise ValueError(f"unknown rule {rule!r}")
        if history:
            rec = {"step": t, "cg_iters": int(iters.max()), "adjoint_iters": int(ait.max()),
                   "grad_norm": float(g.norm()), "eta": eta}
            if info is not None:
                rec.update(info)
            recs.append(rec)
    hgl.set_weights(handle, w)
    return w, recs
