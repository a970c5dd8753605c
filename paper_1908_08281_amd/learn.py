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
        g, Z, _, _, st = hgl.weight_grad(ctx.handle, ctx.lam, F, G=grad_F.contiguous().to(F.dtype),
                                         mode=ctx.mode, tol=ctx.tol, want_z=True)
        if st != 0:
            raise RuntimeError(f"adjoint solve did not converge (status {st})")
        grad_w = g if ctx.needs_input_grad[0] else None
        grad_Y = Z if ctx.needs_input_grad[1] else None
        return grad_w, grad_Y, None, None, None, None


def learn_weights(handle, Y: torch.Tensor, lam: float, mu: float, steps: int, w0: torch.Tensor,
                  eta: float | None = None, tol: float = 1e-6, mode: str = "f32", history: bool = False,
                  rr_period: int = 0, rule: str = "projection", strict: bool = True):
    """Descent on the simplex for the adaptive-weight objective.  rule
    "projection": w <- Proj(w - eta g) (hgl_projected_gradient_step);
    "active_set": the steepest-descent step on the Lagrangian of eq. 5 with
    its active constraints (hgl_active_set_step, the step shortened to stay
    feasible).  eta None: the library sets the fixed step from the first
    gradient (0.5 ||w0||_inf / ||g0 - mean(g0)||_inf).  rr_period: periodic
    residual replacement of the forward solves (0: only at the claim checks,
    which verify every column's FP64 residual anyway).  strict: raise when a
    forward or adjoint solve does not converge; otherwise record its status
    and go on.  Returns (w, per-step records); each record holds the forward
    and adjoint statuses ("cg_status", "adjoint_status", 0 = converged)."""
    w = w0.clone()
    recs = []
    eta_dev = None
    for t in range(steps):
        hgl.set_weights(handle, w)
        F, iters, rel, st = hgl.cg_solve(handle, lam, Y, mode=mode, tol=tol, rr_period=rr_period)
        if strict and st != 0:
            raise RuntimeError(f"forward solve did not converge at step {t} (status {st})")
        g, _, ait, _, ast = hgl.weight_grad(handle, lam, F, Y=Y, mu=mu, mode=mode, tol=tol)
        if strict and ast != 0:
            raise RuntimeError(f"adjoint solve did not converge at step {t} (status {ast})")
        info = None
        if rule == "projection":
            w, eta_dev = hgl.projected_gradient_step(w, g, eta)
        elif rule == "active_set":
            if eta is None:
                _, eta_dev = hgl.projected_gradient_step(w, g, None)
            w, info, _ = hgl.active_set_step(w, g, eta if eta is not None else float(eta_dev.item()))
        else:
            raise ValueError(f"unknown rule {rule!r}")
        if eta is None:
            eta = float(eta_dev.item())  # the step set from the first gradient is kept
        if history:
            rec = {"step": t, "cg_iters": int(iters.max()), "adjoint_iters": int(ait.max()),
                   "grad_norm": float(g.norm()), "eta": eta, "cg_status": int(st), "adjoint_status": int(ast)}
            if info is not None:
                rec.update(info)
            recs.append(rec)
    hgl.set_weights(handle, w)
    return w, recs
