"""The ranking solve, eqs. (3) and (6), and conjugate gradient, eqs. (16)-(20).

The library solves (I + L/lambda) F = Y column by column.  With theta = lambda
this is eq. (6) scaled by (1 + theta)/theta: minimising f'Lf + theta||f - y||^2
gives (L + theta I) f = theta y, i.e. ((1 + theta) I - A) f = theta y, i.e.
X f = theta/(1 + theta) y.  So every column F_j equals the paper's f* for the
query y = Y_j.

Readings:
* f0 is not given by the paper; f0 = 0 unless a start is passed.
* the stopping rule is not given; a column stops when its true relative
  residual ||y - M f|| / ||y|| (recomputed from f, not the recurrence) is at
  most tol; the residual of eq. (6) gives the same ratio.
* a zero query column has the solution 0 and counts as converged at once.
* "many tag columns" means independent columns, each with its own alpha and
  beta (each test image is its own query in the paper), not block CG.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def solve_dense(M: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """F = M^-1 Y by Cholesky (LAPACK potrf/potrs); M is SPD."""
    c = sla.cho_factor(M, lower=True)
    return sla.cho_solve(c, Y)


def ranking_solution(X: np.ndarray, y: np.ndarray, theta: float) -> np.ndarray:
    """Eq. (3): f* = theta/(1+theta) X^-1 y (dense)."""
    return theta / (1.0 + theta) * np.linalg.solve(X, y)


def relres(apply_M, F: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Per-column ||Y_j - M F_j|| / ||Y_j|| (0 for a zero column with F_j = 0)."""
    R = Y - apply_M(F)
    rn = np.linalg.norm(R, axis=0)
    yn = np.linalg.norm(Y, axis=0)
    out = np.where(yn > 0, rn / np.where(yn > 0, yn, 1.0), rn)
    return out


def conjugate_gradient(apply_X, b: np.ndarray, tol: float, max_iter: int,
                       f0: np.ndarray | None = None):
    """Eqs. (16)-(20) for X f = b, one independent recurrence per column.

    r0 = b - X f0, p0 = r0; for i >= 1:
        alpha_i = r'r / p'Xp          (19)
        f_i = f_{i-1} + alpha_i p     (16)
        r_i = r_{i-1} - alpha_i X p   (17)
        beta_i = r_i'r_i / r'r        (20)
        p_i = r_i + beta_i p          (18)
    A column stops when ||b - X f|| / ||b|| <= tol (true residual).
    Returns (f, iterations per column, true relres per column).
    """
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 1:
        b = b[:, None]
    n, k = b.shape
    f = np.zeros_like(b) if f0 is None else np.array(f0, dtype=np.float64).reshape(n, k)
    r = b - apply_X(f)
    p = r.copy()
    rr = np.einsum("ij,ij->j", r, r)
    bn = np.linalg.norm(b, axis=0)
    active = bn > 0
    f[:, ~active] = 0.0
    iters = np.zeros(k, dtype=np.int64)
    true_rel = np.zeros(k)

    def true_relres(cols):
        rt = b[:, cols] - apply_X(f[:, cols])
        return np.linalg.norm(rt, axis=0) / bn[cols]

    if active.any():
        cols = np.nonzero(active)[0]
        tr = true_relres(cols)
        true_rel[cols] = tr
        active[cols[tr <= tol]] = False
    for _ in range(max_iter):
        if not active.any():
            break
        cols = np.nonzero(active)[0]
        pc = p[:, cols]
        Xp = apply_X(pc)
        pXp = np.einsum("ij,ij->j", pc, Xp)
        alpha = rr[cols] / pXp
        f[:, cols] += alpha * pc
        r[:, cols] -= alpha * Xp
        rr_new = np.einsum("ij,ij->j", r[:, cols], r[:, cols])
        beta = rr_new / rr[cols]
        p[:, cols] = r[:, cols] + beta * pc
        rr[cols] = rr_new
        iters[cols] += 1
        tr = true_relres(cols)
        true_rel[cols] = tr
        active[cols[tr <= tol]] = False
    return f, iters, true_rel


def cg_ranking(H_or_op, w, theta: float, Y: np.ndarray, tol: float, max_iter: int = 10_000):
    """CG on the paper's system X f = theta/(1+theta) y for every column of Y.

    ``H_or_op`` is either a dense incidence matrix or an object with an
    ``adjacency_apply`` method (the sparse second tier).
    """
    from .laplacian import adjacency
    if hasattr(H_or_op, "adjacency_apply"):
        def apply_X(P):
            return P - H_or_op.adjacency_apply(P) / (1.0 + theta)
    else:
        A = adjacency(H_or_op, w)

        def apply_X(P):
            return P - A @ P / (1.0 + theta)
    b = theta / (1.0 + theta) * np.asarray(Y, dtype=np.float64)
    return conjugate_gradient(apply_X, b, tol, max_iter)
