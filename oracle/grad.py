"""Derivatives with respect to the hyperedge weights w (section 2, eq. 4).

The paper defers the gradient formula to its reference on steepest-descent
weight updates, so it is derived here from eq. (1).  With s_v = delta(v)^-1/2,
c_e = w_e / delta(e) and A = S H C H' S:

    dA/dw_e = (1/delta(e)) (S h_e)(S h_e)' - 1/2 (D_e A + A D_e),
    D_e = diag(s_v^2 [v in e])

(the second term is the dependence of Dv on w).  For N x k matrices P, Q
    Gamma_e(P, Q) = <P, dA/dw_e Q>
                  = <u_e(P), u_e(Q)>/delta(e)
                    - 1/2 sum_{v in e} s_v^2 (<P_v, (AQ)_v> + <(AP)_v, Q_v>),
    u_e(P) = sum_{v in e} s_v P_v.

Since F = M^-1 Y with M = I + L/lambda = (1 + 1/lambda) I - A/lambda,
    dF/dw_e = M^-1 (dA/dw_e) F / lambda,
so a loss l(F) with G = dl/dF has dl/dw_e = Gamma_e(M^-1 G, F) / lambda.

The adaptive-weight objective used for learning w (the paper's P(w) with the
ranking term and the paper's kappa written mu):
    J(w) = tr(F' L F) + lambda ||F - Y||^2 + mu ||w||^2,  F = F(w),
    dJ/dw_e = -Gamma_e(F, F) + Gamma_e(Z, F)/lambda + 2 mu w_e,
    Z = M^-1 (2 lambda (M F - Y)).
This is the total derivative (Dv depends on w); it is the only reading a
finite-difference check can confirm.
"""
from __future__ import annotations

import numpy as np

from .laplacian import (adjacency, edge_degrees, incidence_dense, inv_sqrt_degrees,
                        system_matrix, laplacian, vertex_degrees)
from .solve import solve_dense


def gamma(H: np.ndarray, w, P: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """Gamma_e(P, Q) for every edge e, written per edge from dA/dw_e."""
    w = np.asarray(w, dtype=np.float64)
    s = inv_sqrt_degrees(vertex_degrees(H, w))
    de = edge_degrees(H)
    A = adjacency(H, w)
    AP, AQ = A @ P, A @ Q
    out = np.zeros(H.shape[1])
    for e in range(H.shape[1]):
        mem = np.nonzero(H[:, e])[0]
        uP = (s[mem, None] * P[mem]).sum(axis=0)
        uQ = (s[mem, None] * Q[mem]).sum(axis=0)
        vt = np.sum(s[mem] ** 2 * (np.einsum("ij,ij->i", P[mem], AQ[mem])
                                   + np.einsum("ij,ij->i", AP[mem], Q[mem])))
        out[e] = uP @ uQ / de[e] - 0.5 * vt
    return out


def dA_dw_dense(H: np.ndarray, w, e: int) -> np.ndarray:
    """dA/dw_e as a dense matrix (for tiny cross-checks)."""
    w = np.asarray(w, dtype=np.float64)
    s = inv_sqrt_degrees(vertex_degrees(H, w))
    de = edge_degrees(H)
    A = adjacency(H, w)
    he = s * H[:, e]
    De = np.diag(s ** 2 * H[:, e])
    return np.outer(he, he) / de[e] - 0.5 * (De @ A + A @ De)


def solve_vjp(H: np.ndarray, w, lam: float, Y: np.ndarray, G: np.ndarray):
    """For F = M^-1 Y and upstream G = dl/dF: (dl/dw, dl/dY = M^-1 G, F)."""
    M = system_matrix(H, w, lam)
    F = solve_dense(M, Y)
    Z = solve_dense(M, G)
    return gamma(H, w, Z, F) / lam, Z, F


def objective(H: np.ndarray, w, lam: float, mu: float, Y: np.ndarray) -> float:
    """J(w) = tr(F'LF) + lambda ||F - Y||^2 + mu ||w||^2 with F = M(w)^-1 Y."""
    w = np.asarray(w, dtype=np.float64)
    F = solve_dense(system_matrix(H, w, lam), Y)
    L = laplacian(H, w)
    return float(np.sum(F * (L @ F)) + lam * np.sum((F - Y) ** 2) + mu * w @ w)


def objective_grad(H: np.ndarray, w, lam: float, mu: float, Y: np.ndarray, F=None):
    """dJ/dw (total derivative); F may be an approximate solve (then the
    adjoint term corrects for it)."""
    w = np.asarray(w, dtype=np.float64)
    M = system_matrix(H, w, lam)
    if F is None:
        F = solve_dense(M, Y)
    G = 2.0 * lam * (M @ F - Y)
    Z = solve_dense(M, G)
    return -gamma(H, w, F, F) + gamma(H, w, Z, F) / lam + 2.0 * mu * w


def gamma_sparse(op, P: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """Gamma_e(P, Q) for every edge from a ``laplacian.SparseOperator`` (same
    formula as ``gamma``, written with sparse products for large N)."""
    s, HT = op.s, op.HT
    de = np.asarray(HT.sum(axis=1)).ravel()
    uP = HT @ (s[:, None] * P)
    uQ = HT @ (s[:, None] * Q)
    AP, AQ = op.adjacency_apply(P), op.adjacency_apply(Q)
    t = s ** 2 * (np.einsum("ij,ij->i", P, AQ) + np.einsum("ij,ij->i", AP, Q))
    return np.einsum("ij,ij->i", uP, uQ) / de - 0.5 * (HT @ t)


def objective_grad_sparse(op, w, lam: float, mu: float, Y: np.ndarray, F: np.ndarray, tol: float = 1e-13):
    """dJ/dw with the sparse tier: the adjoint Z = M^-1 (2 lam (M F - Y)) by
    FP64 CG (eqs. 16-20) to relres tol."""
    from .solve import cg_ranking
    G = 2.0 * lam * (op(F) - Y)
    Z, _, _ = cg_ranking(op, w, lam, G, tol=tol)
    # cg_ranking solves X z = lam/(1+lam) g, i.e. M z = g
    return -gamma_sparse(op, F, F) + gamma_sparse(op, Z, F) / lam + 2.0 * mu * np.asarray(w)


def central_difference(fun, w, e: int, h: float) -> float:
    wp = np.array(w, dtype=np.float64)
    wm = wp.copy()
    wp[e] += h
    wm[e] -= h
    return (fun(wp) - fun(wm)) / (2.0 * h)


def richardson_difference(fun, w, e: int, h: float) -> float:
    """(4 D(h/2) - D(h)) / 3: cancels the h^2 term of the central difference."""
    return (4.0 * central_difference(fun, w, e, h / 2) - central_difference(fun, w, e, h)) / 3.0
