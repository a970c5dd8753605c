"""Algorithm 1 (randomized SVD via subspace iteration), its power-scheme
variant (eq. 10), the diagonal-block tessellation (eq. 11) and the block
inverse (eq. 15), FP64.

Readings:
* the paper writes pi both for the oversampling (l = k + pi) and for the number
  of subspace iterations of Algorithm 1; here p is the oversampling and q the
  number of iterations.
* the diagonal blocks of X = I - A/(1+theta) are full-rank (their eigenvalues
  lie in [theta/(1+theta), 1]); the low-rank object is the block A_bb of the
  normalised adjacency, so Algorithm 1 is run on A_bb.
* eq. (15) inverts a truncated SVD; a rank-k truncation of a full-rank block
  is not an inverse, so the block inverse used here is the exact
  identity-plus-low-rank form
      M_bb^-1 ~ lambda/(1+lambda) [I + U diag(s_i / (1 + lambda - s_i)) U'],
  which equals (I + L_bb/lambda)^-1 whenever rank(A_bb) <= k, and the solve
  is finished by preconditioned CG on the full system.
* the QR factorisation is LAPACK Householder here; any QR gives the same
  subspaces, and S is compared only through sign- and rotation-invariant
  quantities.
"""
from __future__ import annotations

import numpy as np


def tessellate(M: np.ndarray, offsets) -> list[np.ndarray]:
    """Diagonal blocks M[o_b:o_{b+1}, o_b:o_{b+1}] (eq. 11 applied recursively)."""
    return [M[offsets[b]:offsets[b + 1], offsets[b]:offsets[b + 1]].copy()
            for b in range(len(offsets) - 1)]


def orth(Y: np.ndarray) -> np.ndarray:
    """Orthonormal basis S of range(Y) from a QR factorisation Y = S R."""
    S, _ = np.linalg.qr(Y, mode="reduced")
    return S


def randomized_svd(X: np.ndarray, Omega: np.ndarray, q: int):
    """Algorithm 1 for an m x m matrix X with sketch Omega (m x l), q iterations.

    Y0 = X Omega, Y0 = S0 R0; for i = 1..q: Yt = X' S_{i-1} = St Rt,
    Y_i = X St = S_i R_i; S = S_q; B = S' X; B = Ut Sigma V'; U = S Ut.
    Returns (U, sigma, V) with sigma in decreasing order.
    """
    S = orth(X @ Omega)
    for _ in range(q):
        St = orth(X.T @ S)
        S = orth(X @ St)
    B = S.T @ X
    Ut, sigma, Vt = np.linalg.svd(B, full_matrices=False)
    return S @ Ut, sigma, Vt.T


def power_sketch(X: np.ndarray, Omega: np.ndarray, q: int) -> np.ndarray:
    """Eq. (10): Y = (X X')^q X Omega, formed by repeated products with no
    orthonormalisation in between (the exponent is the number of iterations
    q; the paper reuses the oversampling's symbol for it)."""
    Y = X @ Omega
    for _ in range(q):
        Y = X @ (X.T @ Y)
    return Y


def randomized_svd_power(X: np.ndarray, Omega: np.ndarray, q: int):
    """Algorithm 1 with steps 2-3 replaced by eq. (10): S is an orthonormal
    basis of range((X X')^q X Omega) from one QR factorisation, then B = S'X,
    B = Ut Sigma V', U = S Ut as in steps 4-6.  In exact arithmetic S spans
    the subspace of Algorithm 1; in floating point the directions of small
    singular values are lost to rounding as q grows (the paper's caveat)."""
    S = orth(power_sketch(X, Omega, q))
    B = S.T @ X
    Ut, sigma, Vt = np.linalg.svd(B, full_matrices=False)
    return S @ Ut, sigma, Vt.T


def block_inverse_factors(A_blocks, omegas, k: int, q: int, scheme: str = "subspace"):
    """Per block: leading-k (U_b, sigma_b) of Algorithm 1 on A_bb
    (scheme "power": with the sketch of eq. (10) in place of steps 2-3)."""
    if scheme not in ("subspace", "power"):
        raise ValueError(f"unknown scheme {scheme!r}")
    svd = randomized_svd if scheme == "subspace" else randomized_svd_power
    out = []
    for Ab, Om in zip(A_blocks, omegas):
        U, s, _ = svd(Ab, Om, q)
        kk = min(k, s.size)
        out.append((U[:, :kk], s[:kk]))
    return out


def block_inverse_apply(factors, offsets, lam: float, R: np.ndarray) -> np.ndarray:
    """Z = blockdiag(M_bb^-1 approx) R, with the identity-plus-low-rank form."""
    Z = np.empty_like(R, dtype=np.float64)
    g = lam / (1.0 + lam)
    for b, (U, s) in enumerate(factors):
        o0, o1 = offsets[b], offsets[b + 1]
        Rb = R[o0:o1]
        d = s / (1.0 + lam - s)
        Z[o0:o1] = g * (Rb + U @ (d[:, None] * (U.T @ Rb)))
    return Z


def preconditioned_cg(apply_M, apply_P, Y: np.ndarray, tol: float, max_iter: int):
    """Per-column preconditioned CG for M F = Y (Barrett et al. templates).

    z = P r; alpha = r'z / p'Mp; f += alpha p; r -= alpha M p;
    beta = r_new'z_new / r'z; p = z + beta p.  Stops on the true relres.
    The starting guess is f0 = P y (the block inverse applied to the query).
    """
    Y = np.asarray(Y, dtype=np.float64)
    n, k = Y.shape
    yn = np.linalg.norm(Y, axis=0)
    F = apply_P(Y)
    F[:, yn == 0] = 0.0
    R = Y - apply_M(F)
    Z = apply_P(R)
    P = Z.copy()
    rz = np.einsum("ij,ij->j", R, Z)
    active = yn > 0
    iters = np.zeros(k, dtype=np.int64)
    rel = np.zeros(k)
    rel[active] = np.linalg.norm(R[:, active], axis=0) / yn[active]
    active &= rel > tol
    for _ in range(max_iter):
        if not active.any():
            break
        c = np.nonzero(active)[0]
        MP = apply_M(P[:, c])
        alpha = rz[c] / np.einsum("ij,ij->j", P[:, c], MP)
        F[:, c] += alpha * P[:, c]
        R[:, c] -= alpha * MP
        Zc = apply_P(R[:, c])
        rz_new = np.einsum("ij,ij->j", R[:, c], Zc)
        beta = rz_new / rz[c]
        P[:, c] = Zc + beta * P[:, c]
        rz[c] = rz_new
        iters[c] += 1
        Rt = Y[:, c] - apply_M(F[:, c])
        rel[c] = np.linalg.norm(Rt, axis=0) / yn[c]
        active[c[rel[c] <= tol]] = False
    return F, iters, rel
