"""Hypergraph operators, section 2 of the paper (FP64, dense and sparse).

Notation: m = |V| vertices (N here), n = |E| hyperedges, binary incidence
H(v, e) = 1 iff v in e, vertex degree delta(v) = sum_e w(e) H(v, e), edge
degree delta(e) = sum_v H(v, e), A = Dv^-1/2 H W De^-1 H' Dv^-1/2 (eq. 1),
L = I - A (Zhou's normalised Laplacian), X = I - A/(1 + theta).

Readings where the paper is silent or garbled:
* the edge-degree diagonal is written "D_v in R^{n x n}" in section 2; it is
  the hyperedge degree matrix D_e;
* a vertex with delta(v) = 0 (in no hyperedge, or only in zero-weight ones)
  has no defined Dv^-1/2; its scale is taken as 0 (pseudo-inverse), so its row
  and column of A are zero and its diagonal of L is 1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def incidence_dense(N: int, E: int, edge_ptr, edge_vtx) -> np.ndarray:
    """H in {0,1}^{N x E} from the edge-major lists (section 2)."""
    H = np.zeros((N, E), dtype=np.float64)
    for e in range(E):
        for j in range(int(edge_ptr[e]), int(edge_ptr[e + 1])):
            H[int(edge_vtx[j]), e] = 1.0
    return H


def incidence_sparse(N: int, E: int, edge_ptr, edge_vtx) -> sp.csr_matrix:
    """Same H as a SciPy CSR matrix (used for matrix-free work at large N)."""
    edge_ptr = np.asarray(edge_ptr, dtype=np.int64)
    cols = np.repeat(np.arange(E), np.diff(edge_ptr))
    rows = np.asarray(edge_vtx, dtype=np.int64)
    return sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(N, E))


def vertex_degrees(H, w) -> np.ndarray:
    """delta(v) = sum_e w(e) H(v, e)."""
    return np.asarray(H @ np.asarray(w, dtype=np.float64)).ravel()


def edge_degrees(H) -> np.ndarray:
    """delta(e) = sum_v H(v, e)."""
    return np.asarray(H.sum(axis=0)).ravel()


def inv_sqrt_degrees(dv: np.ndarray) -> np.ndarray:
    """Diagonal of Dv^-1/2, with 0 where delta(v) = 0 (pseudo-inverse reading)."""
    s = np.zeros_like(dv)
    pos = dv > 0
    s[pos] = 1.0 / np.sqrt(dv[pos])
    return s


def adjacency(H: np.ndarray, w) -> np.ndarray:
    """Eq. (1): A = Dv^-1/2 H W De^-1 H' Dv^-1/2, built densely."""
    w = np.asarray(w, dtype=np.float64)
    Dv_inv_sqrt = np.diag(inv_sqrt_degrees(vertex_degrees(H, w)))
    W = np.diag(w)
    De_inv = np.diag(1.0 / edge_degrees(H))
    return Dv_inv_sqrt @ H @ W @ De_inv @ H.T @ Dv_inv_sqrt


def laplacian(H: np.ndarray, w) -> np.ndarray:
    """Zhou's normalised hypergraph Laplacian L = I - A (section 2)."""
    return np.eye(H.shape[0]) - adjacency(H, w)


def ranking_matrix(H: np.ndarray, w, theta: float) -> np.ndarray:
    """X = I - A / (1 + theta) (section 2, the matrix inverted in eq. 3)."""
    return np.eye(H.shape[0]) - adjacency(H, w) / (1.0 + theta)


def system_matrix(H: np.ndarray, w, lam: float) -> np.ndarray:
    """M = I + L / lambda, the system the library solves: M F = Y.

    With theta = lambda, M = (1 + 1/theta) X, so M f = y is eq. (6)
    multiplied by (1 + theta)/theta and has the same solution f* as eq. (3).
    """
    return np.eye(H.shape[0]) + laplacian(H, w) / lam


class SparseOperator:
    """Matrix-free FP64 M = I + L/lambda from a sparse H (large-N second tier).

    Computes A P = S H C H' S P with S = Dv^-1/2 and C = W De^-1 as two sparse
    products; mathematically identical to the dense eq. (1)."""

    def __init__(self, N, E, edge_ptr, edge_vtx, w, lam):
        self.H = incidence_sparse(N, E, edge_ptr, edge_vtx)
        self.HT = self.H.T.tocsr()
        w = np.asarray(w, dtype=np.float64)
        self.s = inv_sqrt_degrees(vertex_degrees(self.H, w))
        self.c = w / edge_degrees(self.H)
        self.lam = float(lam)
        self.N = N

    def adjacency_apply(self, P: np.ndarray) -> np.ndarray:
        sP = self.s[:, None] * P
        Z = self.c[:, None] * (self.HT @ sP)
        return self.s[:, None] * (self.H @ Z)

    def __call__(self, P: np.ndarray) -> np.ndarray:
        P = np.asarray(P, dtype=np.float64)
        LP = P - self.adjacency_apply(P)
        return P + LP / self.lam
