"""The block inverse through Schur complements (eqs. 12-14) under nested
tessellation along the main diagonal, with the inverse from the SVD (eq. 15)
at the smallest submatrices; FP64.

Test infrastructure: imported only by the tests, smoke() and the bench's CPU
baseline, never by the library.

Readings:
* eq. 12 splits a square matrix into a 2x2 block matrix with square diagonal
  blocks; here the first diagonal block holds floor(n/2) rows.
* the minimum "rank" of the nested tessellation is the size of its smallest
  diagonal submatrices: a submatrix is halved while both halves keep at least
  min_block rows (n >= 2 min_block), so the smallest ones hold min_block to
  2 min_block - 1 rows, and a matrix smaller than 2 min_block is not split.
* under nested tessellation the four inverses the text leaves to the
  randomized SVD (X11^-1, X22^-1, Z1^-1, Z2^-1) are the same 2x2 construction
  one level down; only the smallest submatrices are inverted by eq. 15, with
  all their singular values (a randomized SVD whose sketch is at least as wide
  as the submatrix returns exactly those), so the whole construction is the
  exact inverse up to rounding.
* eq. 13 (Z1) is the Schur complement of X22, eq. 14 (Z2) that of X11; the
  inverse of eq. 12 is [[Z1^-1, -X11^-1 X12 Z2^-1], [-Z2^-1 X21 X11^-1, Z2^-1]].
  The formula needs no symmetry; the tests use it on nonsymmetric matrices so
  that a transposed operand shows.
"""
from __future__ import annotations

import numpy as np

from . import laplacian as lap


def split_point(n: int, min_block: int):
    """Rows of the first diagonal block when an n x n submatrix is split, or
    None when it is one of the smallest submatrices."""
    if min_block < 1:
        raise ValueError("min_block must be >= 1")
    return n // 2 if n >= 2 * min_block else None


def nested_tessellation(n: int, min_block: int, offset: int = 0) -> list[tuple[int, int]]:
    """(first row, rows) of the smallest diagonal submatrices, in order."""
    n1 = split_point(n, min_block)
    if n1 is None:
        return [(offset, n)]
    return nested_tessellation(n1, min_block, offset) + nested_tessellation(n - n1, min_block, offset + n1)


def svd_inverse(X: np.ndarray) -> np.ndarray:
    """Eq. 15: X = U Sigma V' gives X^-1 = V Sigma^-1 U'."""
    U, s, Vt = np.linalg.svd(np.asarray(X, dtype=np.float64))
    return Vt.T @ (U.T / s[:, None])


def schur_inverse(X: np.ndarray, min_block: int) -> np.ndarray:
    """Eqs. 12-14 applied recursively down to the nested tessellation's
    smallest submatrices, which eq. 15 inverts."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    n1 = split_point(n, min_block)
    if n1 is None:
        return svd_inverse(X)
    X11, X12 = X[:n1, :n1], X[:n1, n1:]
    X21, X22 = X[n1:, :n1], X[n1:, n1:]
    X11i = schur_inverse(X11, min_block)
    X22i = schur_inverse(X22, min_block)
    Z1 = X11 - X12 @ X22i @ X21          # eq. 13
    Z2 = X22 - X21 @ X11i @ X12          # eq. 14
    Z1i = schur_inverse(Z1, min_block)
    Z2i = schur_inverse(Z2, min_block)
    return np.block([[Z1i, -X11i @ X12 @ Z2i],
                     [-Z2i @ X21 @ X11i, Z2i]])


def block_schur_inverses(M_blocks, min_block: int) -> list[np.ndarray]:
    """The inverse of every diagonal block of the tessellation (eq. 11)."""
    return [schur_inverse(Mb, min_block) for Mb in M_blocks]


def block_dense_apply(inverses, offsets, R: np.ndarray) -> np.ndarray:
    """Z = blockdiag(M_bb^-1) R."""
    R = np.asarray(R, dtype=np.float64)
    Z = np.empty_like(R)
    for b, Mi in enumerate(inverses):
        o0, o1 = offsets[b], offsets[b + 1]
        Z[o0:o1] = Mi @ R[o0:o1]
    return Z


def system_block(H_csr, w, lam: float, o0: int, o1: int) -> np.ndarray:
    """M_bb = (I + L/lambda)[o0:o1, o0:o1] from a sparse incidence (vertex x
    edge, SciPy CSR), without forming the whole matrix:
    A_bb = S_b H_b W De^-1 H_b' S_b with S = Dv^-1/2 (eq. 1)."""
    w = np.asarray(w, dtype=np.float64)
    s = lap.inv_sqrt_degrees(lap.vertex_degrees(H_csr, w))
    de = lap.edge_degrees(H_csr)
    c = np.where(de > 0, w / np.where(de > 0, de, 1.0), 0.0)
    Hb = H_csr[o0:o1]
    Ab = (Hb.multiply(c[None, :]) @ Hb.T).toarray()
    Ab = s[o0:o1, None] * Ab * s[None, o0:o1]
    return (1.0 + 1.0 / lam) * np.eye(o1 - o0) - Ab / lam
