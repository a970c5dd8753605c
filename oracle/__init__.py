"""FP64 CPU oracle for the hypergraph ranking solve -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct NumPy/SciPy implementations of what the GPU
library computes, written from the paper (Karantaidis, Sarridis, Kotropoulos,
"Block randomized optimization for adaptive hypergraph learning"):

* ``laplacian``  -- degrees, normalised adjacency A (eq. 1), Zhou's Laplacian
  L = I - A, the ranking system matrix (section 2).
* ``solve``      -- the ranking solution (eq. 3 / eq. 6) by dense Cholesky, and
  conjugate gradient in the paper's recurrences (eqs. 16-20, section 3).
* ``rsvd``       -- Algorithm 1 (randomized SVD by subspace iteration), the
  diagonal-block tessellation (eq. 11) and the block inverse (eq. 15, read as
  the identity-plus-low-rank form), and preconditioned CG.
* ``schur``      -- the 2x2 block inverse through Schur complements (eqs.
  12-14) under nested tessellation, with eq. 15 at the smallest submatrices.
* ``grad``       -- derivative of the weight objective P(w) (eq. 4) and of
  losses through the solve, plus finite differences.
* ``simplex``    -- Euclidean projection onto {w >= 0, 1'w = 1} (constraints of
  eq. 4), and the active-set steepest-descent step on the Lagrangian of eq. 5.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
and imports nothing from it.
"""
from . import laplacian, solve, rsvd, schur, grad, simplex  # noqa: F401
