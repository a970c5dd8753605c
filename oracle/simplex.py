"""Euclidean projection onto the simplex {w >= 0, 1'w = 1}, the feasible set
of eq. (4).

The paper updates w by steepest descent on a Lagrangian with active-set
multipliers (eq. 5); the projected-gradient form w+ = Proj(w - eta g) uses the
same constraints.  The projection is max(v - tau, 0) with tau chosen so the
result sums to one (Held, Wolfe and Crowder 1974; Duchi et al. 2008); found
here by sorting.
"""
from __future__ import annotations

import numpy as np


def project(v) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    u = np.sort(v)[::-1]
    css = np.cumsum(u)
    j = np.arange(1, v.size + 1)
    cond = u - (css - 1.0) / j > 0
    rho = int(np.nonzero(cond)[0][-1])
    tau = (css[rho] - 1.0) / (rho + 1)
    return np.maximum(v - tau, 0.0)


def project_bruteforce(v) -> np.ndarray:
    """Enumerate supports: for each nonempty support S, the minimiser of
    ||w - v||^2 on {w_S sums to 1, w outside S = 0} is v_S - (sum v_S - 1)/|S|;
    keep the feasible (nonnegative) one with the smallest distance."""
    v = np.asarray(v, dtype=np.float64)
    n = v.size
    best, best_d = None, np.inf
    for mask in range(1, 1 << n):
        S = [i for i in range(n) if mask >> i & 1]
        w = np.zeros(n)
        w[S] = v[S] - (v[S].sum() - 1.0) / len(S)
        if (w >= -1e-15).all():
            d = np.sum((w - v) ** 2)
            if d < best_d:
                best, best_d = np.maximum(w, 0.0), d
    return best
