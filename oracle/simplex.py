"""Euclidean projection onto the simplex {w >= 0, 1'w = 1}, the feasible set
of eq. (4).

The paper updates w by steepest descent on a Lagrangian with active-set
multipliers (eq. 5); the projected-gradient form w+ = Proj(w - eta g) uses the
same constraints.  The projection is max(v - tau, 0) with tau chosen so the
result sums to one (Held, Wolfe and Crowder 1974; Duchi et al. 2008); found
here by sorting.

The paper's own rule is also here (active_set_direction, active_set_step):
steepest descent on the Lagrangian of eq. 5 with the active constraints'
multipliers, and a step shortened to stay feasible.
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


def initial_step(w, g) -> float:
    """The fixed step of the projected-gradient weight update, set once from
    the first gradient (the paper leaves the adaptation step unspecified):
    eta = 0.5 max|w| / max|g - mean(g)|, so the first step moves no weight
    by more than half the largest weight before the projection; 0 when g is
    constant (then the projection leaves w unchanged anyway)."""
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    gc = g - g.mean()
    d = np.abs(gc).max()
    return float(0.5 * np.abs(w).max() / d) if d > 0 else 0.0


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


def active_set_direction(w, g):
    """Steepest descent on the Lagrangian of eq. 5: S = P + c_1 (1'w - 1) +
    sum over the active bounds of c_j w_i.  The multipliers make -grad S the
    steepest direction that keeps every active constraint: the projection of
    -g onto {d : sum(d) = 0, d_i >= 0 where w_i = 0}, i.e.
        d_i = nu - g_i            where w_i > 0,
        d_i = max(nu - g_i, 0)    where w_i = 0,
    with nu (= -c_1) the root of sum(d) = 0.  A bound stays active (d_i = 0,
    multiplier c_j = g_i - nu >= 0) where g_i >= nu and is released where
    g_i < nu.  The sum is increasing in nu, with slope at least the number of
    positive weights, so the root is unique; it is found here by walking the
    sorted breakpoints g_i of the zero weights.
    Returns (d, nu)."""
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    free = w > 0
    if not free.any():
        raise ValueError("w has no positive entry (it is not on the simplex)")
    bps = np.sort(g[~free])
    s, c = g[free].sum(), int(free.sum())
    nu = s / c
    for b in bps:            # release breakpoints below the current root
        if b >= nu:
            break
        s += b
        c += 1
        nu = s / c
    d = np.where(free, nu - g, np.maximum(nu - g, 0.0))
    return d, nu


def active_set_step(w, g, mu: float):
    """w_new = w - mu_eff grad S = w + mu_eff d, with mu_eff the largest step
    up to mu that keeps w >= 0 (ratio test over the entries with d_i < 0);
    the entries that reach 0 with it are set to exactly 0 and join the active
    set.  Returns (w_new, d, nu, mu_eff)."""
    w = np.asarray(w, dtype=np.float64)
    d, nu = active_set_direction(w, g)
    neg = d < 0
    mu_eff = float(mu)
    ratios = np.full(w.size, np.inf)
    ratios[neg] = w[neg] / -d[neg]
    if neg.any():
        mu_eff = min(mu_eff, float(ratios.min()))
    w_new = w + mu_eff * d
    w_new[neg & (ratios <= mu_eff)] = 0.0
    return w_new, d, nu, mu_eff
