"""Pins of the active-set steepest descent of eq. 5 (oracle.simplex.
active_set_direction / active_set_step): hand-worked steps, brute force over
the released bounds with the KKT conditions checked, the known minimiser of
a quadratic over the simplex as a fixed point, convergence to it, and the
invariants (sum kept, feasibility, active entries untouched)."""
import itertools

import numpy as np
import pytest

import synth
from oracle import simplex


def test_hand_worked_steps():
    # w3 = 0 with g3 above nu = (1 + 0)/2 stays active; d = -(g - nu) on the rest
    w, d, nu, mu = simplex.active_set_step([0.5, 0.5, 0.0], [1.0, 0.0, 2.0], 0.4)
    assert nu == 0.5 and mu == 0.4
    assert np.allclose(d, [-0.5, 0.5, 0.0], atol=0) and np.allclose(w, [0.3, 0.7, 0.0], atol=1e-16)
    # the ratio test stops the step where w1 reaches 0 (mu_eff = 0.5 / 0.5)
    w, d, nu, mu = simplex.active_set_step([0.5, 0.5, 0.0], [1.0, 0.0, 2.0], 2.0)
    assert mu == 1.0 and w.tolist() == [0.0, 1.0, 0.0]
    # w2 = w3 = 0: g3 = -1 lies below nu and is released, g2 = 1 stays;
    # nu = (0 - 1)/2
    w, d, nu, mu = simplex.active_set_step([1.0, 0.0, 0.0], [0.0, 1.0, -1.0], 1.0)
    assert nu == -0.5 and d.tolist() == [-0.5, 0.0, 0.5] and w.tolist() == [0.5, 0.0, 0.5]


def _kkt_bruteforce(w, g):
    """Every subset R of the zero weights as the released set: nu = mean of g
    over the positive weights and R; keep the R whose nu is consistent
    (g_i < nu on R, g_i >= nu on the other zero weights)."""
    free = w > 0
    zeros = np.nonzero(~free)[0]
    found = []
    for r in range(len(zeros) + 1):
        for R in itertools.combinations(zeros, r):
            m = free.copy()
            m[list(R)] = True
            nu = g[m].mean()
            if all(g[i] < nu for i in R) and all(g[i] >= nu for i in zeros if i not in R):
                d = np.where(m, nu - g, 0.0)
                found.append((d, nu))
    return found


@pytest.mark.parametrize("seed", range(8))
def test_direction_against_bruteforce(seed):
    rng = synth.rng_for(400 + seed)
    E = 7
    w = rng.dirichlet(np.ones(E))
    w[rng.random(E) < 0.5] = 0.0
    if not (w > 0).any():
        w[0] = 1.0
    w /= w.sum()
    g = rng.standard_normal(E)
    d, nu = simplex.active_set_direction(w, g)
    sols = _kkt_bruteforce(w, g)
    assert len(sols) == 1      # the released set is unique
    assert np.allclose(d, sols[0][0], atol=1e-14) and abs(nu - sols[0][1]) < 1e-14
    # d is the projection of -g onto the tangent cone: sum zero, d >= 0 on
    # the zero weights, and -g - d is orthogonal to d
    assert abs(d.sum()) < 1e-14 and (d[w == 0] >= 0).all()
    assert abs(np.dot(-g - d, d)) < 1e-13


def test_minimiser_is_a_fixed_point():
    # P(w) = 1/2 ||w - v||^2 has its minimum over the simplex at project(v)
    # (pinned separately by brute force); the gradient there is w* - v
    v = synth.rng_for(410).standard_normal(40) * 0.3
    ws = simplex.project(v)
    assert (ws == 0).any() and (ws > 0).any()
    d, _ = simplex.active_set_direction(ws, ws - v)
    assert np.abs(d).max() < 1e-15


def test_descent_reaches_the_minimiser():
    """With mu = 1 each step on P(w) = 1/2 ||w - v||^2 either lands on the
    minimiser of the current face or makes one more weight zero, so the
    minimiser is reached within E steps."""
    E = 30
    v = synth.rng_for(411).standard_normal(E) * 0.2
    w = np.full(E, 1.0 / E)
    for _ in range(E + 1):
        w, d, nu, mu = simplex.active_set_step(w, w - v, 1.0)
        assert (w >= 0).all() and abs(w.sum() - 1.0) < 1e-13
    assert np.allclose(w, simplex.project(v), atol=1e-12)


def test_step_invariants():
    rng = synth.rng_for(412)
    E = 500
    w = rng.dirichlet(np.ones(E) * 0.3)
    w[w < 1e-3] = 0.0
    w /= w.sum()
    g = rng.standard_normal(E)
    w2, d, nu, mu = simplex.active_set_step(w, g, 10.0)
    assert (w2 >= 0).all() and abs(w2.sum() - 1.0) < 1e-12
    stay = (w == 0) & (g >= nu)
    assert (w2[stay] == 0).all() and (d[stay] == 0).all()
    assert mu < 10.0 and (w2[(w > 0) & (d < 0)] == 0).sum() >= 1   # the ratio test bound
    with pytest.raises(ValueError):
        simplex.active_set_direction(np.zeros(4), np.ones(4))
