"""Pins for the oracle's weight derivatives (eq. 4) and the simplex step."""
import numpy as np
import pytest

import synth
from oracle import grad, simplex
from oracle import laplacian as lap
from oracle import solve


def _tiny(seed, N=14, E=9, k=3):
    p = synth.random_small(seed, N, E, 2, 5, k=k)
    return p, lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)


@pytest.mark.parametrize("seed", range(3))
def test_dA_dw_matches_finite_difference_of_eq1(seed):
    p, H = _tiny(seed)
    for e in range(0, p.E, 3):
        fd = np.zeros((p.N, p.N))
        h = 1e-5
        wp, wm = p.w.copy(), p.w.copy()
        wp[e] += h
        wm[e] -= h
        fd = (lap.adjacency(H, wp) - lap.adjacency(H, wm)) / (2 * h)
        assert np.allclose(grad.dA_dw_dense(H, p.w, e), fd, atol=1e-6 * np.abs(fd).max() + 1e-9)


@pytest.mark.parametrize("seed", range(3))
def test_vjp_matches_richardson_fd(seed):
    p, H = _tiny(seed)
    G = synth.rng_for(seed + 50).standard_normal(p.Y.shape)

    def loss(w):
        return float(np.sum(G * solve.solve_dense(lap.system_matrix(H, w, p.lam), p.Y)))
    g, Z, F = grad.solve_vjp(H, p.w, p.lam, p.Y, G)
    fd = np.array([grad.richardson_difference(loss, p.w, e, 1e-4) for e in range(p.E)])
    assert np.linalg.norm(g - fd) / np.linalg.norm(fd) < 1e-8
    # dl/dY = M^-1 G
    M = lap.system_matrix(H, p.w, p.lam)
    assert np.allclose(M @ Z, G, atol=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_objective_grad_matches_richardson_fd(seed):
    p, H = _tiny(seed)
    mu = 0.01
    g = grad.objective_grad(H, p.w, p.lam, mu, p.Y)
    fd = np.array([grad.richardson_difference(lambda w: grad.objective(H, w, p.lam, mu, p.Y),
                                              p.w, e, 1e-4) for e in range(p.E)])
    assert np.linalg.norm(g - fd) / np.linalg.norm(fd) < 1e-8


def test_objective_grad_with_inexact_F_uses_adjoint():
    """With a perturbed F the adjoint term restores the exact total derivative."""
    p, H = _tiny(4)
    mu = 0.01
    M = lap.system_matrix(H, p.w, p.lam)
    F = solve.solve_dense(M, p.Y)
    g_exact = grad.objective_grad(H, p.w, p.lam, mu, p.Y, F)
    g_pert = grad.objective_grad(H, p.w, p.lam, mu, p.Y,
                                 F + 1e-4 * synth.rng_for(1).standard_normal(F.shape))
    # error is second order in the perturbation of F
    assert np.linalg.norm(g_pert - g_exact) / np.linalg.norm(g_exact) < 1e-5


@pytest.mark.parametrize("seed", range(4))
def test_homogeneity(seed):
    """A is degree-0 homogeneous in w: sum_e w_e dJ/dw_e = 2 mu ||w||^2."""
    p, H = _tiny(seed)
    mu = 0.37
    g = grad.objective_grad(H, p.w, p.lam, mu, p.Y)
    assert abs(p.w @ g - 2 * mu * p.w @ p.w) < 1e-12 * max(1.0, np.abs(g).max())
    P = synth.rng_for(seed + 7).standard_normal(p.Y.shape)
    Q = synth.rng_for(seed + 8).standard_normal(p.Y.shape)
    assert abs(p.w @ grad.gamma(H, p.w, P, Q)) < 1e-12 * np.abs(grad.gamma(H, p.w, P, Q)).sum()


def test_sparse_gamma_and_gradient_match_dense():
    p, H = _tiny(6, N=40, E=25, k=4)
    op = lap.SparseOperator(p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam)
    P = synth.rng_for(1).standard_normal(p.Y.shape)
    Q = synth.rng_for(2).standard_normal(p.Y.shape)
    assert np.allclose(grad.gamma_sparse(op, P, Q), grad.gamma(H, p.w, P, Q), atol=1e-13)
    M = lap.system_matrix(H, p.w, p.lam)
    F = solve.solve_dense(M, p.Y) + 1e-3 * synth.rng_for(3).standard_normal(p.Y.shape)
    g_s = grad.objective_grad_sparse(op, p.w, p.lam, 0.05, p.Y, F)
    g_d = grad.objective_grad(H, p.w, p.lam, 0.05, p.Y, F)
    assert np.linalg.norm(g_s - g_d) / np.linalg.norm(g_d) < 1e-10


@pytest.mark.parametrize("seed", range(8))
def test_simplex_projection_bruteforce(seed):
    rng = synth.rng_for(seed)
    n = int(rng.integers(1, 7))
    v = rng.normal(0.2, 0.6, size=n)
    w = simplex.project(v)
    assert np.allclose(w, simplex.project_bruteforce(v), atol=1e-13)
    assert np.all(w >= 0) and abs(w.sum() - 1) < 1e-13


def test_simplex_projection_fixed_point_and_kkt():
    w0 = synth.dirichlet_weights(50, 3)
    assert np.allclose(simplex.project(w0), w0, atol=1e-15)
    v = synth.rng_for(2).normal(0, 0.05, 50) + w0
    w = simplex.project(v)
    sup = w > 0
    tau = (v - w)[sup]
    assert np.allclose(tau, tau[0], atol=1e-14)        # w = v - tau on the support
    assert np.all(v[~sup] <= tau[0] + 1e-14)           # v <= tau off the support


def test_initial_step_rule():
    """The fixed step of the weight update: a hand-worked value, the constant
    gradient (no move), and the invariances it must have. Adding a constant
    to g leaves the projected step unchanged (the projection absorbs it into
    tau), so eta must not change. Scaling g by c scales eta by 1/c, so the
    first step eta * g stays the same."""
    # w = (0.5, 0.3, 0.2), g = (1, 2, 6): mean 3, max|g - 3| = 3, max|w| = 0.5
    assert abs(simplex.initial_step([0.5, 0.3, 0.2], [1.0, 2.0, 6.0]) - 1.0 / 12.0) < 1e-16
    assert simplex.initial_step([0.5, 0.5], [3.0, 3.0]) == 0.0
    w = synth.dirichlet_weights(40, 5)
    g = synth.rng_for(6).normal(0, 1, 40)
    eta = simplex.initial_step(w, g)
    assert abs(simplex.initial_step(w, g + 7.5) - eta) <= 1e-14 * eta
    assert abs(simplex.initial_step(w, 4.0 * g) - eta / 4.0) <= 1e-14 * eta
    # the first step moves no weight by more than half the largest one
    # (before the projection, relative to the mean shift)
    step = eta * (g - g.mean())
    assert np.abs(step).max() <= 0.5 * w.max() * (1 + 1e-14)
