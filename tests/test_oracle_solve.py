"""Pins for the oracle's solve (eqs. 3, 6) and CG (eqs. 16-20)."""
import numpy as np
import pytest

import synth
from oracle import laplacian as lap
from oracle import solve


def _tiny(seed, N=16, E=10, smin=1, smax=5, k=3):
    p = synth.random_small(seed, N, E, smin, smax, k=k)
    return p, lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)


def test_single_edge_closed_form():
    N, lam = 11, 0.6
    ep, ev = synth.explicit_hyperedges([list(range(N))])
    H = lap.incidence_dense(N, 1, ep, ev)
    Y = synth.rng_for(2).standard_normal((N, 3))
    PY = np.ones((N, N)) / N @ Y
    F = solve.solve_dense(lap.system_matrix(H, [1.0], lam), Y)
    assert np.allclose(F, PY + lam / (1 + lam) * (Y - PY), atol=1e-14)


def test_isolated_vertex_and_optimality():
    p, H = _tiny(3, N=20, E=6, smin=2, smax=3)
    M = lap.system_matrix(H, p.w, p.lam)
    F = solve.solve_dense(M, p.Y)
    iso = H.sum(axis=1) == 0
    assert iso.any()
    assert np.allclose(F[iso], p.lam / (1 + p.lam) * p.Y[iso], atol=1e-15)
    # F minimises tr(F'LF) + lambda ||F - Y||^2: gradient L F + lambda (F - Y) = 0
    L = lap.laplacian(H, p.w)
    assert np.linalg.norm(L @ F + p.lam * (F - p.Y)) < 1e-13


def test_woodbury_edge_space_route():
    """Second route: M^-1 = lam/(1+lam)[I + K((1+lam)I - K'K)^-1 K'],
    K = Dv^-1/2 H W^1/2 De^-1/2 (an E x E solve instead of N x N)."""
    p, H = _tiny(5, N=25, E=8)
    w = p.w
    s = lap.inv_sqrt_degrees(lap.vertex_degrees(H, w))
    K = s[:, None] * H * np.sqrt(w / lap.edge_degrees(H))[None, :]
    lam = p.lam
    inner = np.linalg.solve((1 + lam) * np.eye(p.E) - K.T @ K, K.T @ p.Y)
    F2 = lam / (1 + lam) * (p.Y + K @ inner)
    F = solve.solve_dense(lap.system_matrix(H, w, lam), p.Y)
    assert np.allclose(F, F2, atol=1e-13)


def test_eq3_form_equals_system_solve():
    p, H = _tiny(6)
    X = lap.ranking_matrix(H, p.w, p.lam)
    f = solve.ranking_solution(X, p.Y, p.lam)
    F = solve.solve_dense(lap.system_matrix(H, p.w, p.lam), p.Y)
    assert np.allclose(f, F, atol=1e-14)


def test_disjoint_union_is_block_diagonal():
    a = synth.random_small(1, 10, 6, 1, 4, k=2)
    b = synth.random_small(2, 8, 5, 1, 4, k=2)
    Ha = lap.incidence_dense(a.N, a.E, a.edge_ptr, a.edge_vtx)
    Hb = lap.incidence_dense(b.N, b.E, b.edge_ptr, b.edge_vtx)
    H = np.zeros((a.N + b.N, a.E + b.E))
    H[:a.N, :a.E] = Ha
    H[a.N:, a.E:] = Hb
    w = np.concatenate([a.w, 3.0 * b.w])
    Y = np.vstack([a.Y, b.Y])
    F = solve.solve_dense(lap.system_matrix(H, w, 0.9), Y)
    Fa = solve.solve_dense(lap.system_matrix(Ha, a.w, 0.9), a.Y)
    Fb = solve.solve_dense(lap.system_matrix(Hb, b.w, 0.9), b.Y)
    assert np.allclose(F, np.vstack([Fa, Fb]), atol=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_cg_terminates_in_at_most_n_steps(seed):
    p, H = _tiny(seed, N=24, E=14, k=4)
    f, it, rel = solve.cg_ranking(H, p.w, p.lam, p.Y, tol=1e-12, max_iter=p.N)
    assert np.all(it <= p.N) and np.all(rel <= 1e-12)
    F = solve.solve_dense(lap.system_matrix(H, p.w, p.lam), p.Y)
    assert np.allclose(f, F, atol=1e-10)


def test_cg_two_distinct_eigenvalues_two_steps():
    N = 13
    ep, ev = synth.explicit_hyperedges([list(range(N))])
    H = lap.incidence_dense(N, 1, ep, ev)
    Y = synth.rng_for(4).standard_normal((N, 2))
    f, it, rel = solve.cg_ranking(H, [1.0], 0.8, Y, tol=1e-13, max_iter=10)
    assert np.all(it <= 2) and np.all(rel <= 1e-13)


def test_cg_zero_column():
    p, H = _tiny(2, k=3)
    Y = p.Y.copy()
    Y[:, 1] = 0
    f, it, rel = solve.cg_ranking(H, p.w, p.lam, Y, tol=1e-12, max_iter=100)
    assert np.all(f[:, 1] == 0) and it[1] == 0


def test_cg_iteration_bound_small_plain():
    """kappa(M) <= 1 + 1/lambda; CG error bound 2((sqrt k - 1)/(sqrt k + 1))^i."""
    p = synth.small_plain(N=600, E=450, k=5)
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    f, it, rel = solve.cg_ranking(H, p.w, p.lam, p.Y, tol=1e-10, max_iter=200)
    kappa = 1 + 1 / p.lam
    rho = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    # residual bound: ||r_i|| <= sqrt(kappa) * 2 rho^i ||r_0||
    bound = int(np.ceil(np.log(1e-10 / (2 * np.sqrt(kappa))) / np.log(rho)))
    assert np.all(it <= bound)
    F = solve.solve_dense(lap.system_matrix(H, p.w, p.lam), p.Y)
    err = np.linalg.norm(f - F) / np.linalg.norm(F)
    assert err <= 2e-10


def test_sparse_cg_matches_dense():
    p = synth.random_small(8, 60, 45, 2, 8, k=3)
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    op = lap.SparseOperator(p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam)
    f, it, rel = solve.cg_ranking(op, p.w, p.lam, p.Y, tol=1e-13)
    F = solve.solve_dense(lap.system_matrix(H, p.w, p.lam), p.Y)
    assert np.allclose(f, F, atol=1e-11)
    assert np.all(solve.relres(op, f, p.Y) <= 1e-12)
