"""Pins for the oracle's Algorithm 1, tessellation and block inverse."""
import numpy as np
import pytest

import synth
from oracle import laplacian as lap
from oracle import rsvd, solve


def _lowrank(m, r, seed):
    rng = synth.rng_for(seed)
    return rng.standard_normal((m, r)) @ rng.standard_normal((r, m))


@pytest.mark.parametrize("q", [0, 1, 2])
def test_exact_rank_recovery(q):
    X = _lowrank(120, 9, 1)
    Om = synth.rng_for(2).standard_normal((120, 14))
    U, s, V = rsvd.randomized_svd(X, Om, q)
    k = 9
    approx = U[:, :k] @ np.diag(s[:k]) @ V[:, :k].T
    assert np.linalg.norm(X - approx) / np.linalg.norm(X) < 1e-12
    assert np.allclose(s[:k], np.linalg.svd(X, compute_uv=False)[:k], rtol=1e-12)


def test_full_width_sketch_is_exact_svd():
    X = synth.rng_for(3).standard_normal((30, 30))
    U, s, V = rsvd.randomized_svd(X, synth.rng_for(4).standard_normal((30, 30)), 1)
    assert np.allclose(s, np.linalg.svd(X, compute_uv=False), rtol=1e-11)
    assert np.allclose(U @ np.diag(s) @ V.T, X, atol=1e-11)


def test_subspace_equals_power_scheme_range():
    """Eq. (10): Algorithm 1's S spans range((X X')^q X Omega) (non-symmetric X)."""
    rng = synth.rng_for(5)
    m, l, q = 60, 8, 2
    Q1, _ = np.linalg.qr(rng.standard_normal((m, m)))
    Q2, _ = np.linalg.qr(rng.standard_normal((m, m)))
    X = Q1 @ np.diag(0.7 ** np.arange(m)) @ Q2.T
    Om = rng.standard_normal((m, l))
    U, s, V = rsvd.randomized_svd(X, Om, q)
    Yp = np.linalg.matrix_power(X @ X.T, q) @ X @ Om
    Sp, _ = np.linalg.qr(Yp)
    # same column space: projectors agree
    assert np.allclose(U @ U.T, Sp @ Sp.T, atol=1e-8)
    # and a different iteration count gives a different subspace
    U1, _, _ = rsvd.randomized_svd(X, Om, q - 1)
    assert not np.allclose(U1 @ U1.T, Sp @ Sp.T, atol=1e-4)


def test_ritz_values_interlace():
    p = synth.random_small(7, 80, 60, 2, 6)
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    A = lap.adjacency(H, p.w)
    true = np.linalg.eigvalsh(A)[::-1]
    U, s, V = rsvd.randomized_svd(A, synth.rng_for(8).standard_normal((80, 12)), 2)
    assert np.all(s <= true[:12] + 1e-12)


def _block_local_hypergraph(sizes, edges_per_block, seed):
    """Edges stay inside contiguous blocks; rank(A_bb) <= edges in the block."""
    rng = synth.rng_for(seed)
    off = synth.block_offsets(np.array(sizes))
    edges = []
    for b, nb in enumerate(sizes):
        for _ in range(edges_per_block):
            sz = int(rng.integers(2, 6))
            edges.append(sorted(rng.choice(nb, size=sz, replace=False) + off[b]))
    ep, ev = synth.explicit_hyperedges(edges)
    return off, ep, ev


def test_block_inverse_exact_when_rank_fits():
    sizes = [40, 55, 30]
    off, ep, ev = _block_local_hypergraph(sizes, 7, 11)
    N, E = off[-1], len(ep) - 1
    H = lap.incidence_dense(N, E, ep, ev)
    w = synth.dirichlet_weights(E, 12)
    lam = 0.8
    A = lap.adjacency(H, w)
    blocks = rsvd.tessellate(A, off)
    oms = [synth.gaussian_sketch(nb, 12, 20 + b)[1] for b, nb in enumerate(sizes)]
    fac = rsvd.block_inverse_factors(blocks, oms, k=10, q=1)
    Y = synth.binary_rhs(N, 3, 0.2, 13)
    F0 = rsvd.block_inverse_apply(fac, off, lam, Y)
    F = solve.solve_dense(lap.system_matrix(H, w, lam), Y)
    assert np.allclose(F0, F, atol=1e-11)


def test_block_inverse_identity_full_eigendecomposition():
    p = synth.random_small(9, 30, 20, 2, 5)
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    A = lap.adjacency(H, p.w)
    off = np.array([0, 12, 30])
    fac = []
    for Ab in rsvd.tessellate(A, off):
        s, U = np.linalg.eigh(Ab)
        fac.append((U, s))
    M = lap.system_matrix(H, p.w, p.lam)
    Mb = rsvd.tessellate(M, off)
    for b, Mbb in enumerate(Mb):
        Zb = rsvd.block_inverse_apply([fac[b]], np.array([0, Mbb.shape[0]]), p.lam,
                                      np.eye(Mbb.shape[0]))
        assert np.allclose(Zb @ Mbb, np.eye(Mbb.shape[0]), atol=1e-12)


def test_pcg_with_block_preconditioner_converges_to_solution():
    p = synth.tessellated(n_blocks=4, lo=40, hi=70, k_rhs=4)
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    A = lap.adjacency(H, p.w)
    M = lap.system_matrix(H, p.w, p.lam)
    blocks = rsvd.tessellate(A, p.blocks)
    oms = [synth.gaussian_sketch(b.shape[0], 16, 30 + i)[1] for i, b in enumerate(blocks)]
    fac = rsvd.block_inverse_factors(blocks, oms, k=12, q=2)
    F, it, rel = rsvd.preconditioned_cg(lambda P: M @ P,
                                        lambda R: rsvd.block_inverse_apply(fac, p.blocks, p.lam, R),
                                        p.Y, 1e-12, 200)
    Fd = solve.solve_dense(M, p.Y)
    assert np.all(rel <= 1e-12)
    assert np.allclose(F, Fd, atol=1e-10)
    # the preconditioner must not slow CG down on this block-dominated operator
    _, it_plain, _ = solve.cg_ranking(H, p.w, p.lam, p.Y, tol=1e-12)
    assert it.max() <= it_plain.max()
