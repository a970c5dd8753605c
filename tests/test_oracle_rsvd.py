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


def _spectrum(m, base, seed):
    """Non-symmetric m x m matrix with singular values base**i (i = 0 .. m-1)."""
    rng = synth.rng_for(seed)
    Q1, _ = np.linalg.qr(rng.standard_normal((m, m)))
    Q2, _ = np.linalg.qr(rng.standard_normal((m, m)))
    sv = base ** np.arange(m)
    return Q1 @ np.diag(sv) @ Q2.T, sv


@pytest.mark.parametrize("q", [0, 1, 3])
def test_power_sketch_is_eq10(q):
    """Eq. (10) literally: (X X')^q X Omega, for a non-symmetric X (X'X in place
    of X X', or a dropped X, fails)."""
    X, _ = _spectrum(40, 0.95, 12)
    Om = synth.rng_for(13).standard_normal((40, 6))
    want = np.linalg.matrix_power(X @ X.T, q) @ X @ Om
    got = rsvd.power_sketch(X, Om, q)
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_power_scheme_exact_rank_recovery(q):
    X = _lowrank(120, 9, 1)
    Om = synth.rng_for(2).standard_normal((120, 14))
    U, s, V = rsvd.randomized_svd_power(X, Om, q)
    k = 9
    approx = U[:, :k] @ np.diag(s[:k]) @ V[:, :k].T
    assert np.linalg.norm(X - approx) / np.linalg.norm(X) < 1e-11
    assert np.allclose(s[:k], np.linalg.svd(X, compute_uv=False)[:k], rtol=1e-11)


def test_power_scheme_matches_algorithm1_on_a_mild_spectrum():
    """Same subspace in exact arithmetic, so with a slowly decaying spectrum the
    two schemes agree to rounding, truncation error included."""
    X, sv = _spectrum(60, 0.9, 11)
    Om = synth.rng_for(14).standard_normal((60, 12))
    U1, s1, _ = rsvd.randomized_svd(X, Om, 2)
    U2, s2, _ = rsvd.randomized_svd_power(X, Om, 2)
    assert np.allclose(s1, s2, rtol=1e-10)
    assert np.allclose(U1[:, :8] @ U1[:, :8].T, U2[:, :8] @ U2[:, :8].T, atol=1e-9)
    # the truncation error itself is far above that: the test compares something
    assert np.abs(s1[:8] - sv[:8]).max() > 1e-4


def test_power_scheme_loses_small_directions():
    """The paper's caveat for eq. (10): without the orthonormalisation between
    products, directions whose singular values fall by more than the working
    precision over 2q+1 products are lost; Algorithm 1 keeps them."""
    X, sv = _spectrum(60, 0.5, 11)
    Om = synth.rng_for(15).standard_normal((60, 12))
    _, s1, _ = rsvd.randomized_svd(X, Om, 4)
    _, s2, _ = rsvd.randomized_svd_power(X, Om, 4)
    assert np.max(np.abs(s1[:8] - sv[:8]) / sv[:8]) < 1e-12
    assert np.max(np.abs(s2[:8] - sv[:8]) / sv[:8]) > 0.1


def test_block_factors_scheme():
    X, _ = _spectrum(30, 0.8, 16)
    A = 0.5 * (X + X.T)
    Om = synth.rng_for(17).standard_normal((30, 8))
    (Up, sp), = rsvd.block_inverse_factors([A], [Om], 6, 2, scheme="power")
    U, s, _ = rsvd.randomized_svd_power(A, Om, 2)
    assert np.array_equal(sp, s[:6]) and np.array_equal(Up, U[:, :6])
    with pytest.raises(ValueError):
        rsvd.block_inverse_factors([A], [Om], 6, 2, scheme="qr-free")


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
