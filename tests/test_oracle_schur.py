"""Pins of the Schur-complement block inverse oracle (eqs. 12-15): closed-form
inverses of 2x2 and 3x3 matrices, X X^-1 = I, the nested tessellation's
coverage and sizes, exactness of the block-diagonal inverse when the
hyperedges stay inside blocks, and the sparse extraction of M_bb."""
import numpy as np
import pytest

import synth
from oracle import laplacian as lap
from oracle import rsvd, schur, solve


def test_two_by_two_closed_form():
    # nonsymmetric, so that a swapped X12 / X21 or Z1 / Z2 changes the result
    a, b, c, d = 3.0, -1.25, 0.5, 2.0
    X = np.array([[a, b], [c, d]])
    det = a * d - b * c
    want = np.array([[d, -b], [-c, a]]) / det
    assert np.allclose(schur.schur_inverse(X, 1), want, rtol=0, atol=1e-15)


def test_three_by_three_adjugate():
    rng = synth.rng_for(71)
    X = rng.standard_normal((3, 3)) + 4 * np.eye(3)
    # the inverse is the transposed cofactor matrix over the determinant
    cof = np.empty((3, 3))
    for i in range(3):
        for j in range(3):
            m = np.delete(np.delete(X, i, 0), j, 1)
            cof[i, j] = (-1) ** (i + j) * (m[0, 0] * m[1, 1] - m[0, 1] * m[1, 0])
    det = sum(X[0, j] * cof[0, j] for j in range(3))
    assert np.allclose(schur.schur_inverse(X, 1), cof.T / det, rtol=0, atol=1e-14)


@pytest.mark.parametrize("n,min_block", [(7, 1), (7, 2), (7, 3), (7, 4), (64, 5), (101, 12)])
def test_inverse_identity_nonsymmetric(n, min_block):
    rng = synth.rng_for(72 + n + min_block)
    X = rng.standard_normal((n, n)) / np.sqrt(n) + 2 * np.eye(n)
    Xi = schur.schur_inverse(X, min_block)
    assert np.abs(X @ Xi - np.eye(n)).max() < 1e-12
    assert np.abs(Xi @ X - np.eye(n)).max() < 1e-12


def test_leaf_is_eq15():
    rng = synth.rng_for(73)
    X = rng.standard_normal((9, 9)) + 3 * np.eye(9)
    # not split (9 < 2 * 5): the inverse from the SVD, eq. 15
    Xi = schur.schur_inverse(X, 5)
    assert np.abs(X @ Xi - np.eye(9)).max() < 1e-13
    # an orthogonal matrix: V Sigma^-1 U' with Sigma = I is the transpose
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    assert np.allclose(schur.svd_inverse(Q), Q.T, atol=1e-14)


@pytest.mark.parametrize("n,min_block", [(1500, 50), (500, 50), (99, 50), (100, 50), (1, 1), (37, 4), (4096, 64)])
def test_nested_tessellation_covers_in_order(n, min_block):
    leaves = schur.nested_tessellation(n, min_block)
    off = 0
    for o, m in leaves:
        assert o == off
        off += m
        if n >= min_block:
            assert min_block <= m < 2 * min_block
        else:
            assert m == n
    assert off == n
    if n == 1500 and min_block == 50:
        # 1500 -> 750 -> 375 -> 187, 188 -> 93, 94: sixteen leaves
        assert len(leaves) == 16 and {m for _, m in leaves} == {93, 94}


def test_spd_blocks_give_symmetric_inverse():
    p = synth.random_small(9, 120, 90, 2, 7)
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    M = lap.system_matrix(H, p.w, 0.5)
    Mi = schur.schur_inverse(M, 10)
    assert np.abs(Mi - Mi.T).max() < 1e-13
    assert np.abs(M @ Mi - np.eye(p.N)).max() < 1e-12
    # eigenvalues of M lie in [1, 1 + 1/lambda], so those of M^-1 in [1/3, 1]
    ev = np.linalg.eigvalsh(0.5 * (Mi + Mi.T))
    assert ev.min() > 1 / 3 - 1e-12 and ev.max() < 1 + 1e-12


def test_system_block_matches_dense():
    p = synth.tessellated(n_blocks=3, lo=40, hi=70, k_rhs=2)
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    Hs = lap.incidence_sparse(p.N, p.E, p.edge_ptr, p.edge_vtx)
    M = lap.system_matrix(H, p.w, 0.7)
    for b, Mb in enumerate(rsvd.tessellate(M, p.blocks)):
        got = schur.system_block(Hs, p.w, 0.7, p.blocks[b], p.blocks[b + 1])
        assert np.allclose(got, Mb, atol=1e-14)


def _block_local(sizes, edges_per_block, seed):
    rng = synth.rng_for(seed)
    off = synth.block_offsets(np.array(sizes))
    edges = []
    for b, nb in enumerate(sizes):
        for _ in range(edges_per_block):
            sz = int(rng.integers(2, 9))
            edges.append(sorted(rng.choice(nb, size=sz, replace=False) + off[b]))
    ep, ev = synth.explicit_hyperedges(edges)
    return off, ep, ev


def test_block_inverse_exact_for_block_local_hyperedges():
    sizes = [120, 75, 101]
    off, ep, ev = _block_local(sizes, 60, 74)
    N, E = int(off[-1]), len(ep) - 1
    H = lap.incidence_dense(N, E, ep, ev)
    w = synth.dirichlet_weights(E, 75)
    lam = 0.6
    M = lap.system_matrix(H, w, lam)
    inv = schur.block_schur_inverses(rsvd.tessellate(M, off), 20)
    Y = synth.binary_rhs(N, 4, 0.1, 76)
    F0 = schur.block_dense_apply(inv, off, Y)
    assert np.allclose(F0, solve.solve_dense(M, Y), atol=1e-12)


def test_pcg_with_schur_preconditioner():
    p = synth.tessellated(n_blocks=4, lo=60, hi=110, k_rhs=4)
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    M = lap.system_matrix(H, p.w, p.lam)
    inv = schur.block_schur_inverses(rsvd.tessellate(M, p.blocks), 16)
    F, it, rel = rsvd.preconditioned_cg(lambda P: M @ P, lambda R: schur.block_dense_apply(inv, p.blocks, R),
                                        p.Y, 1e-12, 200)
    assert np.all(rel <= 1e-12)
    assert np.allclose(F, solve.solve_dense(M, p.Y), atol=1e-10)
    _, it_plain, _ = solve.cg_ranking(H, p.w, p.lam, p.Y, tol=1e-12)
    assert it.max() <= it_plain.max()
