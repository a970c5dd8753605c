"""Pins for the oracle's hypergraph operators (section 2, eq. 1).

Each test checks the oracle against something other than its own formula: a
hand-derived example, a library routine the operator reduces to, a closed
form, spectral facts, or the per-edge expansion of eq. (1)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.csgraph as csgraph

import synth
from oracle import laplacian as lap

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tiny(seed, N=12, E=9, smin=1, smax=5):
    p = synth.random_small(seed, N, E, smin, smax)
    return p, lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)


def test_golden_hand_derived_example():
    g = json.load(open(os.path.join(GOLDEN, "tiny_hypergraph.json")))
    ep, ev = synth.explicit_hyperedges(g["hypergraph"]["edges"])
    H = lap.incidence_dense(3, 2, ep, ev)
    w = np.array(g["hypergraph"]["w"])
    assert np.allclose(lap.vertex_degrees(H, w), g["dv"], rtol=0, atol=1e-15)
    assert np.allclose(lap.edge_degrees(H), g["de"], rtol=0, atol=1e-15)
    assert np.allclose(lap.adjacency(H, w), np.array(g["A"]), rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", range(6))
def test_spectrum_symmetry_and_null_vector(seed):
    p, H = _tiny(seed)
    L = lap.laplacian(H, p.w)
    assert np.allclose(L, L.T, atol=1e-14)
    ev = np.linalg.eigvalsh(L)
    # A is PSD and similar to a row-stochastic matrix: eig(L) in [0, 1]
    assert ev.min() > -1e-12 and ev.max() < 1 + 1e-12
    dv = lap.vertex_degrees(H, p.w)
    assert np.allclose(L @ np.sqrt(dv), 0.0, atol=1e-13)


def _components_with_edges(N, ep, ev):
    parent = list(range(N))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a
    touched = np.zeros(N, bool)
    for e in range(len(ep) - 1):
        m = ev[ep[e]:ep[e + 1]]
        touched[m] = True
        for v in m[1:]:
            parent[find(int(v))] = find(int(m[0]))
    return len({find(v) for v in range(N) if touched[v]})


@pytest.mark.parametrize("seed", range(6))
def test_zero_eigenvalue_multiplicity_counts_components(seed):
    p, H = _tiny(seed, N=14, E=6, smin=1, smax=3)
    ev = np.linalg.eigvalsh(lap.laplacian(H, p.w))
    assert np.sum(np.abs(ev) < 1e-10) == _components_with_edges(p.N, p.edge_ptr, p.edge_vtx)
    # isolated vertices: L_vv = 1 (pseudo-inverse reading for delta(v) = 0)
    iso = H.sum(axis=1) == 0
    L = lap.laplacian(H, p.w)
    assert np.allclose(np.diag(L)[iso], 1.0)


def test_scale_invariance():
    p, H = _tiny(3)
    assert np.allclose(lap.laplacian(H, p.w), lap.laplacian(H, 7.5 * p.w), atol=1e-14)


def test_two_uniform_is_half_normalised_graph_laplacian():
    rng = synth.rng_for(5)
    N = 10
    pairs = [(i, (i + 1) % N) for i in range(N)] + [(0, 5), (2, 7), (3, 8)]
    ep, ev = synth.explicit_hyperedges([list(pq) for pq in pairs])
    w = rng.uniform(0.2, 2.0, size=len(pairs))
    H = lap.incidence_dense(N, len(pairs), ep, ev)
    Wg = np.zeros((N, N))
    for (a, b), we in zip(pairs, w):
        Wg[a, b] += we
        Wg[b, a] += we
    ref = csgraph.laplacian(Wg, normed=True)
    assert np.allclose(lap.laplacian(H, w), 0.5 * ref, atol=1e-14)


def test_single_edge_over_all_vertices():
    N = 9
    ep, ev = synth.explicit_hyperedges([list(range(N))])
    H = lap.incidence_dense(N, 1, ep, ev)
    assert np.allclose(lap.laplacian(H, [0.3]), np.eye(N) - np.ones((N, N)) / N, atol=1e-15)


@pytest.mark.parametrize("seed", range(4))
def test_per_edge_expansion(seed):
    """A = sum_e (w_e/delta_e) (S h_e)(S h_e)' written out edge by edge."""
    p, H = _tiny(seed)
    N = p.N
    dv = np.zeros(N)
    for e in range(p.E):
        for j in range(p.edge_ptr[e], p.edge_ptr[e + 1]):
            dv[p.edge_vtx[j]] += p.w[e]
    A = np.zeros((N, N))
    for e in range(p.E):
        mem = p.edge_vtx[p.edge_ptr[e]:p.edge_ptr[e + 1]]
        for u in mem:
            for v in mem:
                A[u, v] += p.w[e] / len(mem) / np.sqrt(dv[u] * dv[v])
    assert np.allclose(lap.adjacency(H, p.w), A, atol=1e-15)


def test_sparse_operator_matches_dense():
    p, H = _tiny(2, N=40, E=30, smax=8)
    op = lap.SparseOperator(p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam)
    P = synth.rng_for(1).standard_normal((p.N, 4))
    M = lap.system_matrix(H, p.w, p.lam)
    assert np.allclose(op(P), M @ P, atol=1e-13)


def test_ranking_matrix_relation():
    p, H = _tiny(4)
    theta = p.lam
    X = lap.ranking_matrix(H, p.w, theta)
    M = lap.system_matrix(H, p.w, theta)
    assert np.allclose(M, (1 + 1 / theta) * X, atol=1e-14)
