"""The seeded generators produce what their recipes state."""
import numpy as np
import pytest

import synth


def _check_sets(ep, ev, N):
    assert ep[0] == 0 and np.all(np.diff(ep) >= 1)
    assert ev.min() >= 0 and ev.max() < N
    for e in range(len(ep) - 1):
        m = ev[ep[e]:ep[e + 1]]
        assert np.all(np.diff(m) > 0), "hyperedge must be a strictly increasing vertex set"


def test_uniform_sizes_and_sets():
    ep, ev = synth.uniform_hyperedges(500, 400, 2, 20, 7)
    sizes = np.diff(ep)
    assert sizes.min() >= 2 and sizes.max() <= 20
    _check_sets(ep, ev, 500)


def test_powerlaw_sizes_hubs_and_sets():
    ep, ev = synth.powerlaw_hyperedges(5000, 4000, 2.1, 2, 200, 1.1, 11)
    sizes = np.diff(ep)
    assert sizes.min() >= 2 and sizes.max() <= 200
    # truncated (not clamped) power law: mean size near 6.6 for [2,200]
    assert 5.0 < sizes.mean() < 8.5
    _check_sets(ep, ev, 5000)
    deg = np.bincount(ev, minlength=5000)
    assert deg.max() > 20 * max(deg.mean(), 1)      # hub vertices exist
    assert (deg == 0).mean() > 0.2                  # many isolated vertices


def test_binary_rhs_exact_density():
    Y = synth.binary_rhs(1000, 37, 0.05, 3)
    assert set(np.unique(Y)) <= {0.0, 1.0}
    assert int(Y.sum()) == round(0.05 * 1000 * 37)


def test_seeds_reproduce():
    a = synth.powerlaw_hyperedges(300, 200, 2.1, 2, 50, 1.1, 5)
    b = synth.powerlaw_hyperedges(300, 200, 2.1, 2, 50, 1.1, 5)
    c = synth.powerlaw_hyperedges(300, 200, 2.1, 2, 50, 1.1, 6)
    assert np.array_equal(a[1], b[1]) and not np.array_equal(a[1], c[1])


def test_bf16_round_is_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 2 ** -8, -3.14159, 0.0])
    bits, vals = synth.bf16_round(x)
    assert vals[0] == 1.0
    assert vals[1] == 1.0                   # tie -> even mantissa
    assert vals[2] == 1.0 + 2 ** -6         # tie -> even (rounds up)
    assert abs(vals[3] - x[3]) <= 2 ** -8 * 4
    assert bits[4] == 0


def test_dirichlet_on_simplex():
    w = synth.dirichlet_weights(1000, 9)
    assert np.all(w > 0) and abs(w.sum() - 1) < 1e-12


@pytest.mark.slow
def test_multi_rhs_recipe_shape():
    p = synth.multi_rhs(N=50_000, E=40_000, k=4)
    deg = np.bincount(p.edge_vtx, minlength=p.N)
    assert 2.0e5 < p.nnz < 3.3e5
    assert 0.35 < (deg == 0).mean() < 0.55
    assert deg.max() > 5000


def test_batch_offsets_consistent():
    p = synth.batch_of_graphs(G=3, nlo=200, nhi=400, k=5)
    assert p.vtx_offsets[-1] == p.N and p.edge_offsets[-1] == p.E
    for g in range(3):
        e0, e1 = p.edge_offsets[g], p.edge_offsets[g + 1]
        m = p.edge_vtx[p.edge_ptr[e0]:p.edge_ptr[e1]]
        assert m.min() >= p.vtx_offsets[g] and m.max() < p.vtx_offsets[g + 1]
