"""GPU parity: structure build, degrees/scales and the operator apply against
the FP64 oracle (section 2, eq. 1)."""
import numpy as np
import pytest

import synth
from oracle import laplacian as lap
from tests.helpers import build, colrelerr, device, hgl, relerr, say

pytestmark = pytest.mark.gpu


def _problems():
    yield "tiny_isolated", synth.random_small(3, 40, 12, 1, 4, k=5)
    yield "g1_small", synth.small_plain(N=700, E=500, k=7)
    # hubs: vertex rows longer than the split threshold exercise the chunked path
    yield "g2_hubs", synth.multi_rhs(N=3000, E=2500, k=9, smax=120)
    ep, ev = synth.explicit_hyperedges([list(range(150))])
    yield "single_edge", synth.Problem(150, 1, ep, ev, np.array([0.37]), 0.6,
                                       synth.rng_for(1).standard_normal((150, 4)))


@pytest.mark.parametrize("name,p", list(_problems()), ids=lambda x: x if isinstance(x, str) else "")
def test_structure_and_scales(name, p):
    dev = device()
    say("structure", name)
    h = build(p, dev)
    op = hgl().get_operator(h)
    H = lap.incidence_sparse(p.N, p.E, p.edge_ptr, p.edge_vtx)
    dv = lap.vertex_degrees(H, p.w)
    assert np.allclose(op["dv"].cpu().numpy(), dv, rtol=1e-14, atol=0)
    assert np.allclose(op["s"].cpu().numpy(), lap.inv_sqrt_degrees(dv), rtol=1e-14, atol=0)
    assert np.allclose(op["c"].cpu().numpy(), p.w / lap.edge_degrees(H), rtol=1e-15, atol=0)
    # vertex-major CSR: exactly the columns of H', each in increasing edge id
    csc = H.tocsc() if False else H.tocsr()
    vp = op["vtx_ptr"].cpu().numpy()
    ve = op["vtx_edge"].cpu().numpy()
    assert np.array_equal(vp, csc.indptr.astype(np.int32))
    for v in range(p.N):
        assert np.array_equal(ve[vp[v]:vp[v + 1]], np.sort(csc.indices[csc.indptr[v]:csc.indptr[v + 1]]))


@pytest.mark.parametrize("k", [1, 3, 50, 64, 200, 300])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_apply_matches_dense(k, dtype):
    import torch
    dev = device()
    p = synth.multi_rhs(N=2500, E=2000, k=1, smax=100)
    say("apply", k, dtype)
    h = build(p, dev)
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    M = lap.system_matrix(H, p.w, p.lam)
    P = synth.rng_for(k).standard_normal((p.N, k))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    Pd = torch.from_numpy(P).to(dev, tdt)
    Q = hgl().apply(h, p.lam, Pd).cpu().numpy()
    ref = M @ Pd.cpu().double().numpy()
    tol = 1e-13 if dtype == "f64" else 2e-6
    assert colrelerr(Q, ref).max() < tol


def test_apply_strided_views_and_ragged_k():
    import torch
    dev = device()
    p = synth.multi_rhs(N=1800, E=1500, k=1, smax=80)
    h = build(p, dev)
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    M = lap.system_matrix(H, p.w, p.lam)
    big = torch.from_numpy(synth.rng_for(2).standard_normal((p.N, 77))).to(dev, torch.float32)
    P = big[:, 3:40]          # ld = 77, k = 37, misaligned start
    out = torch.zeros((p.N, 45), dtype=torch.float32, device=dev)
    hgl().apply(h, 2.0, P, out=out[:, 5:42])
    ref = lap.system_matrix(H, p.w, 2.0) @ P.cpu().double().numpy()
    assert colrelerr(out[:, 5:42].cpu().numpy(), ref).max() < 2e-6
    assert float(out[:, :5].abs().max()) == 0.0 and float(out[:, 42:].abs().max()) == 0.0
    del M


def test_batched_apply_is_block_diagonal():
    import torch
    dev = device()
    p = synth.batch_of_graphs(G=4, nlo=300, nhi=900, k=6)
    h = build(p, dev)
    P = torch.from_numpy(synth.rng_for(5).standard_normal((p.N, 6))).to(dev)
    Q = hgl().apply(h, 0.5, P).cpu().numpy()
    for g in range(4):
        v0, v1 = p.vtx_offsets[g], p.vtx_offsets[g + 1]
        e0, e1 = p.edge_offsets[g], p.edge_offsets[g + 1]
        ep = p.edge_ptr[e0:e1 + 1] - p.edge_ptr[e0]
        ev = p.edge_vtx[p.edge_ptr[e0]:p.edge_ptr[e1]] - v0
        Hg = lap.incidence_dense(v1 - v0, e1 - e0, ep, ev)
        ref = lap.system_matrix(Hg, p.w[e0:e1], 0.5) @ P[v0:v1].cpu().numpy()
        assert relerr(Q[v0:v1], ref) < 1e-13


@pytest.mark.parametrize("bad", ["dup", "range", "empty", "negw", "nanw", "ptr"])
def test_invalid_structure_rejected(bad):
    import torch
    dev = device()
    h = hgl()
    edges = [[0, 1, 2], [2, 3], [1, 4]]
    w = np.array([0.2, 0.3, 0.5])
    N = 5
    if bad == "dup":
        edges[1] = [3, 3]
    if bad == "range":
        edges[2] = [1, 5]
    ep, ev = synth.explicit_hyperedges(edges)
    if bad == "empty":
        ep = np.array([0, 3, 3, 5], np.int32)
        ev = np.array([0, 1, 2, 1, 4], np.int32)
    if bad == "negw":
        w[1] = -0.1
    if bad == "nanw":
        w[2] = np.nan
    if bad == "ptr":
        ep = ep.copy()
        ep[1] = 9
    t = lambda a, d: torch.from_numpy(np.ascontiguousarray(a)).to(dev, d)  # noqa: E731
    say("invalid", bad)
    with pytest.raises(Exception) as ei:
        h.build_laplacian(t(ep, torch.int32), t(ev, torch.int32), t(w, torch.float64), N)
    assert "HGL_EINVAL" in str(ei.value)


def test_set_weights_recomputes_scales():
    import torch
    dev = device()
    p = synth.small_plain(N=400, E=300, k=3)
    h = build(p, dev)
    w2 = synth.dirichlet_weights(p.E, 77)
    hgl().set_weights(h, torch.from_numpy(w2).to(dev))
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    P = torch.from_numpy(synth.rng_for(3).standard_normal((p.N, 4))).to(dev)
    Q = hgl().apply(h, 0.8, P).cpu().numpy()
    assert relerr(Q, lap.system_matrix(H, w2, 0.8) @ P.cpu().numpy()) < 1e-13
    with pytest.raises(Exception):
        w3 = w2.copy()
        w3[0] = -1
        hgl().set_weights(h, torch.from_numpy(w3).to(dev))
