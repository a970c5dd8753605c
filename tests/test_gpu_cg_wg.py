"""GPU parity: the one-workgroup CG (hgl_cg_solve_wg, each column's whole
FP32 solve in one workgroup of one launch) against the FP64 oracle, and its
edge cases."""
import ctypes as C

import numpy as np
import pytest

import synth
from oracle import laplacian as lap
from oracle import solve
from tests.helpers import build, colrelerr, device, hgl, say

pytestmark = pytest.mark.gpu


def _dense_solution(p, Y):
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    return solve.solve_dense(lap.system_matrix(H, p.w, p.lam), Y)


def _g2(N, E, k, seed, lam=0.5):
    ep, ev = synth.powerlaw_hyperedges(N, E, 2.1, 2, 200, 1.1, seed)
    return synth.Problem(N, E, ep, ev, synth.dirichlet_weights(E, seed + 1), lam,
                         synth.binary_rhs(N, k, 0.05, seed + 2))


# (lambda, relres target, forward-error bar): the bar is kappa(M) * tol with
# kappa <= 1 + 1/lambda; at lambda = 0.05 a target of 1e-6/(1 + 1/lambda)
# would lie below FP32's attainable residual, so it is 5e-7 there
@pytest.mark.parametrize("lam,tol,bar", [(0.5, 1e-6 / 3, 1e-6), (0.05, 5e-7, 21 * 5e-7)])
def test_matches_cholesky_with_hubs_and_long_hyperedges(lam, tol, bar):
    """N = 2000 G2 graph: 48 rows above 32 hyperedges (degree up to 800) and
    44 hyperedges above 32 members (the one-wave paths), 546 isolated
    vertices; k = 37 columns, one of them zero."""
    import torch
    dev = device()
    p = _g2(2000, 1600, 37, 77, lam)
    Y = p.Y.copy()
    Y[:, 5] = 0.0
    say("cg_wg vs cholesky lam", lam)
    h = build(p, dev)
    F, it, rel, st = hgl().cg_solve_wg(h, lam, torch.from_numpy(Y).to(dev, torch.float32), tol=tol)
    assert st == 0 and np.all(rel <= tol)
    assert it[0, 5] == 0 and rel[0, 5] == 0.0
    F = F.cpu().double().numpy()
    assert np.all(F[:, 5] == 0.0)
    Fo = _dense_solution(p, Y)
    nz = [j for j in range(Y.shape[1]) if j != 5]
    assert colrelerr(F[:, nz], Fo[:, nz]).max() <= bar
    # the iteration count of unpreconditioned CG on the same system
    _, it_mk, _, _ = hgl().cg_solve(h, lam, torch.from_numpy(Y).to(dev, torch.float32), tol=tol)
    assert abs(int(it.max()) - int(it_mk.max())) <= 2


def test_single_query_shape_against_cholesky():
    """The paper's query shape (N = 5867, E = 4694, one RHS per image): k = 1
    and k = 64 columns against dense Cholesky."""
    import torch
    dev = device()
    p = synth.single_query(k=64)
    tol = 1e-6 / (1 + 1 / p.lam)
    say("cg_wg single-query shape")
    h = build(p, dev)
    Fo = _dense_solution(p, p.Y)
    F1, it1, rel1, st1 = hgl().cg_solve_wg(h, p.lam, torch.from_numpy(p.Y[:, :1].copy()).to(dev, torch.float32),
                                           tol=tol)
    assert st1 == 0 and rel1[0, 0] <= tol
    assert colrelerr(F1.cpu().double().numpy(), Fo[:, :1]).max() <= 1e-6
    F, it, rel, st = hgl().cg_solve_wg(h, p.lam, torch.from_numpy(p.Y).to(dev, torch.float32), tol=tol)
    assert st == 0 and np.all(rel <= tol)
    assert colrelerr(F.cpu().double().numpy(), Fo).max() <= 1e-6
    # a column's result does not depend on the other columns of the launch
    assert np.array_equal(F1.cpu().numpy()[:, 0], F.cpu().numpy()[:, 0])


def test_bitwise_repeatable_and_strided():
    """Two solves give identical bits; a strided Y view (ld > k) and an F
    written into a wider buffer give the same columns."""
    import torch
    dev = device()
    p = _g2(1500, 1200, 12, 91)
    h = build(p, dev)
    Yd = torch.from_numpy(p.Y).to(dev, torch.float32)
    F1, _, _, _ = hgl().cg_solve_wg(h, p.lam, Yd, tol=1e-7)
    F2, _, _, _ = hgl().cg_solve_wg(h, p.lam, Yd, tol=1e-7)
    assert torch.equal(F1, F2)
    wide = torch.zeros((p.N, 20), dtype=torch.float32, device=dev)
    wide[:, 3:15] = Yd
    F3, _, _, _ = hgl().cg_solve_wg(h, p.lam, wide[:, 3:15], tol=1e-7)
    assert torch.equal(F1, F3)


def test_x0_limits_and_breakdown():
    import torch
    dev = device()
    p = _g2(800, 640, 6, 95)
    tol = 1e-6 / (1 + 1 / p.lam)
    h = build(p, dev)
    Yd = torch.from_numpy(p.Y).to(dev, torch.float32)
    Fo = _dense_solution(p, p.Y)
    # start from the solution (rounded to FP32, relres about 1e-7): finished
    # by the first check, no iteration
    x0 = torch.from_numpy(Fo).to(dev, torch.float32)
    F, it, rel, st = hgl().cg_solve_wg(h, p.lam, Yd, tol=1e-6, x0=x0)
    assert st == 0 and it.max() == 0 and np.all(rel <= 1e-6)
    # iteration limit: the last iterate and its true residual come back
    F, it, rel, st = hgl().cg_solve_wg(h, p.lam, Yd, tol=1e-7, max_iter=2)
    assert st == 1 and it.max() == 2 and np.all(rel > 1e-7) and np.all(np.isfinite(rel))
    # NaN input: breakdown, reported as an error
    Yn = Yd.clone()
    Yn[3, 2] = float("nan")
    with pytest.raises(Exception) as ei:
        hgl().cg_solve_wg(h, p.lam, Yn, tol=tol)
    assert "EBREAKDOWN" in str(ei.value)
    with pytest.raises(Exception) as ei:
        hgl().cg_solve_wg(h, -1.0, Yd, tol=tol)
    assert "EINVAL" in str(ei.value)


@pytest.mark.parametrize("case", ["sparse", "all_vertex_edge"])
def test_share_boundaries(case):
    """The per-thread shares of the CSRs: fewer incidences than threads
    (empty shares inside row spans) and one hyperedge over all vertices (a row
    running through hundreds of shares), against dense Cholesky."""
    import torch
    dev = device()
    rng = synth.rng_for(101)
    if case == "sparse":
        N, E = 400, 90
        edges = [sorted(rng.choice(N, size=int(rng.integers(2, 5)), replace=False)) for _ in range(E)]
    else:
        N, E = 3000, 1200
        edges = [list(range(N))] + [sorted(rng.choice(N, size=int(rng.integers(2, 9)), replace=False))
                                    for _ in range(E - 1)]
    ep, ev = synth.explicit_hyperedges(edges)
    p = synth.Problem(N, E, ep, ev, rng.uniform(0.2, 1.0, size=E), 0.6, rng.standard_normal((N, 9)))
    tol = 1e-6 / (1 + 1 / p.lam)
    say("cg_wg share boundaries", case, "nnz", len(ev))
    h = build(p, dev)
    F, it, rel, st = hgl().cg_solve_wg(h, p.lam, torch.from_numpy(p.Y).to(dev, torch.float32), tol=tol)
    assert st == 0 and np.all(rel <= tol)
    assert colrelerr(F.cpu().double().numpy(), _dense_solution(p, p.Y)).max() <= 1e-6


def test_no_hyperedges_and_unsupported_requests():
    import torch
    from paper_1908_08281_amd import _lib
    dev = device()
    rng = synth.rng_for(97)
    lam = 0.7
    N, k = 700, 5
    Y0 = rng.standard_normal((N, k))
    p0 = synth.Problem(N, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), lam, Y0)
    h0 = build(p0, dev)
    F, it, rel, st = hgl().cg_solve_wg(h0, lam, torch.from_numpy(Y0).to(dev, torch.float32), tol=2e-7)
    assert st == 0 and it.max() <= 2
    assert colrelerr(F.cpu().double().numpy(), lam / (1 + lam) * Y0).max() <= 1e-6
    # FP64 mode is not part of this path
    lib = _lib.load()
    Y64 = torch.from_numpy(Y0).to(dev, torch.float64)
    F64 = torch.empty_like(Y64)
    opts = _lib.CgOpts(_lib.HGL_CG_PLAIN_F64, 1e-10, 100, 0, 0, 0, 0, 0)
    with torch.cuda.device(dev):
        st = lib.hgl_cg_solve_wg(h0.ptr, lam, C.byref(opts), C.c_void_p(Y64.data_ptr()), k,
                                 C.c_void_p(F64.data_ptr()), k, k, None, None,
                                 C.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    assert st == _lib.HGL_EUNSUPPORTED
    # more incidences than the threads' shares hold (N and E within bounds)
    ep, ev = synth.uniform_hyperedges(6000, 5000, 8, 12, 98)
    pc = synth.Problem(6000, 5000, ep, ev, synth.uniform_weights(5000), lam, np.ones((6000, 1)))
    hc = build(pc, dev)
    with pytest.raises(Exception) as ei:
        hgl().cg_solve_wg(hc, lam, torch.ones((6000, 1), dtype=torch.float32, device=dev))
    assert "EUNSUPPORTED" in str(ei.value)
    # a graph above the row and hyperedge bounds
    ep, ev = synth.uniform_hyperedges(30000, 24000, 2, 6, 99)
    pb = synth.Problem(30000, 24000, ep, ev, synth.uniform_weights(24000), lam, np.ones((30000, 1)))
    hb = build(pb, dev)
    with pytest.raises(Exception) as ei:
        hgl().cg_solve_wg(hb, lam, torch.ones((30000, 1), dtype=torch.float32, device=dev))
    assert "EUNSUPPORTED" in str(ei.value)


def _graph(p, g):
    """Graph g of a batched problem as a problem of its own (local ids)."""
    v0, v1 = int(p.vtx_offsets[g]), int(p.vtx_offsets[g + 1])
    e0, e1 = int(p.edge_offsets[g]), int(p.edge_offsets[g + 1])
    ep = (p.edge_ptr[e0:e1 + 1] - p.edge_ptr[e0]).astype(np.int32)
    ev = (p.edge_vtx[p.edge_ptr[e0]:p.edge_ptr[e1]] - v0).astype(np.int32)
    return synth.Problem(v1 - v0, e1 - e0, ep, ev, p.w[e0:e1], float(p.lams[g]), p.Y[v0:v1])


def test_batched_graphs_against_cholesky():
    """Six G2 graphs of 300-5000 vertices, one without hyperedges, one lambda
    per graph: every (graph, column) is its own workgroup; each graph's
    block against dense Cholesky, and the whole batch against the
    multi-kernel batched solver."""
    import torch
    dev = device()
    pb = synth.batch_of_graphs(seed_offset=3, G=6, nlo=300, nhi=5000, k=7, smax=100)
    # graph 2 loses its hyperedges (an operator of (1 + 1/lambda) I there)
    e0, e1 = int(pb.edge_offsets[2]), int(pb.edge_offsets[3])
    keep = np.r_[0:e0, e1:pb.E]
    counts = np.diff(pb.edge_ptr)[keep]
    starts = pb.edge_ptr[:-1][keep]
    ev = np.concatenate([pb.edge_vtx[s:s + c] for s, c in zip(starts, counts)]).astype(np.int32)
    ep = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    eoff = pb.edge_offsets.copy()
    eoff[3:] -= e1 - e0
    lams = np.array([0.5, 0.3, 0.8, 0.5, 1.0, 0.4])
    p = synth.Problem(pb.N, pb.E - (e1 - e0), ep, ev, pb.w[keep], 0.5, pb.Y, vtx_offsets=pb.vtx_offsets,
                      edge_offsets=eoff, lams=lams)
    tol = 1e-6 / (1 + 1 / lams.min())
    say("cg_wg batched graphs", p.N)
    h = build(p, dev)
    Yd = torch.from_numpy(p.Y).to(dev, torch.float32)
    F, it, rel, st = hgl().cg_solve_wg_batched(h, lams, Yd, tol=tol)
    assert st == 0 and it.shape == (6, 7) and np.all(rel <= tol)
    F = F.cpu().double().numpy()
    for g in range(6):
        q = _graph(p, g)
        v0, v1 = int(p.vtx_offsets[g]), int(p.vtx_offsets[g + 1])
        assert colrelerr(F[v0:v1], _dense_solution(q, q.Y)).max() <= 1e-6, g
    Fm, itm, relm, stm = hgl().cg_solve_batched(h, lams, Yd, tol=tol)
    assert stm == 0
    assert colrelerr(F, Fm.cpu().double().numpy()).max() <= 2e-6


def test_batched_graph_too_large_is_refused():
    import torch
    dev = device()
    p = synth.batch_of_graphs(seed_offset=4, G=3, nlo=6500, nhi=7000, k=2, smax=50)
    h = build(p, dev)
    with pytest.raises(Exception) as ei:
        hgl().cg_solve_wg_batched(h, p.lams, torch.from_numpy(p.Y).to(dev, torch.float32))
    assert "EUNSUPPORTED" in str(ei.value)
