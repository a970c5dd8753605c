"""GPU parity: CG solves (section 3, eqs. 16-20) against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import laplacian as lap
from oracle import solve
from tests.helpers import build, colrelerr, device, hgl, say

pytestmark = pytest.mark.gpu


def _dense_solution(p, lam=None):
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    return solve.solve_dense(lap.system_matrix(H, p.w, p.lam if lam is None else lam), p.Y)


def test_plain_f64_small_config_matches_cholesky():
    """Plain method, small: N=2000, E=1500, k=50, FP64 CG to relres 1e-10."""
    import torch
    dev = device()
    p = synth.small_plain()
    say("cg f64 small_plain")
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev)
    F, iters, rel, st = hgl().cg_solve(h, p.lam, Y, mode="f64", tol=1e-10, max_iter=200)
    assert st == 0
    Fo = _dense_solution(p)
    F = F.cpu().numpy()
    assert colrelerr(F, Fo).max() <= 2e-10
    op = lap.SparseOperator(p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam)
    rel_oracle = solve.relres(op, F, p.Y)
    assert np.all(rel_oracle <= 1e-10)
    assert np.allclose(rel[0], rel_oracle, rtol=1e-3, atol=1e-14)
    assert iters.max() <= 30


@pytest.mark.parametrize("k", [1, 17, 64, 200])
def test_f32_mixed_matches_oracle(k):
    import torch
    dev = device()
    p = synth.multi_rhs(N=4000, E=3200, k=k, smax=150)
    say("cg f32", k)
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    tol = 1e-6 / (1 + 1 / p.lam)
    F, iters, rel, st = hgl().cg_solve(h, p.lam, Y, mode="f32", tol=tol, max_iter=300)
    assert st == 0
    Fo = _dense_solution(p)
    F = F.cpu().numpy()
    assert colrelerr(F, Fo).max() <= 1e-6
    op = lap.SparseOperator(p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam)
    assert np.all(solve.relres(op, F, p.Y) <= tol * 1.01)


def test_zero_column_x0_and_limits():
    import torch
    dev = device()
    p = synth.multi_rhs(N=1500, E=1200, k=6, smax=60)
    Yn = p.Y.copy()
    Yn[:, 2] = 0.0
    h = build(p, dev)
    Y = torch.from_numpy(Yn).to(dev, torch.float32)
    F, iters, rel, st = hgl().cg_solve(h, p.lam, Y, tol=1e-6, max_iter=300)
    assert st == 0 and iters[0, 2] == 0 and float(F[:, 2].abs().max()) == 0.0
    # warm start from the solution: converged at once
    F2, iters2, rel2, st2 = hgl().cg_solve(h, p.lam, Y, tol=1e-6, max_iter=300, x0=F)
    assert st2 == 0 and iters2.max() <= 1
    # iteration limit -> NOT_CONVERGED, relres of the returned iterate reported
    F3, iters3, rel3, st3 = hgl().cg_solve(h, p.lam, Y, tol=1e-9, max_iter=1)
    assert st3 == 1
    op = lap.SparseOperator(p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam)
    ro = solve.relres(op, F3.cpu().double().numpy(), Yn)
    assert np.allclose(rel3[0], ro, rtol=1e-4, atol=1e-12)


@pytest.mark.parametrize("mode", ["f32", "f64"])
def test_decoupled_rows_solved_at_the_start(mode):
    """Rows with s_v = 0 (isolated vertices, and vertices whose every
    hyperedge has weight 0) are decoupled: M_vv = 1 + 1/lambda and row v of
    A is zero (reading R2).  The fused solver sets F_v = Y_v / (1 + 1/lambda)
    at the start and leaves them out of the iteration.  The whole solution
    still matches dense Cholesky, those rows hold Y_v lambda/(1+lambda) to
    rounding, a start x0 with garbage on them is corrected, and the reported
    relres of an unconverged solve is still the true one."""
    import torch
    dev = device()
    p = synth.multi_rhs(N=2500, E=2000, k=9, smax=80)
    w = p.w.copy()
    w[synth.rng_for(5).choice(p.E, size=p.E // 4, replace=False)] = 0.0  # zero-weight hyperedges
    p.w = w
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    dv = H @ w
    dec = dv == 0
    member = H.sum(axis=1) > 0
    assert dec.sum() > 100 and (dec & member).sum() > 10  # both kinds present
    M = lap.system_matrix(H, w, p.lam)
    Fo = solve.solve_dense(M, p.Y)
    h = build(p, dev)
    dt = torch.float32 if mode == "f32" else torch.float64
    tol = 1e-6 / (1 + 1 / p.lam) if mode == "f32" else 1e-10
    bar = 1e-6 if mode == "f32" else 2e-10
    Y = torch.from_numpy(p.Y).to(dev, dt)
    say("decoupled", mode)
    F, it, rel, st = hgl().cg_solve(h, p.lam, Y, mode=mode, tol=tol, max_iter=500)
    assert st == 0 and np.all(rel <= tol)
    Fn = F.cpu().double().numpy()
    assert colrelerr(Fn, Fo).max() <= bar
    exact = p.Y[dec] * (p.lam / (1 + p.lam))
    eps = np.finfo(np.float32 if mode == "f32" else np.float64).eps
    assert np.all(np.abs(Fn[dec] - exact) <= eps * np.abs(exact))
    # a start with garbage everywhere, decoupled rows included
    x0 = torch.from_numpy(synth.rng_for(6).standard_normal(p.Y.shape)).to(dev, dt)
    F2, it2, rel2, st2 = hgl().cg_solve(h, p.lam, Y, mode=mode, tol=tol, max_iter=500, x0=x0)
    assert st2 == 0 and colrelerr(F2.cpu().double().numpy(), Fo).max() <= bar
    assert np.all(np.abs(F2.cpu().double().numpy()[dec] - exact) <= eps * np.abs(exact))
    # one iteration from that start: the reported relres is the true one
    F3, _, rel3, st3 = hgl().cg_solve(h, p.lam, Y, mode=mode, tol=1e-12, max_iter=1, x0=x0)
    assert st3 == 1
    ro = np.linalg.norm(p.Y - M @ F3.cpu().double().numpy(), axis=0) / np.linalg.norm(p.Y, axis=0)
    assert np.allclose(rel3[0], ro, rtol=1e-6, atol=1e-14)


@pytest.mark.parametrize("max_iter", [1, 2, 3, 4, 5])
def test_iteration_limits_of_every_parity(max_iter):
    """Regression: the FP64 flag words must stay 8-byte aligned for any max_iter."""
    import torch
    dev = device()
    p = synth.multi_rhs(N=1200, E=1000, k=5, smax=50)
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    say("max_iter", max_iter)
    F, iters, rel, st = hgl().cg_solve(h, p.lam, Y, tol=1e-12, max_iter=max_iter)
    assert st == 1 and iters.max() <= max_iter
    op = lap.SparseOperator(p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam)
    ro = solve.relres(op, F.cpu().double().numpy(), p.Y)
    assert np.allclose(rel[0], ro, rtol=1e-4, atol=1e-12)


def test_breakdown_on_nan_and_bad_lambda():
    import torch
    dev = device()
    p = synth.small_plain(N=300, E=200, k=3)
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    Y[5, 1] = float("nan")
    with pytest.raises(Exception) as ei:
        hgl().cg_solve(h, p.lam, Y, tol=1e-6)
    assert "BREAKDOWN" in str(ei.value)
    with pytest.raises(Exception) as ei:
        hgl().cg_solve(h, -1.0, Y, tol=1e-6)
    assert "EINVAL" in str(ei.value)


def test_bitwise_repeatable():
    import torch
    dev = device()
    p = synth.multi_rhs(N=6000, E=5000, k=40, smax=200)
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    a = hgl().cg_solve(h, p.lam, Y, tol=3e-7)[0]
    b = hgl().cg_solve(h, p.lam, Y, tol=3e-7)[0]
    assert torch.equal(a, b)


def test_batched_graphs_each_match_oracle_and_single_solve():
    import torch
    dev = device()
    p = synth.batch_of_graphs(G=5, nlo=400, nhi=1500, k=12)
    lams = np.array([0.5, 1.0, 0.25, 2.0, 0.7])
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    say("batched 5 graphs")
    F, iters, rel, st = hgl().cg_solve_batched(h, lams, Y, tol=2e-7, max_iter=300)
    assert st == 0
    F = F.cpu().numpy()
    for g in range(5):
        v0, v1 = p.vtx_offsets[g], p.vtx_offsets[g + 1]
        e0, e1 = p.edge_offsets[g], p.edge_offsets[g + 1]
        ep = (p.edge_ptr[e0:e1 + 1] - p.edge_ptr[e0]).astype(np.int32)
        ev = (p.edge_vtx[p.edge_ptr[e0]:p.edge_ptr[e1]] - v0).astype(np.int32)
        sub = synth.Problem(v1 - v0, e1 - e0, ep, ev, p.w[e0:e1], lams[g], p.Y[v0:v1])
        Fo = _dense_solution(sub)
        assert colrelerr(F[v0:v1], Fo).max() <= 1e-6
        hs = build(sub, dev)
        Fs = hgl().cg_solve(hs, lams[g], torch.from_numpy(sub.Y).to(dev, torch.float32), tol=2e-7)[0]
        assert colrelerr(F[v0:v1], Fs.cpu().numpy()).max() <= 1e-6


@pytest.mark.slow
def test_multi_rhs_full_size_against_sparse_oracle():
    """Full multi-RHS workload (N=50,000, E=40,000, k=200, lambda=0.5) in the
    bench's launch configuration; every column against the FP64 Tier-2 CG."""
    import torch
    dev = device()
    p = synth.multi_rhs()
    say("cg f32 full size")
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    tol = 1e-6 / (1 + 1 / p.lam)
    F, iters, rel, st = hgl().cg_solve(h, p.lam, Y, tol=tol, max_iter=300)
    assert st == 0
    op = lap.SparseOperator(p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam)
    cols = np.arange(0, 200, 7)
    fo, _, relo = solve.cg_ranking(op, p.w, p.lam, p.Y[:, cols], tol=1e-13)
    assert np.all(relo <= 1e-13)
    assert colrelerr(F.cpu().numpy()[:, cols], fo).max() <= 1e-6
    assert np.all(solve.relres(op, F.cpu().double().numpy(), p.Y) <= tol * 1.01)


@pytest.mark.slow
def test_batch_full_size_against_sparse_oracle():
    """Full batching workload (64 graphs, N_g ~ U[2000, 30000], about 1e6
    vertices, k=100, lambda=0.5) in the bench's launch configuration (no
    periodic replacement, autotuned shapes): every column's FP64 true
    residual on the sampled graphs, and sampled columns against the FP64
    Tier-2 CG of each sampled graph on its own."""
    import torch
    dev = device()
    p = synth.batch_of_graphs()
    say("cg f32 batch full size")
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    tol = 1e-6 / (1 + 1 / 0.5)
    F, iters, rel, st = hgl().cg_solve_batched(h, p.lams, Y, tol=tol, max_iter=300, rr_period=0, tune=True)
    assert st == 0 and np.all(rel <= tol)
    F = F.cpu().double().numpy()
    G = len(p.lams)
    sizes = np.diff(p.vtx_offsets)
    graphs = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 17, 42})
    cols = np.arange(3, 100, 13)
    for g in graphs:
        v0, v1 = p.vtx_offsets[g], p.vtx_offsets[g + 1]
        e0, e1 = p.edge_offsets[g], p.edge_offsets[g + 1]
        ep = (p.edge_ptr[e0:e1 + 1] - p.edge_ptr[e0]).astype(np.int32)
        ev = (p.edge_vtx[p.edge_ptr[e0]:p.edge_ptr[e1]] - v0).astype(np.int32)
        op = lap.SparseOperator(v1 - v0, e1 - e0, ep, ev, p.w[e0:e1], p.lams[g])
        assert np.all(solve.relres(op, F[v0:v1], p.Y[v0:v1]) <= tol * 1.01), g
        fo, _, relo = solve.cg_ranking(op, p.w[e0:e1], p.lams[g], p.Y[v0:v1][:, cols], tol=1e-13)
        assert np.all(relo <= 1e-13)
        assert colrelerr(F[v0:v1][:, cols], fo).max() <= 1e-6, g
    assert G == 64


def test_graph_replay_matches_direct_launches():
    """The first chunk of iterations recorded as a HIP graph: every replay
    (new data at the same addresses, eager solves and synchronisations in
    between) gives bitwise the result of direct launches; a new output
    address records a new graph."""
    import torch
    dev = device()
    p = synth.multi_rhs(N=3000, E=2400, k=24, smax=120)
    h = build(p, dev)
    tol = 1e-6 / (1 + 1 / p.lam)
    rng = synth.rng_for(21)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    out = torch.empty_like(Y)
    Fo = None
    for rep in range(3):
        say("graph replay", rep)
        if rep > 0:  # new right-hand sides at the same address
            Y.copy_(torch.from_numpy((rng.random(p.Y.shape) < 0.03).astype(np.float32)).to(dev))
        F_eager, it_e, rel_e, st_e = hgl().cg_solve(h, p.lam, Y, tol=tol, rr_period=0)
        torch.cuda.synchronize()
        F_g, it_g, rel_g, st_g = hgl().cg_solve(h, p.lam, Y, tol=tol, rr_period=0, graph=True, out=out)
        torch.cuda.synchronize()
        assert st_e == 0 and st_g == 0
        assert torch.equal(F_g, F_eager)
        assert np.array_equal(it_g, it_e) and np.array_equal(rel_g, rel_e)
        if Fo is None:
            Fo = _dense_solution(p)
            assert colrelerr(F_g.cpu().numpy(), Fo).max() <= 1e-6
    out2 = torch.empty_like(Y)
    F2, _, _, st2 = hgl().cg_solve(h, p.lam, Y, tol=tol, rr_period=0, graph=True, out=out2)
    F3, _, _, _ = hgl().cg_solve(h, p.lam, Y, tol=tol, rr_period=0)
    assert st2 == 0 and torch.equal(F2, F3)


@pytest.mark.parametrize("k", [24, 200])
def test_autotuned_shape_matches_oracle_and_is_cached(k):
    """The autotuner picks the column shape by timing on first use; the
    solve still meets the oracle bar, and later solves reuse the cached shape
    (bitwise the same result)."""
    import torch
    dev = device()
    p = synth.multi_rhs(N=3000, E=2400, k=k, smax=120)
    h = build(p, dev)
    tol = 1e-6 / (1 + 1 / p.lam)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    say("autotune", k)
    assert h.gather_shape() == {"edge": (0, 0, 0), "vertex": (0, 0, 0)}
    F1, _, _, st1 = hgl().cg_solve(h, p.lam, Y, tol=tol, tune=True)
    shape1 = h.gather_shape()
    F2, _, _, st2 = hgl().cg_solve(h, p.lam, Y, tol=tol, tune=True)
    assert st1 == 0 and st2 == 0
    for gl, v, slabs in shape1.values():
        assert gl in (4, 8, 16, 32, 64) and v in (1, 2, 4) and slabs >= 1
        assert gl * v * slabs >= k and gl * v * (slabs - 1) < k
    assert h.gather_shape() == shape1
    assert torch.equal(F1, F2)
    assert colrelerr(F1.cpu().numpy(), _dense_solution(p)).max() <= 1e-6


def test_claimed_columns_restart_after_a_failed_check():
    """FP32 CG near its attainable accuracy (no periodic residual
    replacement, and every 8 iterations): the FP32 recursion drifts from the
    true residual, so a check step finds claimed columns short of tol; they
    restart from the recomputed residual and every column still reaches tol
    in the true FP64 residual.  A column still iterating at a check, or at a
    periodic replacement, keeps its direction only while its true residual
    agrees with the recursive one (keeping it regardless diverges at
    lambda = 0.01, tol = 5e-7 in an FP32 model of the recurrence).

    The tolerances sit above the FP32 floor: the exact solution rounded to
    FP32 (the best any FP32 F can do, up to luck in the rounding) has a
    relative residual of up to 3.3e-7 on these columns at lambda = 0.01, so a
    tol of 3e-7 there is below what an FP32 F can be relied on to reach.  A
    tol far below the floor ends at max_iter with status 'not converged' and
    the true residual reported."""
    import torch
    dev = device()
    p = synth.multi_rhs(N=3000, E=2400, k=16, smax=120)
    h = build(p, dev)
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)

    def true_relres(F, lam):
        M = lap.system_matrix(H, p.w, lam)
        Fn = F.cpu().numpy().astype(np.float64)
        return np.linalg.norm(p.Y - M @ Fn, axis=0) / np.linalg.norm(p.Y, axis=0)

    # the FP32 floor at lambda = 0.01: relres of the rounded exact solution
    F_exact = solve.solve_dense(lap.system_matrix(H, p.w, 0.01), p.Y)
    floor = true_relres(torch.from_numpy(F_exact.astype(np.float32)), 0.01).max()
    assert 3e-7 < floor < 5e-7 / 1.25, floor

    resumed = 0
    for lam, tol, rr_period in ((0.5, 1e-7, 0), (0.1, 1e-7, 0), (0.01, 1e-6, 0), (0.01, 5e-7, 0),
                                (0.01, 5e-7, 8)):
        say("restart", lam, tol, rr_period)
        F, it, rel, st = hgl().cg_solve(h, lam, Y, tol=tol, max_iter=3000, rr_period=rr_period)
        stats = h.cg_stats()
        assert st == 0, (lam, tol, rr_period, stats)
        assert stats["checks"] >= 1 and stats["iterations"] >= int(it.max())
        tr = true_relres(F, lam)
        # the reported relres is the FP64 residual of the returned FP32 F
        assert np.allclose(rel[0], tr, rtol=1e-6, atol=0)
        assert tr.max() <= tol
        resumed += stats["resumed"]
    assert resumed >= 1, "no check step sent a column back: the cases do not test the restart"

    say("restart: unattainable tol")
    F, it, rel, st = hgl().cg_solve(h, 0.002, Y, tol=1e-6, max_iter=200, rr_period=0)
    stats = h.cg_stats()
    assert st == 1 and stats["iterations"] == 200 and stats["resumed"] >= 1
    tr = true_relres(F, 0.002)
    assert np.allclose(rel[0], tr, rtol=1e-6, atol=0)
    assert tr.max() > 1e-6


@pytest.mark.parametrize("mode", ["f32", "f64"])
def test_degenerate_hypergraphs(mode):
    """Edge cases of the fused step: no hyperedges at all (no edge tiles, the
    hyperedge half of p'Mp empty: F = lambda/(1+lambda) Y exactly up to
    rounding), a batch in which one graph has no hyperedges, and a
    hypergraph whose hyperedges are all large enough for a whole workgroup
    each (no short hyperedge in any edge tile)."""
    import torch
    dev = device()
    dt = torch.float32 if mode == "f32" else torch.float64
    tol = 2e-7 if mode == "f32" else 1e-12
    bar = 1e-6 if mode == "f32" else 1e-10
    rng = synth.rng_for(11)
    lam = 0.7
    # 1. no hyperedges
    N, k = 500, 7
    Y0 = rng.standard_normal((N, k))
    p0 = synth.Problem(N, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), lam, Y0)
    say("degenerate: E = 0", mode)
    h0 = build(p0, dev)
    F, it, rel, st = hgl().cg_solve(h0, lam, torch.from_numpy(Y0).to(dev, dt), mode=mode, tol=tol)
    assert st == 0
    assert colrelerr(F.cpu().double().numpy(), lam / (1 + lam) * Y0).max() <= bar
    # 2. all hyperedges large (40..90 members)
    N2, E2, k2 = 600, 25, 5
    sizes = rng.integers(40, 91, size=E2)
    ev = np.concatenate([np.sort(rng.choice(N2, size=s, replace=False)) for s in sizes]).astype(np.int32)
    ep = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    w2 = rng.uniform(0.2, 1.0, size=E2)
    Y2 = rng.standard_normal((N2, k2))
    p2 = synth.Problem(N2, E2, ep, ev, w2, lam, Y2)
    say("degenerate: all hyperedges large", mode)
    h2 = build(p2, dev)
    assert h2.partition()["long_edges"] == E2
    F2, it2, rel2, st2 = hgl().cg_solve(h2, lam, torch.from_numpy(Y2).to(dev, dt), mode=mode, tol=tol)
    assert st2 == 0
    assert colrelerr(F2.cpu().double().numpy(), _dense_solution(p2)).max() <= bar
    # 3. a batch whose middle graph has no hyperedges
    pb = synth.batch_of_graphs(G=3, nlo=300, nhi=700, k=4)
    v0, v1 = pb.vtx_offsets[1], pb.vtx_offsets[2]
    e0, e1 = pb.edge_offsets[1], pb.edge_offsets[2]
    keep = np.r_[0:e0, e1:pb.E]
    counts = np.diff(pb.edge_ptr)[keep]
    starts = pb.edge_ptr[:-1][keep]
    ev3 = np.concatenate([pb.edge_vtx[s:s + c] for s, c in zip(starts, counts)]).astype(np.int32)
    ep3 = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    eo3 = pb.edge_offsets.copy()
    eo3[2:] -= e1 - e0
    p3 = synth.Problem(pb.N, pb.E - (e1 - e0), ep3, ev3, pb.w[keep], lam, pb.Y, vtx_offsets=pb.vtx_offsets,
                       edge_offsets=eo3, lams=np.array([0.5, lam, 2.0]))
    say("degenerate: batch with an empty graph", mode)
    h3 = build(p3, dev)
    F3, it3, rel3, st3 = hgl().cg_solve_batched(h3, p3.lams, torch.from_numpy(p3.Y).to(dev, dt), mode=mode, tol=tol)
    assert st3 == 0
    F3 = F3.cpu().double().numpy()
    assert colrelerr(F3[v0:v1], lam / (1 + lam) * p3.Y[v0:v1]).max() <= bar
    for g in (0, 2):
        a0, a1 = p3.vtx_offsets[g], p3.vtx_offsets[g + 1]
        b0, b1 = eo3[g], eo3[g + 1]
        epg = (ep3[b0:b1 + 1] - ep3[b0]).astype(np.int32)
        evg = (ev3[ep3[b0]:ep3[b1]] - a0).astype(np.int32)
        sub = synth.Problem(a1 - a0, b1 - b0, epg, evg, p3.w[b0:b1], p3.lams[g], p3.Y[a0:a1])
        assert colrelerr(F3[a0:a1], _dense_solution(sub)).max() <= bar
