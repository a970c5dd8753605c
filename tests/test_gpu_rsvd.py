"""GPU parity: block randomized SVD (Algorithm 1 on the tessellated diagonal
blocks), the block inverse (eq. 15, identity-plus-low-rank form) and the
refined solve, against the FP64 oracle on the same sketch Omega."""
import numpy as np
import pytest

import synth
from oracle import laplacian as lap
from oracle import philox, rsvd, solve
from tests.helpers import build, colrelerr, device, hgl, say

pytestmark = pytest.mark.gpu


def _omega(p, l, seed):
    bits, vals = synth.gaussian_sketch(p.N, l, seed)
    return bits, vals


def _to_dev_bits(bits, dev):
    import torch
    return torch.from_numpy(bits.view(np.int16).copy()).to(dev)


def _block_local(sizes, edges_per_block, seed):
    rng = synth.rng_for(seed)
    off = synth.block_offsets(np.array(sizes))
    edges = []
    for b, nb in enumerate(sizes):
        for _ in range(edges_per_block):
            sz = int(rng.integers(2, 7))
            edges.append(sorted(rng.choice(nb, size=sz, replace=False) + off[b]))
    ep, ev = synth.explicit_hyperedges(edges)
    N, E = int(off[-1]), len(ep) - 1
    return synth.Problem(N, E, ep, ev, synth.dirichlet_weights(E, seed + 1), 0.8,
                         synth.binary_rhs(N, 6, 0.1, seed + 2), blocks=off)


def test_f64_exact_rank_recovery():
    """Blocks of rank <= k are recovered exactly (FP64 products)."""
    dev = device()
    p = _block_local([100, 130, 96], 10, 21)
    k, pp = 16, 8
    bits, vals = _omega(p, k + pp, 5)
    say("rsvd f64 exact rank")
    h = build(p, dev)
    U, sig = hgl().block_rsvd(h, p.blocks, k, pp, 2, sketch="f64", omega=_to_dev_bits(bits, dev))
    U, sig = U.cpu().double().numpy(), sig.cpu().numpy()
    A = lap.adjacency(lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx), p.w)
    for b, Ab in enumerate(rsvd.tessellate(A, p.blocks)):
        Ub = U[p.blocks[b]:p.blocks[b + 1]]
        ev = np.sort(np.linalg.eigvalsh(Ab))[::-1][:k]
        assert np.allclose(sig[b], ev, atol=1e-6 * ev[0])   # U stored in FP32
        rec = Ub @ np.diag(sig[b]) @ Ub.T
        assert np.linalg.norm(rec - Ab) / np.linalg.norm(Ab) < 1e-6


def _tess_problem(n_blocks=6, lo=150, hi=300):
    return synth.tessellated(n_blocks=n_blocks, lo=lo, hi=hi, k_rhs=12)


@pytest.mark.parametrize("k,pp,n_blocks", [(24, 8, 6), (1, 1, 6), (2, 1, 6), (3, 2, 6), (80, 16, 6), (24, 8, 1),
                                            (24, 8, 3)])
def test_bf16_sigma_and_approximation_match_oracle(k, pp, n_blocks):
    """Same Omega: top-k sigma and the approximation error agree with the
    oracle's Algorithm 1 run on the BF16-rounded blocks (kernel correctness);
    the error against the FP64 blocks is reported as the true error.  Sketch
    widths l = k + p from 2 (no Householder step) and 3 (one) to 96, the
    widest supported; one block (a single group of blocks) and three (groups
    of one and two)."""
    dev = device()
    p = _tess_problem(n_blocks=n_blocks)
    q = 2
    bits, vals = _omega(p, k + pp, 9)
    say(f"rsvd bf16 vs oracle k={k} p={pp} blocks={n_blocks}")
    h = build(p, dev)
    U, sig = hgl().block_rsvd(h, p.blocks, k, pp, q, sketch="bf16", omega=_to_dev_bits(bits, dev))
    U, sig = U.cpu().double().numpy(), sig.cpu().numpy()
    A = lap.adjacency(lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx), p.w)
    for b, Ab in enumerate(rsvd.tessellate(A, p.blocks)):
        o0, o1 = p.blocks[b], p.blocks[b + 1]
        Ab16 = synth.bf16_round(Ab)[1]
        Uo, so, _ = rsvd.randomized_svd(Ab16, vals[o0:o1], q)
        assert np.max(np.abs(sig[b] - so[:k]) / so[:k]) <= 1e-3
        Ub = U[o0:o1]
        err_gpu = np.linalg.norm(Ab - Ub @ np.diag(sig[b]) @ Ub.T)
        err_or = np.linalg.norm(Ab - Uo[:, :k] @ np.diag(so[:k]) @ Uo[:, :k].T)
        assert abs(err_gpu - err_or) <= 1e-3 * err_or
        # the kept Ritz values never exceed the true eigenvalues (interlacing)
        ev = np.sort(np.linalg.eigvalsh(Ab))[::-1][:k]
        assert np.all(sig[b] <= ev * (1 + 3e-3) + 1e-12)


def test_block_inverse_start_matches_oracle():
    """F0 = blockdiag(M_bb^-1) Y (no refinement) against the oracle's
    identity-plus-low-rank inverse built from its own Algorithm 1 (same Omega)."""
    import torch
    dev = device()
    p = _tess_problem()
    k, pp, q = 24, 8, 2
    bits, vals = _omega(p, k + pp, 9)
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    F0, it, rel, sig, st = hgl().block_rsvd_invert(h, p.lam, p.blocks, Y, k, pp, q, omega=_to_dev_bits(bits, dev),
                                                   refine_tol=10.0)
    assert st == 0 and it.max() == 0
    A = lap.adjacency(lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx), p.w)
    blocks = [synth.bf16_round(Ab)[1] for Ab in rsvd.tessellate(A, p.blocks)]
    oms = [vals[p.blocks[b]:p.blocks[b + 1]] for b in range(len(blocks))]
    fac = rsvd.block_inverse_factors(blocks, oms, k, q)
    F0o = rsvd.block_inverse_apply(fac, p.blocks, p.lam, p.Y)
    assert colrelerr(F0.cpu().numpy(), F0o).max() <= 1e-3


def test_refined_solve_matches_cholesky():
    """BF16-sketch block inverse + preconditioned CG refined to 1e-6 forward error."""
    import torch
    dev = device()
    p = _tess_problem()
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    tol = 1e-6 / (1 + 1 / p.lam)
    F, it, rel, sig, st = hgl().block_rsvd_invert(h, p.lam, p.blocks, Y, 24, 8, 2, seed=3, refine_tol=tol)
    assert st == 0 and np.all(rel <= tol)
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    Fo = solve.solve_dense(lap.system_matrix(H, p.w, p.lam), p.Y)
    assert colrelerr(F.cpu().numpy(), Fo).max() <= 1e-6
    # the preconditioner does not slow CG down
    _, it_cg, _, _ = hgl().cg_solve(h, p.lam, Y, tol=tol)
    assert it.max() <= it_cg.max()


def test_block_local_operator_is_inverted_exactly():
    """Edges inside blocks and rank(A_bb) <= k: the block inverse is the exact
    inverse, so the refinement needs at most one iteration."""
    import torch
    dev = device()
    p = _block_local([100, 130, 96], 10, 33)
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    F, it, rel, sig, st = hgl().block_rsvd_invert(h, p.lam, p.blocks, Y, 16, 8, 1, sketch="f64", seed=1,
                                                  refine_tol=1e-6)
    assert st == 0 and it.max() <= 1
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    Fo = solve.solve_dense(lap.system_matrix(H, p.w, p.lam), p.Y)
    assert colrelerr(F.cpu().numpy(), Fo).max() <= 1e-6


def test_philox_sketch_matches_published_generator():
    dev = device()
    rows, l, seed = 1500, 37, 0x1234_5678_9ABC
    g = hgl().sketch_gaussian(rows, l, seed, dev).cpu().numpy().view(np.uint16)
    ref_bits, _ = synth.bf16_round(philox.gaussian_sketch(rows, l, seed))
    same = np.mean(g == ref_bits)
    assert same >= 0.999
    diff = np.abs(g.astype(np.int64) - ref_bits.astype(np.int64))
    assert diff.max() <= 1   # at most one BF16 ulp (last-bit rounding of log/cos)


def test_philox_words_bit_exact():
    """The device generator's integer words, bit for bit: the published
    known-answer vectors and a sweep of counters and keys, against the
    oracle's independently written Philox4x32-10 (itself pinned by the same
    known answers on the CPU)."""
    import torch
    dev = device()
    kat = [((0, 0, 0, 0), 0, (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
           ((0xFFFFFFFF,) * 4, 0xFFFFFFFF_FFFFFFFF, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
           ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0x299F31D0 << 32) | 0xA4093822,
            (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, out in kat:
        c = torch.from_numpy(np.array([ctr], dtype=np.uint32).view(np.int32)).to(dev)
        got = hgl().philox4x32_10(c, key).cpu().numpy().view(np.uint32)[0]
        assert tuple(int(x) for x in got) == out
    rng = synth.rng_for(77)
    for key in (0, 0x1234_5678_9ABC, int(rng.integers(0, 2**63))):
        say("philox words key", hex(key))
        n = 100_003
        c = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64)
        c[:1000, 2:] = 0  # the sketch's counters: (index low, index high, 0, 0)
        c[:1000, 0] = np.arange(1000)
        c[:1000, 1] = 0
        got = hgl().philox4x32_10(torch.from_numpy(c.astype(np.uint32).view(np.int32)).to(dev), key)
        got = got.cpu().numpy().view(np.uint32)
        ref = philox.philox4x32_10([c[:, i] for i in range(4)], [np.uint64(key & 0xFFFFFFFF),
                                                                   np.uint64(key >> 32)])
        for i in range(4):
            assert np.array_equal(got[:, i].astype(np.uint64), ref[i]), (key, i)


def test_errors():
    import torch
    dev = device()
    p = _tess_problem(n_blocks=3, lo=60, hi=80)
    h = build(p, dev)
    with pytest.raises(Exception) as ei:   # a block smaller than l
        hgl().block_rsvd(h, p.blocks, 60, 30, 1)
    assert "EINVAL" in str(ei.value)
    with pytest.raises(Exception) as ei:   # offsets do not cover [0, N)
        hgl().block_rsvd(h, p.blocks[:-1], 8, 4, 1)
    assert "EINVAL" in str(ei.value)
    zero = torch.zeros((p.N, 12), dtype=torch.int16, device=dev)
    with pytest.raises(Exception) as ei:   # a zero sketch has a singular Gram matrix
        hgl().block_rsvd(h, p.blocks, 8, 4, 1, omega=zero)
    assert "ECHOLQR" in str(ei.value)


@pytest.mark.slow
def test_full_size_tessellation():
    """The batched rSVD workload at full size (50 blocks of 500-1500 rows,
    k=64, p=10, q=2): sigma of sampled blocks against the oracle on the same
    Omega, and the refined solve against the FP64 Tier-2 oracle on sampled
    columns."""
    import torch
    dev = device()
    p = synth.tessellated()
    k, pp, q = 64, 10, 2
    bits, vals = _omega(p, k + pp, 11)
    say("rsvd full size", p.N)
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    tol = 1e-6 / (1 + 1 / p.lam)
    F, it, rel, sig, st = hgl().block_rsvd_invert(h, p.lam, p.blocks, Y, k, pp, q,
                                                  omega=_to_dev_bits(bits, dev), refine_tol=tol)
    assert st == 0 and np.all(rel <= tol)
    sig = sig.cpu().numpy()
    op = lap.SparseOperator(p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam)
    for b in (0, 17, 49):
        o0, o1 = p.blocks[b], p.blocks[b + 1]
        E_b = np.eye(o1 - o0)
        Ab = np.zeros((o1 - o0, o1 - o0))
        for j in range(0, o1 - o0, 256):    # A_bb column panels from the sparse operator
            P = np.zeros((p.N, min(256, o1 - o0 - j)))
            P[o0:o1] = E_b[:, j:j + P.shape[1]]
            Ab[:, j:j + P.shape[1]] = op.adjacency_apply(P)[o0:o1]
        Ab16 = synth.bf16_round(Ab)[1]
        _, so, _ = rsvd.randomized_svd(Ab16, vals[o0:o1], q)
        assert np.max(np.abs(sig[b] - so[:k]) / so[:k]) <= 1e-3
    cols = np.arange(0, p.Y.shape[1], 7)
    fo, _, relo = solve.cg_ranking(op, p.w, p.lam, p.Y[:, cols], tol=1e-13)
    assert colrelerr(F.cpu().numpy()[:, cols], fo).max() <= 1e-6


def test_recorded_graph_replays_match_direct_launches():
    """The rSVD's launches are recorded once and replayed (the host swaps
    the roles of two buffers while recording): replays, a new recording
    after direct launches, and the direct launches themselves give the same
    U and sigma bit for bit."""
    import torch
    dev = device()
    p = _tess_problem()
    k, pp, q = 24, 8, 2
    bits, _ = _omega(p, k + pp, 9)
    say("rsvd graph replays vs direct launches")
    h = build(p, dev)
    om = _to_dev_bits(bits, dev)
    runs = []
    for mode in ("graph", "graph", "graph", "direct", "graph", "graph"):
        if mode == "direct":
            hgl().profile(h, True)
        U, sig = hgl().block_rsvd(h, p.blocks, k, pp, q, sketch="bf16", omega=om)
        torch.cuda.synchronize()
        if mode == "direct":
            hgl().profile(h, False)
        runs.append((U.cpu().numpy(), sig.cpu().numpy()))
    for U, sig in runs[1:]:
        assert np.array_equal(U, runs[0][0]) and np.array_equal(sig, runs[0][1])
