"""The execution plan of the Schur-complement block inverse, checked on the
CPU: the library's own task lists (hgl_block_schur_plan, a host-only call)
are executed in NumPy FP64 on a flat workspace, with every view checked
against the workspace's bounds, unwritten elements poisoned with NaN, and no
task of a phase reading or writing what another task of that phase writes.
The result must be the oracle's inverse (eqs. 12-15)."""
import numpy as np
import pytest

import synth
from oracle import laplacian as lap
from oracle import schur

hgl = pytest.importorskip("paper_1908_08281_amd.hgl")


def _lib_or_skip():
    from paper_1908_08281_amd import _lib
    try:
        _lib.load()
    except Exception as e:  # the library is built by __graft_entry__.build()
        pytest.skip(f"libhgl.so not loadable: {e}")


def _idx(size, off, ld, rows, cols):
    assert off >= 0 and ld >= cols >= 1 and rows >= 1
    last = off + (rows - 1) * ld + cols - 1
    assert last < size, "view past the end of the workspace"
    return off + np.arange(rows)[:, None] * ld + np.arange(cols)[None, :]


def run_plan(plan, M_blocks):
    size = plan["arena_elems"]
    arena = np.full(size, np.nan)
    for b, Mb in enumerate(M_blocks):
        n = Mb.shape[0]
        arena[_idx(size, int(plan["moff"][b]), n, n, n)] = Mb
    tasks, leaves, tiles = plan["tasks"], plan["leaves"], plan["tiles"]
    seen_tasks = np.zeros(len(tasks), dtype=np.int64)
    for tile0, ntiles, leaf0, nleaves, leaf_n in plan["phases"]:
        writes, results, reads = [], [], []
        for i, o, ldi, ldo, n in leaves[leaf0:leaf0 + nleaves]:
            assert n <= leaf_n
            src = _idx(size, i, ldi, n, n)
            X = arena[src]
            assert np.isfinite(X).all(), "a leaf reads unwritten memory"
            dst = _idx(size, o, ldo, n, n)
            reads.append(src)
            writes.append(dst)
            results.append(np.linalg.inv(X))
        ph_tiles = tiles[tile0:tile0 + ntiles]
        # empty slots (product -1) pad the XCD order: the tiles of a product
        # all sit at positions of one residue modulo 8
        for t in dict.fromkeys(ph_tiles[:, 0].tolist()):
            if t < 0:
                continue
            assert len(set((np.nonzero(ph_tiles[:, 0] == t)[0] % 8).tolist())) == 1
            a, b, c, d, lda, ldb, ldc, ldd, m, n, k, alpha, beta = tasks[t].tolist()
            mine = ph_tiles[ph_tiles[:, 0] == t, 1]
            want = {(i << 16) | j for i in range(-(-m // 64)) for j in range(-(-n // 64))}
            assert sorted(mine.tolist()) == sorted(want), "tiles do not cover the product once each"
            seen_tasks[t] += 1
            ia, ib = _idx(size, a, lda, m, k), _idx(size, b, ldb, k, n)
            A, B = arena[ia], arena[ib]
            assert np.isfinite(A).all() and np.isfinite(B).all(), "a product reads unwritten memory"
            D = alpha * (A @ B)
            reads += [ia, ib]
            if beta != 0:
                ic = _idx(size, c, ldc, m, n)
                C = arena[ic]
                assert np.isfinite(C).all()
                D = D + beta * C
                reads.append(ic)
            writes.append(_idx(size, d, ldd, m, n))
            results.append(D)
        mask = np.zeros(size, dtype=bool)
        for w in writes:
            assert not mask[w].any(), "two tasks of one phase write the same element"
            mask[w] = True
        for r in reads:
            assert not mask[r].any(), "a task reads what its own phase writes"
        for w, v in zip(writes, results):
            arena[w] = v
    assert (seen_tasks == 1).all(), "a product runs in no phase or in several"
    out, at = [], 0
    for Mb in M_blocks:
        n = Mb.shape[0]
        out.append(arena[at:at + n * n].reshape(n, n).copy())
        at += n * n
    assert at == plan["inv_elems"]
    return out


def _blocks(sizes, seed, lam=0.5):
    off = synth.block_offsets(np.array(sizes))
    N = int(off[-1])
    ep, ev = synth.uniform_hyperedges(N, int(0.75 * N), 2, 20, seed)
    Hs = lap.incidence_sparse(N, len(ep) - 1, ep, ev)
    w = synth.dirichlet_weights(len(ep) - 1, seed + 1)
    return off, [schur.system_block(Hs, w, lam, off[b], off[b + 1]) for b in range(len(sizes))]


@pytest.mark.parametrize("sizes,min_block", [([300, 257, 130, 64, 17], 16), ([700, 99, 100, 101], 50),
                                             ([513, 64, 128], 64), ([31], 16), ([1300, 600, 131], 500)])
def test_plan_executes_to_the_oracle_inverse(sizes, min_block):
    _lib_or_skip()
    off, Ms = _blocks(sizes, 91 + min_block)
    plan = hgl.block_schur_plan(off, min_block)
    # the leaves are the nested tessellation's smallest submatrices
    for n in sizes:
        for _, m in schur.nested_tessellation(n, min_block):
            assert m < 2 * min_block
    assert (plan["leaves"][:, 4] <= 127).all()
    flops = sum(2 * t[8] * t[9] * t[10] for t in plan["tasks"].tolist())
    assert plan["flops"] == flops
    got = run_plan(plan, Ms)
    for Mb, Gi in zip(Ms, got):
        want = schur.schur_inverse(Mb, min_block)
        assert np.abs(Gi - want).max() < 1e-12


def test_plan_phase_count_and_argument_checks():
    _lib_or_skip()
    from paper_1908_08281_amd._lib import HglError
    plan = hgl.block_schur_plan([0, 1500], 50)
    # depth 4 (1500 -> 750 -> 375 -> 187/188 -> 93/94): P(d) = 2 P(d-1) + 3, P(0) = 1
    assert len(plan["phases"]) == 61
    assert len(plan["leaves"]) == 4 ** 4
    for bad in ([0, 5000], [0, 0, 10]):
        with pytest.raises(HglError):
            hgl.block_schur_plan(bad, 50)
    for mb in (15, 4097):
        with pytest.raises(HglError):
            hgl.block_schur_plan([0, 500], mb)
    # the paper's minimum of 500: smallest submatrices of 500-999 rows, each
    # inverted exactly by the construction carried on to pieces of <= 127 rows
    plan = hgl.block_schur_plan([0, 1500], 500)
    assert (plan["leaves"][:, 4] <= 127).all()
    assert [m for _, m in schur.nested_tessellation(1500, 500)] == [750, 750]
