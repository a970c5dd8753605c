"""The handle takes every device buffer from the caller's allocator
(hgl_allocator): with torch's caching allocator, the structure, the solver
workspaces and the build temporaries show up in torch's allocation counter and
all go back to it on destroy; with the library's own hipMalloc they do not.
Both give the same operator and the same solve bit for bit."""
import numpy as np
import pytest

import synth
from tests.helpers import device, hgl, say, upload

pytestmark = pytest.mark.gpu


def test_torch_allocator_owns_every_buffer():
    import torch
    dev = device()
    p = synth.multi_rhs(N=6000, E=4800, k=24, smax=150)
    ep, ev, w = upload(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated(dev)
    say("allocator: torch build")
    h = hgl().build_laplacian(ep, ev, w, p.N, allocator="torch")
    torch.cuda.synchronize()
    after_build = torch.cuda.memory_allocated(dev)
    # structure and scales: 2 nnz int32 + (N + 1) + (E + 1) int32, FP64 and FP32 scales, w
    floor = 4 * (2 * p.nnz + p.N + p.E) + 8 * (2 * p.N + 2 * p.E) + 4 * (p.N + p.E)
    assert after_build - base >= floor, (after_build - base, floor)
    say("allocator: torch solve")
    F1, _, _, st1 = hgl().cg_solve(h, p.lam, Y, tol=3.3e-7)
    torch.cuda.synchronize()
    after_solve = torch.cuda.memory_allocated(dev)
    # the CG workspaces (R, P, Q at least: 3 N k FP32) come from torch too;
    # F1 itself is torch's (N k FP32)
    assert after_solve - after_build >= 4 * p.N * 24 * 4, (after_solve - after_build)
    del F1
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated(dev)
    h.destroy()
    torch.cuda.synchronize()
    assert held > base
    assert torch.cuda.memory_allocated(dev) == base, "destroy must hand every buffer back"

    say("allocator: hip build")
    h2 = hgl().build_laplacian(ep, ev, w, p.N, allocator="hip")
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(dev) == base
    F2, _, _, st2 = hgl().cg_solve(h2, p.lam, Y, tol=3.3e-7)
    h3 = hgl().build_laplacian(ep, ev, w, p.N)  # default: torch
    F3, _, _, st3 = hgl().cg_solve(h3, p.lam, Y, tol=3.3e-7)
    assert st2 == 0 and st3 == 0 and st1 == 0
    assert torch.equal(F2, F3)
    op2, op3 = hgl().get_operator(h2), hgl().get_operator(h3)
    for key in op2:
        assert torch.equal(op2[key], op3[key]), key
    h2.destroy()
    h3.destroy()


def test_transpose_of_hub_rows_and_empty_graph_parts():
    """The hand-written transpose on rows of every kind: isolated vertices,
    short rows (one wave each), hub rows ranked by chunks (up to several
    thousand hyperedges), against the CSC of H built on the host."""
    import torch
    dev = device()
    # one very popular vertex (in every hyperedge) and a tail of short rows
    rng = synth.rng_for(11)
    N, E = 5000, 6000
    edges = []
    for e in range(E):
        m = set(rng.choice(np.arange(1, N), size=int(rng.integers(1, 6)), replace=False).tolist())
        if e % 2 == 0:
            m.add(0)
        edges.append(sorted(m))
    ep, ev = synth.explicit_hyperedges(edges)
    w = synth.dirichlet_weights(E, 3)
    say("transpose: hub of", E // 2)
    h = hgl().build_laplacian(torch.from_numpy(ep).to(dev), torch.from_numpy(ev).to(dev),
                              torch.from_numpy(w).to(dev), N)
    op = hgl().get_operator(h)
    vp = op["vtx_ptr"].cpu().numpy()
    ve = op["vtx_edge"].cpu().numpy()
    import scipy.sparse as sp
    H = sp.csr_matrix((np.ones(ev.size), ev, ep), shape=(E, N)).T.tocsr()
    assert np.array_equal(vp, H.indptr.astype(np.int32))
    for v in range(N):
        assert np.array_equal(ve[vp[v]:vp[v + 1]], np.sort(H.indices[H.indptr[v]:H.indptr[v + 1]])), v
    assert h.partition()["hub_rows"] >= 1
