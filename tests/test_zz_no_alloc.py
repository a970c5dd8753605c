"""The entry point that allocates nothing (hgl_apply_noalloc) against hgl_apply:
two calls in a row (the second with a smaller input) give the same Q, no device
memory is taken by the call, and an input too large for the fixed scratch is
refused.  Operator: section 2, eq. 1."""
import numpy as np
import pytest

import synth
from oracle import laplacian as lap
from tests.helpers import build, colrelerr, device, hgl, say

pytestmark = pytest.mark.gpu


def _apply_both(h, lam, P, noalloc_first=False):
    import torch
    Q_ref = torch.empty_like(P)
    Q_na = torch.full_like(P, float("nan"))
    if noalloc_first:
        hgl().apply(h, lam, P, out=Q_na, noalloc=True)
        hgl().apply(h, lam, P, out=Q_ref)
    else:
        hgl().apply(h, lam, P, out=Q_ref)
        hgl().apply(h, lam, P, out=Q_na, noalloc=True)
    torch.cuda.synchronize()
    return Q_ref, Q_na


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_matches_apply_on_two_calls(dtype):
    import torch
    dev = device()
    tdt = torch.float32 if dtype == "f32" else torch.float64
    # hubs (chunked rows) and long hyperedges, several tiles, ragged k
    p = synth.multi_rhs(N=3000, E=2500, k=1, smax=120)
    h = build(p, dev)
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    M = lap.system_matrix(H, p.w, p.lam)
    tol = 1e-13 if dtype == "f64" else 2e-6
    for call, (k, lam) in enumerate(((67, p.lam), (9, 0.2))):
        say("noalloc", dtype, "call", call, "k", k, "lam", lam)
        P = torch.from_numpy(synth.rng_for(100 + k).standard_normal((p.N, k))).to(dev, tdt)
        Q_ref, Q_na = _apply_both(h, lam, P, noalloc_first=(call == 0))
        assert torch.equal(Q_ref, Q_na), (dtype, k)  # same kernels, same order: bit for bit
        Mref = lap.system_matrix(H, p.w, lam) if lam != p.lam else M
        assert colrelerr(Q_na.cpu().numpy(), Mref @ P.cpu().double().numpy()).max() < tol


def test_noalloc_takes_no_device_memory_and_refuses_oversize():
    import torch
    dev = device()
    p = synth.multi_rhs(N=40_000, E=32_000, k=1, smax=200)
    h = build(p, dev)
    k = 200
    P = torch.from_numpy(synth.rng_for(7).standard_normal((p.N, k))).to(dev, torch.float32)
    Q = torch.empty_like(P)
    # first call on a fresh handle: hgl_apply would reserve Z (E x k x 4 = 25.6 MB)
    say("noalloc: fresh handle, memory")
    hgl().apply(h, p.lam, P[:, :8].contiguous(), out=Q[:, :8].contiguous(), noalloc=True)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info(dev)
    held0 = torch.cuda.memory_allocated(dev)  # the handle's buffers come from torch's allocator
    hgl().apply(h, p.lam, P, out=Q, noalloc=True)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info(dev)
    assert free0 - free1 < 4 << 20, (free0, free1)
    assert torch.cuda.memory_allocated(dev) == held0
    Q_ref = hgl().apply(h, p.lam, P)
    assert torch.equal(Q, Q_ref)
    # E x k x 8 = 51 MB of FP64 Z, plus the hub partials: over 64 MiB at k = 300
    say("noalloc: oversize refused")
    P64 = torch.zeros((p.N, 300), dtype=torch.float64, device=dev)
    Q64 = torch.full_like(P64, 1.0)
    from paper_1908_08281_amd import _lib
    with pytest.raises(_lib.HglError) as ei:
        hgl().apply(h, p.lam, P64, out=Q64, noalloc=True)
    assert ei.value.status == _lib.HGL_EUNSUPPORTED
    torch.cuda.synchronize()
    assert bool((Q64 == 1.0).all())  # nothing was launched
