"""Shared helpers for the GPU parity tests."""
from __future__ import annotations

import sys

import numpy as np
import pytest

try:
    import torch
except Exception:  # pragma: no cover
    torch = None


def device():
    if torch is None or not torch.cuda.is_available():
        pytest.skip("no ROCm GPU visible")
    return torch.device("cuda:0")


def hgl():
    from paper_1908_08281_amd import hgl as _h
    _h.lib()  # raises if libhgl.so is not built: no fallback
    return _h


def say(*a):
    """Name the case before a GPU step (flushed, so it survives a crash)."""
    print(*a, file=sys.stderr, flush=True)


def upload(p, dev):
    ep = torch.from_numpy(np.ascontiguousarray(p.edge_ptr, dtype=np.int32)).to(dev)
    ev = torch.from_numpy(np.ascontiguousarray(p.edge_vtx, dtype=np.int32)).to(dev)
    w = torch.from_numpy(np.ascontiguousarray(p.w, dtype=np.float64)).to(dev)
    return ep, ev, w


def build(p, dev):
    h = hgl()
    ep, ev, w = upload(p, dev)
    if p.vtx_offsets is not None:
        return h.build_laplacian_batched(p.vtx_offsets, p.edge_offsets, ep, ev, w)
    return h.build_laplacian(ep, ev, w, p.N)


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def colrelerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b, axis=0)
    return np.linalg.norm(a - b, axis=0) / np.where(nb > 0, nb, 1.0)
