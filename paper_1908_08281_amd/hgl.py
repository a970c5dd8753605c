"""Thin PyTorch-facing binding of the C ABI (include/hgl.h).

Torch supplies device memory and the current HIP stream; every step of the
computation runs in the library's kernels.  Functions take and return torch
tensors on a ROCm device; names follow the C entry points without the
``hgl_`` prefix.
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref

import numpy as np
import torch

from . import _lib
from ._lib import CgOpts, check

MODES = {"f64": _lib.HGL_CG_PLAIN_F64, "f32": _lib.HGL_CG_F32_F64DOT_RR}


def lib():
    return _lib.load()


def _stream(device: torch.device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor | None) -> C.c_void_p:
    return C.c_void_p(t.data_ptr() if t is not None else 0)


def _need(t: torch.Tensor, dtype, name: str, device=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a torch tensor on a ROCm device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    return t


def _rows(t: torch.Tensor, name: str) -> int:
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D row-major tensor with unit column stride")
    return t.stride(0)


class TorchAllocator:
    """torch's caching allocator behind hgl_allocator, so that torch owns every
    device buffer of a handle (its allocations are made for the stream of the
    library call that asks, and go back to torch's cache when freed)."""

    def __init__(self, device: torch.device):
        index = device.index if device.index is not None else torch.cuda.current_device()

        def alloc(nbytes, ctx, stream):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), index, int(stream or 0))
            except Exception:  # the library reports HGL_ENOMEM
                return None

        def free(ptr, ctx, stream):
            try:
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:
                pass

        self._alloc = _lib.ALLOC_FN(alloc)
        self._free = _lib.FREE_FN(free)
        self.struct = _lib.Allocator(self._alloc, self._free, None)


_live_handles = weakref.WeakSet()


@atexit.register
def _destroy_live_handles():
    # before the interpreter tears torch down: the handles' buffers go back
    # to torch's allocator while it still exists
    for h in list(_live_handles):
        h.destroy()


def _allocator(device: torch.device, allocator):
    if allocator == "torch":
        return TorchAllocator(device)
    if allocator is None or allocator == "hip":
        return None
    raise ValueError(f"allocator must be 'torch' or 'hip', got {allocator!r}")


class Handle:
    """Owns an hgl_handle (the built operator of one or more hypergraphs)."""

    def __init__(self, ptr: C.c_void_p, device: torch.device, allocator: TorchAllocator | None = None):
        self._ptr = ptr
        self.device = device
        self._allocator = allocator  # kept alive as long as the handle
        _live_handles.add(self)
        N, E, G = C.c_int32(), C.c_int32(), C.c_int32()
        nnz = C.c_int64()
        check(lib().hgl_get_sizes(ptr, C.byref(N), C.byref(E), C.byref(nnz), C.byref(G)),
              "hgl_get_sizes")
        self.N, self.E, self.nnz, self.G = N.value, E.value, nnz.value, G.value

    def partition(self) -> dict:
        """Work partition of the operator gathers (row tiles, hub rows and
        their chunks, hyperedges handled by a whole workgroup)."""
        v = [C.c_int32() for _ in range(4)]
        check(lib().hgl_get_partition(self.ptr, *(C.byref(x) for x in v)), "hgl_get_partition")
        return dict(zip(("tiles", "hub_rows", "hub_chunks", "long_edges"), (x.value for x in v)))

    def gather_shape(self) -> dict:
        """{"edge": (lanes per row, elements per lane, column slabs), "vertex":
        (...)} of the operator gathers of the latest CG solve on this handle;
        zeros before one."""
        v = (C.c_int32 * 6)()
        check(lib().hgl_get_gather_shape(self.ptr, v), "hgl_get_gather_shape")
        x = [int(a) for a in v]
        return {"edge": tuple(x[:3]), "vertex": tuple(x[3:])}

    def cg_stats(self) -> dict:
        """Iterations enqueued, chunks, check steps and check steps after
        which columns went on, of the latest CG solve on this handle."""
        v = (C.c_int32 * 4)()
        check(lib().hgl_get_cg_stats(self.ptr, v), "hgl_get_cg_stats")
        return dict(zip(("iterations", "chunks", "checks", "resumed"), (int(x) for x in v)))

    @property
    def ptr(self) -> C.c_void_p:
        if self._ptr is None:
            raise RuntimeError("handle already destroyed")
        return self._ptr

    def destroy(self):
        if self._ptr is not None:
            lib().hgl_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def build_laplacian(edge_ptr: torch.Tensor, edge_vtx: torch.Tensor, w: torch.Tensor, N: int,
                    allocator: str | None = "torch") -> Handle:
    """allocator "torch" (default): the handle's device memory comes from torch's
    caching allocator; "hip" or None: the library's hipMalloc."""
    dev = w.device
    _need(edge_ptr, torch.int32, "edge_ptr", dev)
    _need(edge_vtx, torch.int32, "edge_vtx", dev)
    _need(w, torch.float64, "w", dev)
    E = edge_ptr.numel() - 1
    out = C.c_void_p()
    al = _allocator(dev, allocator)
    with torch.cuda.device(dev):
        check(lib().hgl_build_laplacian(N, E, edge_vtx.numel(), _ptr(edge_ptr), _ptr(edge_vtx), _ptr(w),
                                        C.byref(al.struct) if al else None, C.byref(out), _stream(dev)),
              "hgl_build_laplacian")
    return Handle(out, dev, al)


def build_laplacian_batched(vtx_offsets, edge_offsets, edge_ptr: torch.Tensor, edge_vtx: torch.Tensor,
                            w: torch.Tensor, allocator: str | None = "torch") -> Handle:
    dev = w.device
    _need(edge_ptr, torch.int32, "edge_ptr", dev)
    _need(edge_vtx, torch.int32, "edge_vtx", dev)
    _need(w, torch.float64, "w", dev)
    vo = np.ascontiguousarray(np.asarray(vtx_offsets, dtype=np.int32))
    eo = np.ascontiguousarray(np.asarray(edge_offsets, dtype=np.int32))
    G = vo.size - 1
    out = C.c_void_p()
    al = _allocator(dev, allocator)
    with torch.cuda.device(dev):
        check(lib().hgl_build_laplacian_batched(
            G, vo.ctypes.data_as(_lib.I32P), eo.ctypes.data_as(_lib.I32P), edge_vtx.numel(),
            _ptr(edge_ptr), _ptr(edge_vtx), _ptr(w), C.byref(al.struct) if al else None, C.byref(out),
            _stream(dev)),
            "hgl_build_laplacian_batched")
    return Handle(out, dev, al)


def set_weights(h: Handle, w: torch.Tensor) -> None:
    _need(w, torch.float64, "w", h.device)
    if w.numel() != h.E:
        raise ValueError("w must have E entries")
    with torch.cuda.device(h.device):
        check(lib().hgl_set_weights(h.ptr, _ptr(w), _stream(h.device)), "hgl_set_weights")


def get_operator(h: Handle) -> dict:
    dev = h.device
    dv = torch.empty(h.N, dtype=torch.float64, device=dev)
    s = torch.empty(h.N, dtype=torch.float64, device=dev)
    c = torch.empty(max(h.E, 1), dtype=torch.float64, device=dev)
    vp = torch.empty(h.N + 1, dtype=torch.int32, device=dev)
    ve = torch.empty(max(h.nnz, 1), dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        check(lib().hgl_get_operator(h.ptr, _ptr(dv), _ptr(s), _ptr(c), _ptr(vp), _ptr(ve),
                                     _stream(dev)), "hgl_get_operator")
    return {"dv": dv, "s": s, "c": c[:h.E], "vtx_ptr": vp, "vtx_edge": ve[:h.nnz]}


def apply(h: Handle, lam: float, P: torch.Tensor, out: torch.Tensor | None = None,
          noalloc: bool = False) -> torch.Tensor:
    """Q = (I + L/lam) P.  noalloc: through hgl_apply_noalloc (the library's fixed
    scratch instead of the handle's workspaces; `out` must then be given by callers
    that cannot allocate)."""
    if P.dtype not in (torch.float32, torch.float64):
        raise TypeError("P must be float32 or float64")
    _need(P, P.dtype, "P", h.device)
    ldp = _rows(P, "P")
    if P.shape[0] != h.N:
        raise ValueError("P must have N rows")
    Q = torch.empty_like(P, memory_format=torch.contiguous_format) if out is None else out
    ldq = _rows(Q, "out")
    dt = _lib.HGL_F64 if P.dtype == torch.float64 else _lib.HGL_F32
    fn = "hgl_apply_noalloc" if noalloc else "hgl_apply"
    with torch.cuda.device(h.device):
        check(getattr(lib(), fn)(h.ptr, float(lam), dt, _ptr(P), ldp, _ptr(Q), ldq, P.shape[1],
                                 _stream(h.device)), fn)
    return Q


def _cg(h: Handle, lams, Y: torch.Tensor, mode: str, tol: float, max_iter: int,
        x0: torch.Tensor | None, rr_period: int, chunk: int, batched: bool, graph: bool = False,
        out: torch.Tensor | None = None, tune: bool = False, wg: bool = False):
    m = MODES[mode]
    dtype = torch.float64 if m == _lib.HGL_CG_PLAIN_F64 else torch.float32
    _need(Y, dtype, "Y", h.device)
    ldy = _rows(Y, "Y")
    if Y.shape[0] != h.N:
        raise ValueError("Y must have N rows")
    k = Y.shape[1]
    if out is not None:
        _need(out, dtype, "out", h.device)
        if tuple(out.shape) != (h.N, k):
            raise ValueError("out must be N x k")
        _rows(out, "out")
        F = out
        if x0 is not None:
            F.copy_(x0)
    elif x0 is not None:
        _need(x0, dtype, "x0", h.device)
        F = x0.clone(memory_format=torch.contiguous_format)
    else:
        F = torch.empty((h.N, k), dtype=dtype, device=h.device)
    opts = CgOpts(m, float(tol), int(max_iter), 1 if x0 is not None else 0, int(rr_period), int(chunk),
                  1 if graph else 0, 1 if tune else 0)
    iters = np.zeros(h.G * k, dtype=np.int32)
    rel = np.zeros(h.G * k, dtype=np.float64)
    with torch.cuda.device(h.device):
        if batched:
            la = np.ascontiguousarray(np.asarray(lams, dtype=np.float64))
            if la.size != h.G:
                raise ValueError("need one lambda per graph")
            fn = lib().hgl_cg_solve_wg_batched if wg else lib().hgl_cg_solve_batched
            st = fn(h.ptr, la.ctypes.data_as(_lib.DP), C.byref(opts), _ptr(Y), ldy, _ptr(F), F.stride(0), k,
                    iters.ctypes.data_as(_lib.I32P), rel.ctypes.data_as(_lib.DP), _stream(h.device))
        else:
            fn = lib().hgl_cg_solve_wg if wg else lib().hgl_cg_solve
            st = fn(h.ptr, float(lams), C.byref(opts), _ptr(Y), ldy, _ptr(F), F.stride(0), k,
                    iters.ctypes.data_as(_lib.I32P), rel.ctypes.data_as(_lib.DP), _stream(h.device))
    check(st, "hgl_cg_solve_wg" if wg else "hgl_cg_solve")
    return F, iters.reshape(h.G, k), rel.reshape(h.G, k), st


def cg_solve(h: Handle, lam: float, Y: torch.Tensor, mode: str = "f32", tol: float = 1e-6,
             max_iter: int = 1000, x0: torch.Tensor | None = None, rr_period: int = 8, chunk: int = 0,
             graph: bool = False, out: torch.Tensor | None = None, tune: bool = False):
    """Solve (I + L/lam) F = Y.  Returns (F, iters[G,k], relres[G,k], status).
    graph: run the first chunk of iterations as a HIP graph, recorded once
    and replayed by later solves with the same arguments (pass the same
    `out` tensor to keep F's address, and so the graph, from call to call).
    tune: pick the kernels' column shape by timing (cached per handle)."""
    return _cg(h, lam, Y, mode, tol, max_iter, x0, rr_period, chunk, batched=False, graph=graph, out=out,
               tune=tune)


def cg_solve_wg(h: Handle, lam: float, Y: torch.Tensor, tol: float = 1e-6, max_iter: int = 1000,
                x0: torch.Tensor | None = None, out: torch.Tensor | None = None):
    """The latency path for small graphs: each (graph, column)'s whole FP32 solve runs in one
    workgroup of one launch (hgl_cg_solve_wg).  Returns (F, iters[G,k], relres[G,k], status) as
    cg_solve."""
    return _cg(h, lam, Y, "f32", tol, max_iter, x0, 0, 0, batched=False, out=out, wg=True)


def cg_solve_wg_batched(h: Handle, lams, Y: torch.Tensor, tol: float = 1e-6, max_iter: int = 1000,
                        x0: torch.Tensor | None = None, out: torch.Tensor | None = None):
    """cg_solve_wg with one lambda per graph of a batched handle (hgl_cg_solve_wg_batched)."""
    return _cg(h, lams, Y, "f32", tol, max_iter, x0, 0, 0, batched=True, out=out, wg=True)


def cg_solve_batched(h: Handle, lams, Y: torch.Tensor, mode: str = "f32", tol: float = 1e-6,
                     max_iter: int = 1000, x0: torch.Tensor | None = None, rr_period: int = 8,
                     chunk: int = 0, graph: bool = False, out: torch.Tensor | None = None,
                     tune: bool = False):
    """One lambda per graph of a batched handle (graph, out, tune: as for cg_solve)."""
    return _cg(h, lams, Y, mode, tol, max_iter, x0, rr_period, chunk, batched=True, graph=graph, out=out,
               tune=tune)


SKETCH = {"bf16": _lib.HGL_SKETCH_BF16, "f64": _lib.HGL_SKETCH_F64}
SCHEME = {"subspace": _lib.HGL_RSVD_SUBSPACE, "power": _lib.HGL_RSVD_POWER}


def _offsets(offsets) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(offsets, dtype=np.int32))


def _rsvd_opts(k, p, q, sketch, seed, refine_tol=1e-6, max_refine=500, chunk=0, scheme="subspace"):
    return _lib.RsvdOpts(int(k), int(p), int(q), SKETCH[sketch], int(seed), float(refine_tol),
                         int(max_refine), int(chunk), SCHEME[scheme])


def _omega_ptr(h: Handle, omega, l: int):
    if omega is None:
        return C.c_void_p(0)
    _need(omega, torch.int16, "omega (bf16 bit patterns as int16)", h.device)
    if omega.shape != (h.N, l) or not omega.is_contiguous():
        raise ValueError(f"omega must be a contiguous ({h.N}, {l}) int16 tensor")
    return _ptr(omega)


def philox4x32_10(ctr: torch.Tensor, key: int) -> torch.Tensor:
    """Raw Philox4x32-10 words of counters ctr [n, 4] (int32 tensor holding the uint32
    bit patterns) under a 64-bit key; returns [n, 4] int32 bit patterns."""
    _need(ctr, torch.int32, "ctr")
    if ctr.dim() != 2 or ctr.shape[1] != 4 or not ctr.is_contiguous():
        raise ValueError("ctr must be a contiguous (n, 4) int32 tensor")
    out = torch.empty_like(ctr)
    with torch.cuda.device(ctr.device):
        check(lib().hgl_philox4x32_10(ctr.shape[0], _ptr(ctr), C.c_uint64(key), _ptr(out), _stream(ctr.device)),
              "hgl_philox4x32_10")
    return out


def block_rsvd(h: Handle, offsets, k: int, p: int, q: int, sketch: str = "bf16", omega=None, seed: int = 0,
               scheme: str = "subspace"):
    """Algorithm 1 on every diagonal block ("power": with the sketch of eq. 10 in place of its
    steps 2-3).  Returns (U [N,k] float32, sigma [n_blocks,k] float64)."""
    off = _offsets(offsets)
    nb = off.size - 1
    U = torch.empty((h.N, k), dtype=torch.float32, device=h.device)
    sig = torch.empty((nb, k), dtype=torch.float64, device=h.device)
    opts = _rsvd_opts(k, p, q, sketch, seed, scheme=scheme)
    with torch.cuda.device(h.device):
        check(lib().hgl_block_rsvd(h.ptr, nb, off.ctypes.data_as(_lib.I32P), C.byref(opts),
                                   _omega_ptr(h, omega, k + p), _ptr(U), _ptr(sig), _stream(h.device)),
              "hgl_block_rsvd")
    return U, sig


def block_rsvd_invert(h: Handle, lam: float, offsets, Y: torch.Tensor, k: int, p: int, q: int,
                      sketch: str = "bf16", omega=None, seed: int = 0, refine_tol: float = 5e-7,
                      max_refine: int = 500, chunk: int = 0, scheme: str = "subspace"):
    """Block-inverse start + preconditioned CG.  Returns (F, iters, relres, sigma, status)."""
    off = _offsets(offsets)
    nb = off.size - 1
    _need(Y, torch.float32, "Y", h.device)
    ldy = _rows(Y, "Y")
    nrhs = Y.shape[1]
    F = torch.empty((h.N, nrhs), dtype=torch.float32, device=h.device)
    sig = torch.empty((nb, k), dtype=torch.float64, device=h.device)
    iters = np.zeros(nrhs, dtype=np.int32)
    rel = np.zeros(nrhs, dtype=np.float64)
    opts = _rsvd_opts(k, p, q, sketch, seed, refine_tol, max_refine, chunk, scheme)
    with torch.cuda.device(h.device):
        st = lib().hgl_block_rsvd_invert(h.ptr, float(lam), nb, off.ctypes.data_as(_lib.I32P), C.byref(opts),
                                         _omega_ptr(h, omega, k + p), _ptr(Y), ldy, _ptr(F), F.stride(0), nrhs,
                                         _ptr(sig), iters.ctypes.data_as(_lib.I32P), rel.ctypes.data_as(_lib.DP),
                                         _stream(h.device))
    check(st, "hgl_block_rsvd_invert")
    return F, iters, rel, sig, st


def block_schur_plan(offsets, min_block: int) -> dict:
    """The execution plan of the Schur-complement block inverse (host only):
    numpy arrays tasks [n x 13], leaves [n x 5], phases [n x 5], tiles
    [n x 2], moff [n_blocks] and the counts (see hgl_block_schur_plan)."""
    off = _offsets(offsets)
    nb = off.size - 1
    cnt = np.zeros(7, dtype=np.int64)
    i64 = lambda a: a.ctypes.data_as(_lib.I64P)
    check(lib().hgl_block_schur_plan(nb, off.ctypes.data_as(_lib.I32P), int(min_block), i64(cnt), None, None,
                                      None, None, None), "hgl_block_schur_plan")
    tasks = np.zeros((int(cnt[0]), 13), dtype=np.int64)
    leaves = np.zeros((int(cnt[1]), 5), dtype=np.int64)
    phases = np.zeros((int(cnt[2]), 5), dtype=np.int32)
    tiles = np.zeros((int(cnt[5]), 2), dtype=np.int64)
    moff = np.zeros(nb, dtype=np.int64)
    check(lib().hgl_block_schur_plan(nb, off.ctypes.data_as(_lib.I32P), int(min_block), i64(cnt), i64(tasks),
                                      i64(leaves), phases.ctypes.data_as(_lib.I32P), i64(tiles), i64(moff)),
          "hgl_block_schur_plan")
    return {"tasks": tasks, "leaves": leaves, "phases": phases, "tiles": tiles, "moff": moff,
            "arena_elems": int(cnt[3]), "inv_elems": int(cnt[4]), "flops": int(cnt[6])}


def block_schur_inverse(h: Handle, lam: float, offsets, min_block: int = 50):
    """Inverses of the diagonal blocks (eqs. 12-15): a list of n_b x n_b FP32
    device tensors (views of one packed buffer) and the products' flops."""
    off = _offsets(offsets)
    nb = off.size - 1
    sizes = np.diff(off).astype(np.int64)
    buf = torch.empty(int((sizes * sizes).sum()), dtype=torch.float32, device=h.device)
    flops = C.c_double(0.0)
    with torch.cuda.device(h.device):
        st = lib().hgl_block_schur_inverse(h.ptr, float(lam), nb, off.ctypes.data_as(_lib.I32P), int(min_block),
                                           _ptr(buf), C.byref(flops), _stream(h.device))
    check(st, "hgl_block_schur_inverse")
    out, at = [], 0
    for n in sizes.tolist():
        out.append(buf[at:at + n * n].view(n, n))
        at += n * n
    return out, flops.value


def block_schur_invert(h: Handle, lam: float, offsets, Y: torch.Tensor, min_block: int = 50,
                       refine_tol: float = 5e-7, max_refine: int = 500, chunk: int = 0):
    """Block-inverse start + preconditioned CG with the Schur-complement block
    inverse.  Returns (F, iters, relres, status)."""
    off = _offsets(offsets)
    nb = off.size - 1
    _need(Y, torch.float32, "Y", h.device)
    ldy = _rows(Y, "Y")
    nrhs = Y.shape[1]
    F = torch.empty((h.N, nrhs), dtype=torch.float32, device=h.device)
    iters = np.zeros(nrhs, dtype=np.int32)
    rel = np.zeros(nrhs, dtype=np.float64)
    with torch.cuda.device(h.device):
        st = lib().hgl_block_schur_invert(h.ptr, float(lam), nb, off.ctypes.data_as(_lib.I32P), int(min_block),
                                          float(refine_tol), int(max_refine), int(chunk), _ptr(Y), ldy, _ptr(F),
                                          F.stride(0), nrhs, iters.ctypes.data_as(_lib.I32P),
                                          rel.ctypes.data_as(_lib.DP), _stream(h.device))
    check(st, "hgl_block_schur_invert")
    return F, iters, rel, st


def measure_peaks(device, copy_bytes: int = 1 << 30, reps: int = 10) -> dict:
    """Achievable HBM GB/s (a copy of copy_bytes between two buffers, each
    larger than the last-level cache; 2 * copy_bytes moved per copy) and
    achievable dense BF16 MFMA TFLOP/s, each the best of `reps` timed calls."""
    dev = torch.device(device)
    src = torch.empty(copy_bytes, dtype=torch.uint8, device=dev)
    src.fill_(1)
    dst = torch.empty_like(src)
    wg, iters = 256 * 8, 1000
    out = torch.zeros(wg, dtype=torch.float32, device=dev)
    st = _stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def best(fn):
        fn()
        ms = float("inf")
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ms = min(ms, e0.elapsed_time(e1))
        return ms

    with torch.cuda.device(dev):
        t_copy = best(lambda: check(lib().hgl_peak_copy(_ptr(src), _ptr(dst), copy_bytes, st), "hgl_peak_copy"))
        t_mfma = best(lambda: check(lib().hgl_peak_mfma_bf16(_ptr(out), wg, iters, st), "hgl_peak_mfma_bf16"))
    if not torch.equal(src[:4096], dst[:4096]):
        raise RuntimeError("hgl_peak_copy produced a wrong copy")
    return {"hbm_gbs": round(2 * copy_bytes / (t_copy * 1e-3) / 1e9, 1),
            "bf16_mfma_tflops": round(524288.0 * wg * iters / (t_mfma * 1e-3) / 1e12, 1),
            "copy_bytes": copy_bytes}


def sketch_gaussian(rows: int, l: int, seed: int, device) -> torch.Tensor:
    """rows x l Philox4x32-10 standard normals rounded to BF16 (bit patterns, int16 tensor)."""
    out = torch.empty((rows, l), dtype=torch.int16, device=device)
    with torch.cuda.device(device):
        check(lib().hgl_sketch_gaussian(int(rows), int(l), int(seed), _ptr(out), _stream(torch.device(device))),
              "hgl_sketch_gaussian")
    return out


def weight_grad(h: Handle, lam: float, F: torch.Tensor, G: torch.Tensor | None = None,
                Y: torch.Tensor | None = None, mu: float = 0.0, mode: str = "f32", tol: float = 1e-6,
                max_iter: int = 1000, want_z: bool = False):
    """d/dw of a loss through the solve (G given: upstream dl/dF) or of the
    objective tr(F'LF) + lam||F-Y||^2 + mu||w||^2 (G None).
    Returns (grad_w [E] float64, Z or None, adjoint iters, adjoint relres,
    adjoint status: 0, or 1 when the adjoint solve stopped at max_iter)."""
    m = MODES[mode]
    dtype = torch.float64 if m == _lib.HGL_CG_PLAIN_F64 else torch.float32
    _need(F, dtype, "F", h.device)
    k = F.shape[1]
    ldf = _rows(F, "F")
    ldg = ldy = 0
    if G is not None:
        _need(G, dtype, "G", h.device)
        ldg = _rows(G, "G")
    if Y is not None:
        _need(Y, dtype, "Y", h.device)
        ldy = _rows(Y, "Y")
    grad = torch.empty(h.E, dtype=torch.float64, device=h.device)
    Z = torch.empty((h.N, k), dtype=dtype, device=h.device) if want_z else None
    opts = CgOpts(m, float(tol), int(max_iter), 0, 0, 0, 0, 0)
    iters = np.zeros(k, dtype=np.int32)
    rel = np.zeros(k, dtype=np.float64)
    with torch.cuda.device(h.device):
        st = lib().hgl_weight_grad(h.ptr, float(lam), float(mu), _ptr(F), ldf, _ptr(G), ldg, _ptr(Y), ldy, k,
                                   C.byref(opts), _ptr(grad), _ptr(Z), k if Z is not None else 0,
                                   iters.ctypes.data_as(_lib.I32P), rel.ctypes.data_as(_lib.DP),
                                   _stream(h.device))
    check(st, "hgl_weight_grad")
    return grad, Z, iters, rel, st


def project_simplex(v: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    _need(v, torch.float64, "v")
    w = torch.empty_like(v) if out is None else out
    with torch.cuda.device(v.device):
        check(lib().hgl_project_simplex(_ptr(v), _ptr(w), v.numel(), _stream(v.device)), "hgl_project_simplex")
    return w


def projected_gradient_step(w: torch.Tensor, g: torch.Tensor, eta: float | None = None,
                            out: torch.Tensor | None = None, eta_out: torch.Tensor | None = None):
    """w_out = Proj_simplex(w - eta g) (hgl_projected_gradient_step).  eta None: the
    library sets the step from this gradient (0.5 max|w| / max|g - mean g|).  Returns
    (w_out, eta as a device FP64 tensor of one element)."""
    _need(w, torch.float64, "w")
    _need(g, torch.float64, "g", w.device)
    if g.numel() != w.numel():
        raise ValueError("w and g must have the same length")
    wo = torch.empty_like(w) if out is None else out
    ed = torch.empty(1, dtype=torch.float64, device=w.device) if eta_out is None else eta_out
    with torch.cuda.device(w.device):
        check(lib().hgl_projected_gradient_step(_ptr(w), _ptr(g), 0.0 if eta is None else float(eta), w.numel(),
                                                _ptr(wo), _ptr(ed), _stream(w.device)),
              "hgl_projected_gradient_step")
    return wo, ed


def active_set_step(w: torch.Tensor, g: torch.Tensor, mu: float, out: torch.Tensor | None = None,
                    direction: bool = False):
    """One steepest-descent step on the Lagrangian of eq. 5 (active-set
    rule, ratio-test step).  Returns (w_new, info dict, d or None)."""
    _need(w, torch.float64, "w")
    _need(g, torch.float64, "g", w.device)
    if w.numel() != g.numel():
        raise ValueError("w and g differ in length")
    w_new = torch.empty_like(w) if out is None else out
    d = torch.empty_like(w) if direction else None
    info_dev = torch.empty(4, dtype=torch.float64, device=w.device)
    info = np.zeros(4, dtype=np.float64)
    with torch.cuda.device(w.device):
        check(lib().hgl_active_set_step(_ptr(w), _ptr(g), float(mu), w.numel(), _ptr(w_new),
                                        _ptr(d) if d is not None else None, _ptr(info_dev),
                                        info.ctypes.data_as(_lib.DP), _stream(w.device)), "hgl_active_set_step")
    return w_new, {"nu": float(info[0]), "mu_eff": float(info[1]), "released": int(info[2]),
                   "active": int(info[3])}, d


PROFILE_KINDS = {0: "edge_gather", 1: "vertex_gather", 2: "cg_update", 3: "cg_direction",
                 4: "reduce", 5: "resid_edge_gather", 6: "resid_vertex_gather", 7: "start",
                 8: "precond", 9: "dense_gemm", 10: "cholqr", 11: "eig", 12: "extract", 13: "grad",
                 14: "hub_row_finish", 15: "schur_leaf"}


def profile(h: Handle, enable: bool, kinds=None, every: int = 1) -> None:
    """Reset the kernel-timing counters of h and switch event timing on/off.
    `kinds` (names or numbers of PROFILE_KINDS) limits the stamped launches
    to those kernels, and `every` > 1 stamps only every n-th launch of each;
    kinds=None stamps every launch."""
    mask = 1
    if enable and kinds is not None:
        names = {v: k for k, v in PROFILE_KINDS.items()}
        mask = 0
        for kd in kinds:
            mask |= 1 << (names[kd] if isinstance(kd, str) else int(kd))
        if mask == 1:  # kind 0 alone: 1 means "all", so add an unused bit
            mask |= 1 << 15
        mask |= (max(1, min(255, int(every))) & 0xFF) << 16
    check(lib().hgl_profile(h.ptr, mask if enable else 0), "hgl_profile")


def profile_read(h: Handle) -> dict:
    """{kind name: (launches, total ms)} recorded since the last profile(h, ...)."""
    out = {}
    for kind, name in PROFILE_KINDS.items():
        n = C.c_int64()
        ms = C.c_double()
        check(lib().hgl_profile_read(h.ptr, kind, C.byref(n), C.byref(ms)), "hgl_profile_read")
        out[name] = (n.value, ms.value)
    return out
