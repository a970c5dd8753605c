"""Seeded synthetic inputs shaped like social-tagging hypergraphs.

This module only draws random structure and values; it holds none of the
method's arithmetic (no degrees, no Laplacian, no solves).  Both the FP64
oracle (through the tests) and the HIP path (through the tests and the
benchmark) take their inputs from here.

The paper's Flickr hypergraph is not available, so these generators stand in
for it (section 4 of the paper describes images, users, groups, geo-tags and
tags joined by hyperedges).  Two families:

* G1 -- every hyperedge is a uniform random vertex set with size uniform in
  [smin, smax].
* G2 -- hyperedge sizes follow a power law P(s) ~ s^-alpha truncated to
  [smin, smax]; member vertices are drawn without replacement with probability
  proportional to rank^-zipf (rank given by a seeded random permutation), which
  produces hub vertices and many isolated vertices, like popular tags/users.

Every hyperedge is returned as a strictly increasing list of vertex ids in an
edge-major CSR (``edge_ptr[E+1]``, ``edge_vtx[nnz]``, int32).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 1908_08281


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# hyperedge structure
# --------------------------------------------------------------------------

def _pack(members: list[np.ndarray]) -> tuple[np.ndarray, np.ndarray]:
    sizes = np.fromiter((len(m) for m in members), dtype=np.int64, count=len(members))
    edge_ptr = np.zeros(len(members) + 1, dtype=np.int64)
    np.cumsum(sizes, out=edge_ptr[1:])
    edge_vtx = np.concatenate(members) if members else np.zeros(0, np.int64)
    return edge_ptr.astype(np.int32), edge_vtx.astype(np.int32)


def uniform_hyperedges(N: int, E: int, smin: int, smax: int, seed: int):
    """G1: sizes ~ U{smin..smax}; members uniform without replacement."""
    rng = rng_for(seed)
    smax = min(smax, N)
    sizes = rng.integers(smin, smax + 1, size=E)
    members = []
    for s in sizes:
        # draw-and-reject keeps this O(s) per edge instead of O(N)
        got = np.unique(rng.integers(0, N, size=int(s)))
        while got.size < s:
            extra = rng.integers(0, N, size=int(s - got.size))
            got = np.unique(np.concatenate([got, extra]))
        members.append(got.astype(np.int64))
    return _pack(members)


def truncated_powerlaw_sizes(E: int, alpha: float, smin: int, smax: int,
                             rng: np.random.Generator) -> np.ndarray:
    support = np.arange(smin, smax + 1)
    p = support.astype(np.float64) ** (-alpha)
    p /= p.sum()
    return rng.choice(support, size=E, p=p)


def powerlaw_hyperedges(N: int, E: int, alpha: float, smin: int, smax: int,
                        zipf: float, seed: int):
    """G2: truncated power-law sizes, Zipf vertex popularity, no repeats."""
    rng = rng_for(seed)
    smax = min(smax, N)
    sizes = truncated_powerlaw_sizes(E, alpha, smin, smax, rng)
    rank = rng.permutation(N) + 1                  # rank of vertex v
    pv = rank.astype(np.float64) ** (-zipf)
    cdf = np.cumsum(pv)
    cdf /= cdf[-1]
    total = int(sizes.sum())
    draws = np.minimum(np.searchsorted(cdf, rng.random(total), side="right"), N - 1)
    members = []
    pos = 0
    for s in sizes:
        s = int(s)
        cand = draws[pos:pos + s]
        pos += s
        got = np.unique(cand)
        while got.size < s:
            # successive sampling without replacement: redraw the repeats
            extra = np.minimum(np.searchsorted(cdf, rng.random(s - got.size), side="right"), N - 1)
            got = np.unique(np.concatenate([got, extra]))
        members.append(got.astype(np.int64))
    return _pack(members)


def explicit_hyperedges(edges: list[list[int]]):
    """Edge-major CSR from explicit vertex lists (sorted, duplicates kept as given)."""
    return _pack([np.sort(np.asarray(e, dtype=np.int64)) for e in edges])


# --------------------------------------------------------------------------
# weights, right-hand sides, blocks, sketch matrices
# --------------------------------------------------------------------------

def uniform_weights(E: int) -> np.ndarray:
    return np.full(E, 1.0 / E, dtype=np.float64)


def dirichlet_weights(E: int, seed: int, alpha: float = 1.0) -> np.ndarray:
    return rng_for(seed).dirichlet(np.full(E, alpha))


def binary_rhs(N: int, k: int, density: float, seed: int) -> np.ndarray:
    """N x k float64 matrix with exactly round(density*N*k) ones, uniformly placed."""
    rng = rng_for(seed)
    count = int(round(density * N * k))
    Y = np.zeros(N * k, dtype=np.float64)
    Y[rng.choice(N * k, size=count, replace=False)] = 1.0
    return Y.reshape(N, k)


def block_sizes(n_blocks: int, lo: int, hi: int, seed: int) -> np.ndarray:
    return rng_for(seed).integers(lo, hi + 1, size=n_blocks)


def block_offsets(sizes: np.ndarray) -> np.ndarray:
    off = np.zeros(len(sizes) + 1, dtype=np.int32)
    np.cumsum(sizes, out=off[1:])
    return off


def bf16_round(x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Round float64 values to bfloat16 (nearest, ties to even).

    Returns (bits uint16, values float64).  Rounding goes through float32
    first; for N(0,1) draws the double rounding never changes the result in
    practice, and both sides receive the same stored bits anyway.
    """
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) >> 16
    bits = u.astype(np.uint16)
    vals = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return bits, vals


def gaussian_sketch(rows: int, l: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Row-major rows x l Gaussian sketch, rounded to bf16: (bits, values)."""
    g = rng_for(seed).standard_normal((rows, l))
    return bf16_round(g)


# --------------------------------------------------------------------------
# workload recipes (sizes and distributions of the measured configurations)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Problem:
    N: int
    E: int
    edge_ptr: np.ndarray
    edge_vtx: np.ndarray
    w: np.ndarray
    lam: float
    Y: np.ndarray
    name: str = ""
    tol: float = 1e-6
    # batched problems: segment offsets over vertices and edges
    vtx_offsets: np.ndarray | None = None
    edge_offsets: np.ndarray | None = None
    lams: np.ndarray | None = None
    # tessellation
    blocks: np.ndarray | None = None

    @property
    def nnz(self) -> int:
        return int(self.edge_ptr[-1])


def small_plain(seed_offset: int = 0, N: int = 2000, E: int = 1500, k: int = 50) -> Problem:
    """Plain method, small: G1 sizes U{2..20}, w = 1/E, lambda = 1, Y at 5%, FP64 to 1e-10."""
    s = BASE_SEED + 0 + 1000 * seed_offset
    ep, ev = uniform_hyperedges(N, E, 2, 20, s)
    return Problem(N, E, ep, ev, uniform_weights(E), 1.0,
                   binary_rhs(N, k, 0.05, s + 1), name=f"g1_N{N}_E{E}_k{k}", tol=1e-10)


def multi_rhs(seed_offset: int = 0, N: int = 50_000, E: int = 40_000, k: int = 200,
              smax: int = 200) -> Problem:
    """Multi-RHS FP32: G2 (alpha 2.1, sizes [2,200], Zipf 1.1), Dirichlet(1) w, lambda 0.5, Y at 2%."""
    s = BASE_SEED + 1 + 1000 * seed_offset
    ep, ev = powerlaw_hyperedges(N, E, 2.1, 2, smax, 1.1, s)
    return Problem(N, E, ep, ev, dirichlet_weights(E, s + 2), 0.5,
                   binary_rhs(N, k, 0.02, s + 1), name=f"g2_N{N}_E{E}_k{k}", tol=1e-6)


def single_query(seed_offset: int = 0, N: int = 5867, E: int = 4694, k: int = 1292,
                 smax: int = 200) -> Problem:
    """The paper's query shape: one RHS per test image (1292 images) on a graph of
    m = 5867 vertices (section 4, Table 1); G2 structure (alpha 2.1, sizes
    [2,200], Zipf 1.1) with E = 0.8 N, Dirichlet(1) w, lambda 0.5, Y at 2%."""
    s = BASE_SEED + 6 + 1000 * seed_offset
    ep, ev = powerlaw_hyperedges(N, E, 2.1, 2, smax, 1.1, s)
    return Problem(N, E, ep, ev, dirichlet_weights(E, s + 2), 0.5,
                   binary_rhs(N, k, 0.02, s + 1), name=f"g2_N{N}_E{E}_k{k}", tol=1e-6)


def tessellated(seed_offset: int = 0, n_blocks: int = 50, lo: int = 500, hi: int = 1500,
                k_rhs: int = 50) -> Problem:
    """Block rSVD workload: G1 at N = sum of block sizes, E = 0.75 N, w = 1/E, lambda 1, Y at 5%."""
    s = BASE_SEED + 2 + 1000 * seed_offset
    sizes = block_sizes(n_blocks, lo, hi, s + 3)
    N = int(sizes.sum())
    E = int(round(0.75 * N))
    ep, ev = uniform_hyperedges(N, E, 2, 20, s)
    return Problem(N, E, ep, ev, uniform_weights(E), 1.0,
                   binary_rhs(N, k_rhs, 0.05, s + 1), name=f"tess_{n_blocks}b_N{N}",
                   tol=1e-6, blocks=block_offsets(sizes))


def weight_learning(seed_offset: int = 0, N: int = 100_000, E: int = 80_000, k: int = 500) -> Problem:
    """Differentiation workload: G1, w0 = 1/E, lambda 1, Y at 5%, k tag columns."""
    s = BASE_SEED + 3 + 1000 * seed_offset
    ep, ev = uniform_hyperedges(N, E, 2, 20, s)
    return Problem(N, E, ep, ev, uniform_weights(E), 1.0,
                   binary_rhs(N, k, 0.05, s + 1), name=f"g1_N{N}_E{E}_k{k}", tol=1e-6)


def batch_of_graphs(seed_offset: int = 0, G: int = 64, nlo: int = 2000, nhi: int = 30_000,
                    k: int = 100, smax: int = 100) -> Problem:
    """Batching: G independent G2 hypergraphs, N_g ~ U[nlo,nhi], E_g = 0.8 N_g, k RHS at 3%.

    Returned as one disjoint-union hypergraph with segment offsets over
    vertices and edges (vertex ids are global)."""
    s = BASE_SEED + 4 + 1000 * seed_offset
    rng = rng_for(s)
    Ns = rng.integers(nlo, nhi + 1, size=G)
    ptrs, vtxs, ws, Ys = [], [], [], []
    voff = np.zeros(G + 1, np.int64)
    eoff = np.zeros(G + 1, np.int64)
    nnz_off = 0
    for g in range(G):
        Ng = int(Ns[g])
        Eg = int(round(0.8 * Ng))
        ep, ev = powerlaw_hyperedges(Ng, Eg, 2.1, 2, smax, 1.1, s + 10 + 3 * g)
        ptrs.append(ep[:-1].astype(np.int64) + nnz_off)
        vtxs.append(ev.astype(np.int64) + voff[g])
        nnz_off += int(ep[-1])
        ws.append(dirichlet_weights(Eg, s + 11 + 3 * g))
        Ys.append(binary_rhs(Ng, k, 0.03, s + 12 + 3 * g))
        voff[g + 1] = voff[g] + Ng
        eoff[g + 1] = eoff[g] + Eg
    edge_ptr = np.concatenate(ptrs + [np.array([nnz_off])]).astype(np.int32)
    edge_vtx = np.concatenate(vtxs).astype(np.int32)
    return Problem(int(voff[-1]), int(eoff[-1]), edge_ptr, edge_vtx, np.concatenate(ws), 0.5,
                   np.concatenate(Ys, axis=0), name=f"batch{G}_N{int(voff[-1])}_k{k}", tol=1e-6,
                   vtx_offsets=voff.astype(np.int32), edge_offsets=eoff.astype(np.int32),
                   lams=np.full(G, 0.5))


def random_small(seed: int, N: int, E: int, smin: int = 1, smax: int = 6,
                 k: int = 3, lam: float = 0.7, dirichlet: bool = True) -> Problem:
    """Tiny random problem for property tests (isolated vertices allowed)."""
    ep, ev = uniform_hyperedges(N, E, smin, min(smax, N), seed)
    w = dirichlet_weights(E, seed + 1) if dirichlet else uniform_weights(E)
    Y = rng_for(seed + 2).standard_normal((N, k))
    return Problem(N, E, ep, ev, w, lam, Y, name=f"tiny_{seed}")
