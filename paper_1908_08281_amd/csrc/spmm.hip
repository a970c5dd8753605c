// Matrix-free application of M = I + L/lambda = (1 + 1/lambda) I - (1/lambda) A
// with A = S H C H' S (paper, section 2, eq. 1), S = diag(delta(v)^-1/2),
// C = diag(w_e/delta(e)).  Two gathers, no atomics:
//   Z = C H' S P        edge-major:   Z[e,:] = c_e * sum_{v in e} s_v P[v,:]
//   Q = a P - b S H Z   vertex-major: Q[v,:] = a P[v,:] - b s_v sum_{e ni v} Z[e,:]
// with a = 1 + 1/lambda, b = 1/lambda.  Rows of P, Z, Q are k-wide and
// contiguous; a group of GL lanes owns one row and each lane moves V
// consecutive elements per access, so every gathered row is one coalesced
// 16-byte-per-lane transaction.  Vertex rows with more than kLongRow incident
// hyperedges (hubs) are split into chunks processed by separate workgroups;
// a second launch sums each row's chunk partials in a fixed order and
// finishes the row, so results do not depend on scheduling.
#include "kernels.h"

namespace hgl {

// ------------------------------------------------------------ edge gather --

// acc += sum_{j in [jb, je)} s[idx[j]] P[idx[j], col .. col+V-1], kGather
// member rows in flight (masked past je), summed in a fixed order.
template <int V, class TIn, class TAcc>
__device__ __forceinline__ void gather_scaled(const TIn* __restrict__ P, int64_t ldp, const TAcc* __restrict__ s,
                                              const int32_t* __restrict__ idx, int jb, int je, int col,
                                              TAcc (&acc)[V]) {
  for (int j = jb; j < je; j += kGather) {
    int v[kGather];
#pragma unroll
    for (int u = 0; u < kGather; ++u) v[u] = j + u < je ? idx[j + u] : -1;
    TAcc sv[kGather];
    TIn x[kGather][V];
#pragma unroll
    for (int u = 0; u < kGather; ++u) {
      if (v[u] >= 0) {
        sv[u] = s[v[u]];
        load_row<V>(P + int64_t(v[u]) * ldp + col, x[u]);
      } else {
        sv[u] = TAcc(0);
#pragma unroll
        for (int i = 0; i < V; ++i) x[u][i] = TIn(0);
      }
    }
#pragma unroll
    for (int u = 0; u < kGather; ++u)
#pragma unroll
      for (int i = 0; i < V; ++i) acc[i] += sv[u] * TAcc(x[u][i]);
  }
}

// Workgroups [0, n_etiles) take one edge tile each (kEdgeTile consecutive
// hyperedges of one graph, offsets and member ids staged in LDS), one
// hyperedge per lane group at a time, skipping the long ones (more than
// kLongEdge members); each further workgroup takes one long hyperedge, its
// groups summing contiguous shares of the members, combined by a fixed-order
// block reduction.  DOT: the workgroup also writes the FP64 partial
// sum_e c_e |u_e|^2 per column (u_e = (H' S P)_e, so Z_e = c_e u_e) to
// part[slot][k], slot = tile, or n_etiles + long-hyperedge index: the
// hyperedge half of p'Mp (eq. 1).
struct EdgeArgs {
  int32_t n_etiles;
  const int32_t* etile_e0;
  const int32_t* etile_e1;
  const int32_t* edge_ptr;
  const int32_t* edge_vtx;
  const int32_t* long_edge;
};

template <class TIn, class TAcc, int GL, int V, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmm_edge(
    EdgeArgs ea, const TAcc* __restrict__ s, const TAcc* __restrict__ c, const TIn* __restrict__ P, int64_t ldp,
    TAcc* __restrict__ Z, int64_t ldz, double* __restrict__ part, int k, Gate gate) {
  if (gate.skip()) return;
  constexpr int GPB = kBlock / GL, W = GL * V;
  const int grp = threadIdx.x / GL, lane = threadIdx.x % GL;
  const int col = blockIdx.y * W + lane * V;
  const int cc = blockIdx.y * W + threadIdx.x;
  __shared__ double lds_raw[4 * W];  // block reductions (either branch)
  if (int(blockIdx.x) < ea.n_etiles) {
    const int t = blockIdx.x;
    const int e0 = ea.etile_e0[t], e1 = ea.etile_e1[t];
    __shared__ int32_t s_ptr[kEdgeTile + 1];
    __shared__ int32_t s_idx[kEdgeStageIdx];
    const int ne = e1 - e0;
    for (int i = threadIdx.x; i <= ne; i += kBlock) s_ptr[i] = ea.edge_ptr[e0 + i];
    __syncthreads();
    const int base = s_ptr[0];
    const int staged = min(s_ptr[ne] - base, kEdgeStageIdx);
    for (int i = threadIdx.x; i < staged; i += kBlock) s_idx[i] = ea.edge_vtx[base + i];
    __syncthreads();
    double dot[V];
#pragma unroll
    for (int i = 0; i < V; ++i) dot[i] = 0.0;
    if (col < k) {
      for (int e = e0 + grp; e < e1; e += GPB) {
        const int b = s_ptr[e - e0], en = s_ptr[e - e0 + 1];
        if (en - b > kLongEdge) continue;
        TAcc acc[V];
#pragma unroll
        for (int i = 0; i < V; ++i) acc[i] = TAcc(0);
        if (en - base <= staged)
          gather_scaled<V>(P, ldp, s, s_idx, b - base, en - base, col, acc);
        else
          gather_scaled<V>(P, ldp, s, ea.edge_vtx, b, en, col, acc);
        const TAcc ce = c[e];
#pragma unroll
        for (int i = 0; i < V; ++i) {
          const TAcc z = ce * acc[i];
          if constexpr (DOT) dot[i] += double(acc[i]) * double(z);
          acc[i] = z;
        }
        store_row<V>(Z + int64_t(e) * ldz + col, acc);
      }
    }
    if constexpr (DOT) {
      const double tot = block_colsum<GL, V>(dot, lds_raw);
      if (threadIdx.x < W && cc < k) part[int64_t(t) * k + cc] = tot;
    }
    return;
  }
  TAcc* lds = reinterpret_cast<TAcc*>(lds_raw);
  const int li = blockIdx.x - ea.n_etiles;
  const int e = ea.long_edge[li];
  const int b = ea.edge_ptr[e], en = ea.edge_ptr[e + 1];
  TAcc acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) acc[i] = TAcc(0);
  if (col < k) {
    const int per = (en - b + GPB - 1) / GPB;
    const int jb = b + grp * per;
    gather_scaled<V>(P, ldp, s, ea.edge_vtx, jb, min(jb + per, en), col, acc);
  }
  const TAcc sum = block_colsum<GL, V>(acc, lds);
  if (threadIdx.x < W && cc < k) {
    const TAcc z = c[e] * sum;
    Z[int64_t(e) * ldz + cc] = z;
    if constexpr (DOT) part[int64_t(ea.n_etiles + li) * k + cc] = double(sum) * double(z);
  }
}

template <class TIn, class TAcc>
int launch_spmm_edge(const hgl_handle* h, const TIn* P, int64_t ldp, TAcc* Z, int64_t ldz, int k,
                     const ColShape& cs, Gate gate, hipStream_t st, double* part) {
  if (h->E == 0) return HGL_OK;
  const TAcc* s;
  const TAcc* c;
  if constexpr (sizeof(TAcc) == 8) {
    s = h->s64;
    c = h->c64;
  } else {
    s = h->s32;
    c = h->c32;
  }
  const EdgeArgs ea{h->n_etiles, h->etile_e0, h->etile_e1, h->edge_ptr, h->edge_vtx, h->long_edge};
  return HGL_DISPATCH_SHAPE(cs, sizeof(TAcc), {
    dim3 grid(h->n_etiles + h->n_long_edge, cs.slabs);
    if (part)
      launch(h, -1, k_spmm_edge<TIn, TAcc, GL, V, true>, grid, dim3(kBlock), 0, st, ea, s, c, P, ldp, Z, ldz,
             part, k, gate);
    else
      launch(h, -1, k_spmm_edge<TIn, TAcc, GL, V, false>, grid, dim3(kBlock), 0, st, ea, s, c, P, ldp, Z, ldz,
             part, k, gate);
    HGL_HIP(hipGetLastError());
    return HGL_OK;
  });
}

// ---------------------------------------------------------- vertex gather --

struct VertexArgs {
  int32_t n_tiles;
  const int32_t* tile_r0;
  const int32_t* tile_r1;
  const int32_t* tile_seg;
  const int32_t* vtx_ptr;
  const int32_t* vtx_edge;
  const int32_t* chunk_slot;
  const int32_t* chunk_begin;
  const int32_t* chunk_end;
  const int32_t* long_row;
  const int32_t* long_seg;
  const int32_t* long_chunk0;
  int32_t n_slots;
  const double* a_seg;
  const double* b_seg;
  const int32_t* chunk_order;  // chunk of workgroup n_tiles + j (-1: none)
};

// MODE 0: Out = a X - b s H Z (X may be null when a = 0: Out = -b s H Z).
// MODE 1: same + partial <X, Out>.
// MODE 2: Out = Y - (a X - b s H Z), partial <Out, Out>, all in TZ (FP64).
// MODE 3 (CG step with X = P): Q = a P - b s H Z stays in registers;
// F += alpha P, R -= alpha Q (u.F, u.R), partial <R, R> of the new R.
// Decoupled rows (s_v = 0, solved at the start of the solve) are skipped:
// no loads, no stores.
// At least 5 waves per SIMD: the fused step (MODE 3) with its row prefetch
// then fits in 96 VGPRs without spilling; the other modes use fewer anyway.
template <class T, class TZ, int GL, int V, int MODE>
__global__ __launch_bounds__(kBlock, 5) void k_spmm_vertex(
    VertexArgs va, const TZ* __restrict__ s, const T* __restrict__ X, int64_t ldx,
    const TZ* __restrict__ Z, int64_t ldz, const T* __restrict__ Y, int64_t ldy, T* __restrict__ Out,
    int64_t ldo, double* __restrict__ part, TZ* __restrict__ chunk_part, int k, Gate gate, UpdArgs<T> u) {
  if (gate.skip()) return;
  constexpr int GPB = kBlock / GL;
  constexpr int W = GL * V;
  __shared__ double lds_d[4 * W];
  __shared__ TZ lds_z[4 * W];
  const int grp = threadIdx.x / GL, lane = threadIdx.x % GL;
  const int col = blockIdx.y * W + lane * V;
  const bool colok = col < k;

  if (int(blockIdx.x) < va.n_tiles) {
    // ------------------------------------------------ a tile of short rows
    const int t = blockIdx.x;
    const int r0 = va.tile_r0[t], r1 = va.tile_r1[t];
    const int g = va.tile_seg[t];
    const TZ a = TZ(va.a_seg[g]), bb = TZ(va.b_seg[g]);
    // stage the tile's row offsets and (up to kStageIdx) hyperedge ids in LDS:
    // one coalesced round trip instead of two dependent ones per row
    __shared__ int32_t s_ptr[kTileRows + 1];
    __shared__ int32_t s_idx[kStageIdx];
    // the row streams (X; F and R in MODE 3) do not depend on the gather.
    // MODE 3 issues each group's first row before the staging and each
    // further row while the group gathers the row before it; the other modes
    // keep their registers (and so their occupancy) and load a row when they
    // reach it.  MODE 0 may have no X (a = 0).
    constexpr bool kAhead = MODE == 3;
    __shared__ uint8_t s_live[kTileRows];  // MODE 3: the row iterates (s_v != 0, not a hub row)
    T x[V] = {}, fv[V] = {}, rv[V] = {};
    auto fetch = [&](int r, T (&xx)[V], T (&ff)[V], T (&rr)[V]) {
      if (MODE != 0 || X) {
        load_row<V>(X + int64_t(r) * ldx + col, xx);
      } else {
#pragma unroll
        for (int i = 0; i < V; ++i) xx[i] = T(0);
      }
      if constexpr (MODE == 3) {
        load_row<V>(u.F + int64_t(r) * u.ldf + col, ff);
        load_row<V>(u.R + int64_t(r) * u.ldr + col, rr);
      }
    };
    int rcur = r0 + grp;
    if (kAhead && rcur < r1 && colok) fetch(rcur, x, fv, rv);
    const int nr = r1 - r0;
    for (int i = threadIdx.x; i <= nr; i += kBlock) s_ptr[i] = va.vtx_ptr[r0 + i];
    TZ sv_own = TZ(0);
    if (MODE == 3 && threadIdx.x < nr) sv_own = s[r0 + threadIdx.x];
    __syncthreads();
    if (MODE == 3 && threadIdx.x < nr)
      s_live[threadIdx.x] = sv_own != TZ(0) && s_ptr[threadIdx.x + 1] - s_ptr[threadIdx.x] <= kLongRow;
    const int base = s_ptr[0];
    const int staged = min(s_ptr[nr] - base, kStageIdx);
    for (int i = threadIdx.x; i < staged; i += kBlock) s_idx[i] = va.vtx_edge[base + i];
    __syncthreads();
    // the group's next row to process at or after r (MODE 3: rows that iterate)
    auto next_row = [&](int r) {
      if constexpr (MODE == 3)
        while (r < r1 && !s_live[r - r0]) r += GPB;
      return r;
    };
    if constexpr (MODE == 3) {
      const int first = next_row(rcur);
      if (first != rcur && first < r1 && colok) fetch(first, x, fv, rv);  // the prefetched row does not iterate
      rcur = first;
    }
    double dot[V];
    T al[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      dot[i] = 0.0;
      if constexpr (MODE == 3) al[i] = colok ? T(u.alpha[int64_t(g) * k + col + i]) : T(0);
    }
    for (int r = rcur; r < r1 && colok;) {
      const int eb = s_ptr[r - r0], ee = s_ptr[r - r0 + 1];
      const int rnext = next_row(r + GPB);
      T xn[V] = {}, fn[V] = {}, rn[V] = {};
      if constexpr (kAhead) {
        if (rnext < r1) fetch(rnext, xn, fn, rn);
      } else {
        fetch(r, x, fv, rv);
      }
      if (ee - eb <= kLongRow) {  // longer rows are finished by their chunks
        T o[V];
        const TZ sr = s[r];
        TZ acc[V];
#pragma unroll
        for (int i = 0; i < V; ++i) acc[i] = TZ(0);
        if (ee - base <= staged)
          gather_rows<V>(Z, ldz, s_idx, eb - base, ee - base, col, acc);
        else
          gather_rows<V>(Z, ldz, va.vtx_edge, eb, ee, col, acc);
        if constexpr (MODE == 2) {
          T y[V];
          load_row<V>(Y + int64_t(r) * ldy + col, y);
#pragma unroll
          for (int i = 0; i < V; ++i) {
            TZ ri = TZ(y[i]) - (a * TZ(x[i]) - bb * sr * acc[i]);
            dot[i] += double(ri) * double(ri);
            o[i] = T(ri);
          }
        } else {
#pragma unroll
          for (int i = 0; i < V; ++i) {
            TZ q = a * TZ(x[i]) - bb * sr * acc[i];
            o[i] = T(q);
            if constexpr (MODE == 1) dot[i] += double(x[i]) * double(o[i]);
            if constexpr (MODE == 3) {
              fv[i] += al[i] * x[i];
              rv[i] -= al[i] * o[i];
              dot[i] += double(rv[i]) * double(rv[i]);
            }
          }
        }
        if constexpr (MODE == 3) {
          store_row<V>(u.F + int64_t(r) * u.ldf + col, fv);
          store_row<V>(u.R + int64_t(r) * u.ldr + col, rv);
        } else {
          store_row<V>(Out + int64_t(r) * ldo + col, o);
        }
      }
      if constexpr (kAhead) {
#pragma unroll
        for (int i = 0; i < V; ++i) {
          x[i] = xn[i];
          fv[i] = fn[i];
          rv[i] = rn[i];
        }
      }
      r = rnext;
    }
    if constexpr (MODE != 0) {
      double tot = block_colsum<GL, V>(dot, lds_d);
      const int c = blockIdx.y * W + threadIdx.x;
      if (threadIdx.x < W && c < k) part[int64_t(t) * k + c] = tot;
    }
    return;
  }

  // ------------------------------------------------ one chunk of a long row
  // (workgroups are ordered so that a chunk reading one eighth of Z runs on
  // the XCD whose L2 serves that eighth)
  const int ch = va.chunk_order[blockIdx.x - va.n_tiles];
  if (ch < 0) return;  // padding (uniform over the workgroup)
  const int slot = va.chunk_slot[ch];
  const int eb = va.chunk_begin[ch], ee = va.chunk_end[ch];
  TZ acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) acc[i] = TZ(0);
  if (colok) {
    // each group sums a contiguous share of the chunk's hyperedges
    const int per = (ee - eb + GPB - 1) / GPB;
    const int jb = eb + grp * per;
    const int je = min(jb + per, ee);
    gather_rows<V>(Z, ldz, va.vtx_edge, jb, je, col, acc);
  }
  TZ csum = block_colsum<GL, V>(acc, lds_z);
  const int c = blockIdx.y * W + threadIdx.x;
  if (threadIdx.x < W && c < k) chunk_part[int64_t(ch) * k + c] = csum;
}

// Finish the long rows (one workgroup per row and column slab): sum the
// row's chunk partials, groups taking chunks round-robin, then a fixed-order
// block reduction (deterministic), and apply the epilogue of MODE.  Runs as
// its own launch after k_spmm_vertex, so the partials are visible without
// cross-workgroup fences.
template <class T, class TZ, int GL, int V, int MODE>
__global__ __launch_bounds__(kBlock) void k_spmm_vertex_finish(
    VertexArgs va, const TZ* __restrict__ s, const T* __restrict__ X, int64_t ldx,
    const T* __restrict__ Y, int64_t ldy, T* __restrict__ Out, int64_t ldo, double* __restrict__ part,
    const TZ* __restrict__ chunk_part, int k, Gate gate, UpdArgs<T> u) {
  if (gate.skip()) return;
  constexpr int GPB = kBlock / GL;
  constexpr int W = GL * V;
  __shared__ TZ lds_z[4 * W];
  const int grp = threadIdx.x / GL, lane = threadIdx.x % GL;
  const int col = blockIdx.y * W + lane * V;
  const bool colok = col < k;
  const int slot = blockIdx.x;
  const int c0 = va.long_chunk0[slot];
  const int nch = va.long_chunk0[slot + 1] - c0;
  TZ acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) acc[i] = TZ(0);
  if (colok) {
    int q = grp;
    for (; q + 3 * GPB < nch; q += 4 * GPB) {
      TZ p0[V], p1[V], p2[V], p3[V];
      load_row<V>(chunk_part + int64_t(c0 + q) * k + col, p0);
      load_row<V>(chunk_part + int64_t(c0 + q + GPB) * k + col, p1);
      load_row<V>(chunk_part + int64_t(c0 + q + 2 * GPB) * k + col, p2);
      load_row<V>(chunk_part + int64_t(c0 + q + 3 * GPB) * k + col, p3);
#pragma unroll
      for (int i = 0; i < V; ++i) acc[i] += ((p0[i] + p1[i]) + p2[i]) + p3[i];
    }
    for (; q < nch; q += GPB) {
      TZ p0[V];
      load_row<V>(chunk_part + int64_t(c0 + q) * k + col, p0);
#pragma unroll
      for (int i = 0; i < V; ++i) acc[i] += p0[i];
    }
  }
  const TZ sum = block_colsum<GL, V>(acc, lds_z);
  const int c = blockIdx.y * W + threadIdx.x;
  if (threadIdx.x >= W || c >= k) return;
  const int r = va.long_row[slot];
  const int g = va.long_seg[slot];
  const TZ a = TZ(va.a_seg[g]), bb = TZ(va.b_seg[g]);
  const TZ sr = s[r];
  const TZ x = (MODE != 0 || X) ? TZ(X[int64_t(r) * ldx + c]) : TZ(0);
  double d = 0.0;
  if constexpr (MODE == 2) {
    TZ ri = TZ(Y[int64_t(r) * ldy + c]) - (a * x - bb * sr * sum);
    Out[int64_t(r) * ldo + c] = T(ri);
    d = double(ri) * double(ri);
  } else if constexpr (MODE == 3) {
    if (sr == TZ(0)) {  // decoupled (every hyperedge of weight 0): solved at the start
      part[int64_t(va.n_tiles + slot) * k + c] = 0.0;
      return;
    }
    const T o = T(a * x - bb * sr * sum);
    const T xv = X[int64_t(r) * ldx + c];
    const T al = T(u.alpha[int64_t(g) * k + c]);
    T fv = u.F[int64_t(r) * u.ldf + c];
    T rv = u.R[int64_t(r) * u.ldr + c];
    fv += al * xv;
    rv -= al * o;
    u.F[int64_t(r) * u.ldf + c] = fv;
    u.R[int64_t(r) * u.ldr + c] = rv;
    d = double(rv) * double(rv);
  } else {
    T o = T(a * x - bb * sr * sum);
    Out[int64_t(r) * ldo + c] = o;
    d = double(X[int64_t(r) * ldx + c]) * double(o);
  }
  if constexpr (MODE != 0) part[int64_t(va.n_tiles + slot) * k + c] = d;
}

template <class T, class TZ>
int launch_spmm_vertex(const hgl_handle* h, VMode mode, const T* X, int64_t ldx, const TZ* Z,
                       int64_t ldz, const T* Y, int64_t ldy, T* Out, int64_t ldo,
                       const double* a_seg, const double* b_seg, double* part, int k,
                       const ColShape& cs, Gate gate, hipStream_t st, UpdArgs<T> u, TZ* chunk_buf) {
  hgl_handle* hm = const_cast<hgl_handle*>(h);
  if (!chunk_buf && h->n_chunks > 0 && hm->ws_chunk.bytes < sizeof(TZ) * size_t(h->n_chunks) * k) {
    // growing a buffer frees the old one: wait for queued work that may use it
    HGL_HIP(hipStreamSynchronize(st));
    HGL_TRY(hm->ws_chunk.reserve(sizeof(TZ) * size_t(h->n_chunks) * k));
  }
  VertexArgs va{h->n_tiles,  h->tile_r0,     h->tile_r1,   h->tile_seg, h->vtx_ptr,
                h->vtx_edge, h->chunk_slot,  h->chunk_begin, h->chunk_end, h->long_row,
                h->long_seg, h->long_chunk0, n_slots(h),  a_seg,       b_seg,
                h->chunk_order};
  const TZ* s;
  if constexpr (sizeof(TZ) == 8) s = h->s64; else s = h->s32;
  TZ* cp = chunk_buf ? chunk_buf : hm->ws_chunk.as<TZ>();
  dim3 grid(h->n_tiles + h->n_dispatch, cs.slabs);
  dim3 grid_fin(h->n_long, cs.slabs);
  if (mode == VMode::Resid && sizeof(TZ) != 8) {
    set_error("residual mode needs FP64 accumulation");
    return HGL_EUNSUPPORTED;
  }
  if (mode == VMode::Step && (!u.F || !u.R || !u.alpha || !part)) {
    set_error("internal: CG step mode needs F, R, alpha and partial sums");
    return HGL_EINVAL;
  }
  auto run = [&](auto kv, auto kf) {
    launch(h, -1, kv, grid, dim3(kBlock), 0, st, va, s, X, ldx, Z, ldz, Y, ldy, Out, ldo, part, cp, k, gate, u);
    if (h->n_long > 0)
      launch(h, kProfFinish, kf, grid_fin, dim3(kBlock), 0, st, va, s, X, ldx, Y, ldy, Out, ldo, part,
             static_cast<const TZ*>(cp), k, gate, u);
  };
  return HGL_DISPATCH_SHAPE(cs, sizeof(T) > sizeof(TZ) ? sizeof(T) : sizeof(TZ), {
    if (mode == VMode::Apply) {
      run(k_spmm_vertex<T, TZ, GL, V, 0>, k_spmm_vertex_finish<T, TZ, GL, V, 0>);
    } else if (mode == VMode::ApplyDot) {
      run(k_spmm_vertex<T, TZ, GL, V, 1>, k_spmm_vertex_finish<T, TZ, GL, V, 1>);
    } else if (mode == VMode::Step) {
      if constexpr (std::is_same<T, TZ>::value)
        run(k_spmm_vertex<T, TZ, GL, V, 3>, k_spmm_vertex_finish<T, TZ, GL, V, 3>);
    } else if constexpr (sizeof(TZ) == 8) {
      run(k_spmm_vertex<T, TZ, GL, V, 2>, k_spmm_vertex_finish<T, TZ, GL, V, 2>);
    }
    HGL_HIP(hipGetLastError());
    return HGL_OK;
  });
}

template <class T>
GatherShapes tune_shapes(hgl_handle* h, int k, const ColShape& base, const T* X, int64_t ldx, T* Z,
                         UpdArgs<T> u, double* epart, double* part, const double* a_seg, const double* b_seg,
                         hipStream_t s) {
  for (const auto& e : h->tuned)
    if (e[0] == k && e[1] == int(sizeof(T)) && e[2] == base.V) {
      GatherShapes g;
      g.edge = ColShape{e[3], e[4], e[5]};
      g.vertex = ColShape{e[6], e[7], e[8]};
      return g;
    }
  // candidates: vector width V' <= base.V; lanes from the smallest power of
  // two covering the row down to 8 (more column slabs); the default (base)
  // comes first and is kept for a kernel unless another candidate runs that
  // kernel 5% faster
  std::vector<ColShape> cand{base};
  for (int V = base.V; V >= 1; V >>= 1) {
    const int need = (k + V - 1) / V;
    int GL = 4;
    while (GL < need && GL < 64) GL <<= 1;
    for (int gl = GL; gl >= 8 && cand.size() < 12; gl >>= 1) {
      ColShape cs;
      cs.GL = gl;
      cs.V = V;
      cs.slabs = (k + gl * V - 1) / (gl * V);
      if (cs.slabs > 16) break;
      if (cs.GL == base.GL && cs.V == base.V && cs.slabs == base.slabs) continue;
      cand.push_back(cs);
    }
  }
  GatherShapes best{base, base};
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto& e2 : ev)
        if (e2) hipEventDestroy(e2);
      return best;
    }
  float best_e = 1e30f, best_v = 1e30f, base_e = -1.f, base_v = -1.f;
  for (const ColShape& cs : cand) {
    // the solver's own launches: edge gather with the hyperedge partials,
    // vertex gather as the fused step (u.alpha is zero: F and R keep their
    // values)
    auto edge = [&]() { return launch_spmm_edge<T, T>(h, X, ldx, Z, k, k, cs, Gate{}, s, epart) == HGL_OK; };
    auto vertex = [&]() {
      return launch_spmm_vertex<T, T>(h, VMode::Step, X, ldx, Z, k, nullptr, 0, nullptr, 0, a_seg, b_seg, part, k,
                                      cs, Gate{}, s, u) == HGL_OK;
    };
    if (!edge() || !vertex()) continue;  // warm-up (and shape check)
    hipEventRecord(ev[0], s);
    bool ok = true;
    for (int rep = 0; rep < 3 && ok; ++rep) ok = edge();
    hipEventRecord(ev[1], s);
    for (int rep = 0; rep < 3 && ok; ++rep) ok = vertex();
    hipEventRecord(ev[2], s);
    float me = 0.f, mv = 0.f;
    if (!ok || hipEventSynchronize(ev[2]) != hipSuccess || hipEventElapsedTime(&me, ev[0], ev[1]) != hipSuccess ||
        hipEventElapsedTime(&mv, ev[1], ev[2]) != hipSuccess)
      continue;
    if (cs.GL == base.GL && cs.V == base.V && cs.slabs == base.slabs) {
      base_e = me;
      base_v = mv;
    }
    if (me < best_e) {
      best_e = me;
      best.edge = cs;
    }
    if (mv < best_v) {
      best_v = mv;
      best.vertex = cs;
    }
  }
  for (auto& e : ev) hipEventDestroy(e);
  clear_error();
  // keep the default unless another shape is clearly faster (timing noise
  // must not flip the choice from one process to the next)
  if (base_e > 0.f && best_e > 0.95f * base_e) best.edge = base;
  if (base_v > 0.f && best_v > 0.95f * base_v) best.vertex = base;
  h->tuned.push_back({k, int(sizeof(T)), base.V, best.edge.GL, best.edge.V, best.edge.slabs, best.vertex.GL,
                      best.vertex.V, best.vertex.slabs});
  return best;
}

template GatherShapes tune_shapes<float>(hgl_handle*, int, const ColShape&, const float*, int64_t, float*,
                                         UpdArgs<float>, double*, double*, const double*, const double*, hipStream_t);
template GatherShapes tune_shapes<double>(hgl_handle*, int, const ColShape&, const double*, int64_t, double*,
                                          UpdArgs<double>, double*, double*, const double*, const double*,
                                          hipStream_t);

template int launch_spmm_edge<float, float>(const hgl_handle*, const float*, int64_t, float*,
                                            int64_t, int, const ColShape&, Gate, hipStream_t, double*);
template int launch_spmm_edge<float, double>(const hgl_handle*, const float*, int64_t, double*,
                                             int64_t, int, const ColShape&, Gate, hipStream_t, double*);
template int launch_spmm_edge<double, double>(const hgl_handle*, const double*, int64_t, double*,
                                              int64_t, int, const ColShape&, Gate, hipStream_t, double*);
template int launch_spmm_vertex<float, float>(const hgl_handle*, VMode, const float*, int64_t,
                                              const float*, int64_t, const float*, int64_t, float*,
                                              int64_t, const double*, const double*, double*, int,
                                              const ColShape&, Gate, hipStream_t, UpdArgs<float>, float*);
template int launch_spmm_vertex<float, double>(const hgl_handle*, VMode, const float*, int64_t,
                                               const double*, int64_t, const float*, int64_t, float*,
                                               int64_t, const double*, const double*, double*, int,
                                               const ColShape&, Gate, hipStream_t, UpdArgs<float>, double*);
template int launch_spmm_vertex<double, double>(const hgl_handle*, VMode, const double*, int64_t,
                                                const double*, int64_t, const double*, int64_t,
                                                double*, int64_t, const double*, const double*,
                                                double*, int, const ColShape&, Gate,
                                                hipStream_t, UpdArgs<double>, double*);

// Per-graph (a, b) = (1 + 1/lambda_g, 1/lambda_g) in a device array [2G].
int upload_ab(hgl_handle* h, const double* lambdas_host, hipStream_t st) {
  DevBuf& buf = h->ws_ab;
  if (buf.p && h->ab_cache.size() == size_t(h->G) &&
      std::equal(h->ab_cache.begin(), h->ab_cache.end(), lambdas_host))
    return HGL_OK;
  h->ab_cache.assign(lambdas_host, lambdas_host + h->G);
  std::vector<double> ab(2 * h->G);
  for (int g = 0; g < h->G; ++g) {
    ab[g] = 1.0 + 1.0 / lambdas_host[g];
    ab[h->G + g] = 1.0 / lambdas_host[g];
  }
  HGL_TRY(ensure_pinned(h, 2 * h->G));
  HGL_TRY(buf.reserve(sizeof(double) * 2 * h->G));
  // staged through pinned memory so the copy is truly asynchronous
  std::copy(ab.begin(), ab.end(), h->pinned_d);
  HGL_HIP(hipMemcpyAsync(buf.p, h->pinned_d, sizeof(double) * 2 * h->G, hipMemcpyHostToDevice, st));
  HGL_HIP(hipStreamSynchronize(st));
  return HGL_OK;
}

}  // namespace hgl

using namespace hgl;

extern "C" int hgl_apply(hgl_handle* h, double lambda, int32_t dt, const void* P, int64_t ldp,
                         void* Q, int64_t ldq, int32_t k, hipStream_t st) {
  clear_error();
  enter(h, st);
  HGL_CHECK_ARG(h != nullptr, "handle is NULL");
  HGL_CHECK_ARG(lambda > 0.0 && std::isfinite(lambda), "lambda must be > 0 (got %g)", lambda);
  HGL_CHECK_ARG(k >= 1, "k must be >= 1");
  HGL_CHECK_ARG(P && Q, "P and Q must not be NULL");
  HGL_CHECK_ARG(ldp >= k && ldq >= k, "leading dimensions must be >= k");
  HGL_CHECK_ARG(dt == HGL_F64 || dt == HGL_F32, "dtype must be HGL_F64 or HGL_F32");
  std::vector<double> lams(h->G, lambda);
  HGL_TRY(upload_ab(h, lams.data(), st));
  const double* a_seg = h->ws_ab.as<double>();
  const double* b_seg = a_seg + h->G;
  if (dt == HGL_F32) {
    ColShape cs = pick_shape(k, 4, {P, Q}, {ldp, ldq, int64_t(k)});
    HGL_TRY(h->ws_z.reserve(sizeof(float) * size_t(h->E) * k));
    float* Z = h->ws_z.as<float>();
    HGL_TRY(launch_spmm_edge<float, float>(h, static_cast<const float*>(P), ldp, Z, k, k, cs, Gate{}, st));
    HGL_TRY(launch_spmm_vertex<float, float>(h, VMode::Apply, static_cast<const float*>(P), ldp, Z, k,
                                             nullptr, 0, static_cast<float*>(Q), ldq, a_seg, b_seg,
                                             nullptr, k, cs, Gate{}, st));
  } else {
    ColShape cs = pick_shape(k, 8, {P, Q}, {ldp, ldq, int64_t(k)});
    HGL_TRY(h->ws_z64.reserve(sizeof(double) * size_t(h->E) * k));
    double* Z = h->ws_z64.as<double>();
    HGL_TRY(launch_spmm_edge<double, double>(h, static_cast<const double*>(P), ldp, Z, k, k, cs, Gate{}, st));
    HGL_TRY(launch_spmm_vertex<double, double>(h, VMode::Apply, static_cast<const double*>(P), ldp, Z,
                                               k, nullptr, 0, static_cast<double*>(Q), ldq, a_seg,
                                               b_seg, nullptr, k, cs, Gate{}, st));
  }
  return HGL_OK;
}
