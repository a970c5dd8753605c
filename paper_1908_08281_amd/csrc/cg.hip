// Conjugate gradient for (I + L/lambda) F = Y, every (graph, column) with its
// own recurrence (paper, section 3, eqs. 16-20):
//   alpha = r'r / p'Mp,  f += alpha p,  r -= alpha Mp,
//   beta = r_new'r_new / r'r,  p = r + beta p.
// One iteration is a fixed sequence of launches on one stream:
//   edge gather (Z = C H' S P) -> vertex gather (Q = M P, partial p'Q)
//   [-> hub-row finish] -> reduce: alpha -> update (F, R, partial r'r)
//   -> [preconditioner] -> reduce: beta, convergence
//   -> direction update (P = R + beta P, or Z + beta P with a preconditioner).
// Residual replacement (R = Y - M F with FP64 accumulation) runs at host
// checks and optionally every rr_period iterations.  The recursion continues
// from the recomputed residual with the same search direction only while the
// two residuals still agree (true norm at most kKeepDir times the recursive
// one); otherwise, and for a claimed column that a check sends back to
// iterate, the direction restarts from the recomputed residual (P = R).
// Inner products are accumulated in FP64 per workgroup and reduced in a fixed
// order (deterministic).  Converged columns get alpha = 0; once every column
// has converged the remaining launches of an enqueued chunk return at once.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "kernels.h"

namespace hgl {

// Column states.  A column whose recursive residual falls to the claim level
// stops (kClaimed: alpha = 0, P kept) until a host-scheduled check
// recomputes its residual: done if that meets tol, else restarted from the
// recomputed residual (kRestart: the restart launch sets P = R, the next
// alpha step makes it active).  A check that finds a column still active
// replaces its residual and leaves its direction.
enum : int32_t { kActive = 0, kDone = 1, kBreakdown = 2, kClaimed = 3, kRestart = 4 };

// A replaced residual keeps the column's search direction only if its norm is
// at most kKeepDir times the recursive residual's.  Near FP32's attainable
// accuracy the recursive residual drifts far below the true one; alpha =
// r'r / p'Mp with the true r'r then overshoots along a direction scaled to
// the recursive residual, and the iteration diverges.  With rounding errors
// uncorrelated with r, |r_true|^2 ~ |r_rec|^2 + |r_true - r_rec|^2, so the
// bound keeps the direction while the deviation is below about 0.46 |r_rec|.
constexpr double kKeepDir = 1.1;
constexpr double kKeepDir2 = kKeepDir * kKeepDir;

struct CgState {
  double* yy;      // [G*k] ||y||^2
  double* rr;      // [G*k] r'r of the current residual
  double* alpha;   // [G*k]
  double* beta;    // [G*k]
  double* relres;  // [G*k] last FP64-recomputed relative residual
  double* rz;      // [G*k] r'z (preconditioned) or r'r
  int32_t* state;  // [G*k]
  int32_t* iters;  // [G*k]
};

// ------------------------------------------------------- row-stream kernels --

// Zero the long-row slots of a partial array (those rows are covered by the
// tile sums in the row-stream kernels).
__device__ __forceinline__ void zero_long_slots(double* part, int n_tiles, int n_slots, int n_long,
                                                int k) {
  const int64_t total = int64_t(n_long) * k;
  double* p = part + int64_t(n_tiles) * k;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

// Start: (x0 not given) F = 0, R = Y; then P = R, or P = Zp when a
// preconditioned residual Zp is given.  Partials of r'r (when x0 is not
// given or rows are decoupled; otherwise the residual pass produced them),
// of y'y, and (part_pp not null) of p'p over the tiles.
// Decoupled rows (sdec not null, s_v = 0: no hyperedge of positive weight,
// so row v of A is zero and M_vv = a, reading R2): their equation is solved
// here, F_v = Y_v / a, and R_v = P_v = 0 keeps them out of the iteration.
template <class T, int GL, int V>
__global__ __launch_bounds__(kBlock) void k_cg_init(int32_t n_tiles, const int32_t* __restrict__ tile_r0,
                                                    const int32_t* __restrict__ tile_r1, int n_slots,
                                                    int n_long, const T* __restrict__ Y, int64_t ldy,
                                                    T* __restrict__ F, int64_t ldf, T* __restrict__ R,
                                                    T* __restrict__ P, int64_t ld, double* __restrict__ part_rr,
                                                    double* __restrict__ part_yy, int k, int x0_given,
                                                    const T* __restrict__ Zp, double* __restrict__ part_pp,
                                                    const T* __restrict__ sdec, const int32_t* __restrict__ tile_seg,
                                                    const double* __restrict__ a_seg) {
  constexpr int GPB = kBlock / GL, W = GL * V;
  __shared__ double lds[4 * W];
  const int grp = threadIdx.x / GL, lane = threadIdx.x % GL;
  const int col = blockIdx.y * W + lane * V;
  const int t = blockIdx.x;
  double rr[V], yy[V], pp[V];
#pragma unroll
  for (int i = 0; i < V; ++i) rr[i] = yy[i] = pp[i] = 0.0;
  if (col < k) {
    const double inv_a = sdec ? 1.0 / a_seg[tile_seg[t]] : 0.0;
    for (int r = tile_r0[t] + grp; r < tile_r1[t]; r += GPB) {
      T y[V], rv[V];
      load_row<V>(Y + int64_t(r) * ldy + col, y);
      if (sdec && sdec[r] == T(0)) {
        T f[V], z[V];
#pragma unroll
        for (int i = 0; i < V; ++i) {
          f[i] = T(double(y[i]) * inv_a);
          z[i] = T(0);
          yy[i] += double(y[i]) * double(y[i]);
        }
        store_row<V>(F + int64_t(r) * ldf + col, f);
        store_row<V>(R + int64_t(r) * ld + col, z);
        store_row<V>(P + int64_t(r) * ld + col, z);
        continue;
      }
      if (!x0_given) {
        T z[V];
#pragma unroll
        for (int i = 0; i < V; ++i) {
          z[i] = T(0);
          rv[i] = y[i];
        }
        store_row<V>(F + int64_t(r) * ldf + col, z);
        store_row<V>(R + int64_t(r) * ld + col, rv);
      } else {
        load_row<V>(R + int64_t(r) * ld + col, rv);
      }
      T pv[V];
      if (Zp) {
        load_row<V>(Zp + int64_t(r) * ld + col, pv);
      } else {
#pragma unroll
        for (int i = 0; i < V; ++i) pv[i] = rv[i];
      }
      store_row<V>(P + int64_t(r) * ld + col, pv);
#pragma unroll
      for (int i = 0; i < V; ++i) {
        yy[i] += double(y[i]) * double(y[i]);
        rr[i] += double(rv[i]) * double(rv[i]);
        pp[i] += double(pv[i]) * double(pv[i]);
      }
    }
  }
  double syy = block_colsum<GL, V>(yy, lds);
  double srr = block_colsum<GL, V>(rr, lds);
  double spp = part_pp ? block_colsum<GL, V>(pp, lds) : 0.0;
  const int c = blockIdx.y * W + threadIdx.x;
  // with decoupled rows the r'r of the residual pass (x0 given) included
  // their old residual: r'r is taken here over the rows that iterate
  const bool own_rr = !x0_given || sdec;
  if (threadIdx.x < W && c < k) {
    part_yy[int64_t(t) * k + c] = syy;
    if (own_rr) part_rr[int64_t(t) * k + c] = srr;
    if (part_pp) part_pp[int64_t(t) * k + c] = spp;
  }
  if (blockIdx.y == 0) {
    // the tile sums above cover every row, hub rows included
    zero_long_slots(part_yy, n_tiles, n_slots, n_long, k);
    if (own_rr) zero_long_slots(part_rr, n_tiles, n_slots, n_long, k);
  }
}

// F += alpha P, R -= alpha Q; partial r'r.
template <class T, int GL, int V>
__global__ __launch_bounds__(kBlock) void k_cg_update(
    int32_t n_tiles, const int32_t* __restrict__ tile_r0, const int32_t* __restrict__ tile_r1,
    const int32_t* __restrict__ tile_seg, int n_slots, int n_long, T* __restrict__ F, int64_t ldf,
    T* __restrict__ R, const T* __restrict__ P, const T* __restrict__ Q, int64_t ld,
    const double* __restrict__ alpha, double* __restrict__ part_rr, int k, Gate gate) {
  if (gate.skip()) return;
  constexpr int GPB = kBlock / GL, W = GL * V;
  __shared__ double lds[4 * W];
  const int grp = threadIdx.x / GL, lane = threadIdx.x % GL;
  const int col = blockIdx.y * W + lane * V;
  const int t = blockIdx.x;
  const int g = tile_seg[t];
  double rr[V];
#pragma unroll
  for (int i = 0; i < V; ++i) rr[i] = 0.0;
  if (col < k) {
    T al[V];
#pragma unroll
    for (int i = 0; i < V; ++i) al[i] = T(alpha[int64_t(g) * k + col + i]);
    for (int r = tile_r0[t] + grp; r < tile_r1[t]; r += GPB) {
      T f[V], rv[V], p[V], q[V];
      load_row<V>(F + int64_t(r) * ldf + col, f);
      load_row<V>(R + int64_t(r) * ld + col, rv);
      load_row<V>(P + int64_t(r) * ld + col, p);
      load_row<V>(Q + int64_t(r) * ld + col, q);
#pragma unroll
      for (int i = 0; i < V; ++i) {
        f[i] += al[i] * p[i];
        rv[i] -= al[i] * q[i];
        rr[i] += double(rv[i]) * double(rv[i]);
      }
      store_row<V>(F + int64_t(r) * ldf + col, f);
      store_row<V>(R + int64_t(r) * ld + col, rv);
    }
  }
  double s = block_colsum<GL, V>(rr, lds);
  const int c = blockIdx.y * W + threadIdx.x;
  if (threadIdx.x < W && c < k) part_rr[int64_t(t) * k + c] = s;
  if (blockIdx.y == 0) zero_long_slots(part_rr, n_tiles, n_slots, n_long, k);
}

// P = R + beta P for the iterating columns; a claimed column keeps P.
// restart_only: P = R (beta is 0 for them) for the columns in kRestart only,
// every other column keeps P.
// part_pp (nullable): tile partials of p'p of the new P (the vertex half of
// the next p'Mp).
// sdec (nullable): rows with s_v = 0 are decoupled (solved at the start) and
// skipped.
template <class T, int GL, int V>
__global__ __launch_bounds__(kBlock) void k_cg_direction(
    const int32_t* __restrict__ tile_r0, const int32_t* __restrict__ tile_r1,
    const int32_t* __restrict__ tile_seg, const T* __restrict__ R, T* __restrict__ P, int64_t ld,
    const double* __restrict__ beta, const int32_t* __restrict__ state, int k, Gate gate,
    double* __restrict__ part_pp, int restart_only, const T* __restrict__ sdec) {
  if (gate.skip()) return;
  constexpr int GPB = kBlock / GL, W = GL * V;
  const int grp = threadIdx.x / GL, lane = threadIdx.x % GL;
  const int col = blockIdx.y * W + lane * V;
  const int t = blockIdx.x;
  double pp[V];
#pragma unroll
  for (int i = 0; i < V; ++i) pp[i] = 0.0;
  if (col < k) {
    const int g = tile_seg[t];
    T be[V];
    bool keep[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      be[i] = T(beta[int64_t(g) * k + col + i]);
      const int32_t sc = state[int64_t(g) * k + col + i];
      keep[i] = restart_only ? sc != kRestart : sc == kClaimed;
    }
    for (int r = tile_r0[t] + grp; r < tile_r1[t]; r += GPB) {
      if (sdec && sdec[r] == T(0)) continue;
      T rv[V], p[V];
      load_row<V>(R + int64_t(r) * ld + col, rv);
      load_row<V>(P + int64_t(r) * ld + col, p);
#pragma unroll
      for (int i = 0; i < V; ++i) {
        p[i] = keep[i] ? p[i] : rv[i] + be[i] * p[i];
        pp[i] += double(p[i]) * double(p[i]);
      }
      store_row<V>(P + int64_t(r) * ld + col, p);
    }
  }
  if (part_pp) {
    __shared__ double lds[4 * W];
    const double spp = block_colsum<GL, V>(pp, lds);
    const int c = blockIdx.y * W + threadIdx.x;
    if (threadIdx.x < W && c < k) part_pp[int64_t(t) * k + c] = spp;
  }
}

// --------------------------------------------------------------- reductions --

// Partial sums are stored slot-major, part[slot][k]: the workgroup that
// owns a slot writes one contiguous row.  A reduction workgroup (kRedThreads
// threads, 16 waves) owns kRedCols columns of one graph: thread (lane l = tid
// % kRedCols, stripe j = tid / kRedCols) adds slots j, j + stripes, ... of
// column c0 + l (a stripe reads kRedCols contiguous values per slot; the
// graph's tiles, then its long rows), kRedBurst independent loads per array
// in flight per round.  The stripes are then added by a fixed butterfly of
// lane exchanges inside each wave and one across the 16 waves, so every sum
// is deterministic.  Results are valid in wave 0.
constexpr int kRedCols = 8;
constexpr int kRedThreads = 1024;
constexpr int kRedStripes = kRedThreads / kRedCols;
constexpr int kRedWaves = kRedThreads / 64;
constexpr int kRedBurst = 16;
static_assert(kRedWaves == 16 && kRedCols == 8, "the cross-wave step pairs waves w and w + 8");

// One partial-sum array and its slot ranges (tiles [t0, t1), long rows or
// long hyperedges [l0, l1)) for one graph.
struct SlotSrc {
  const double* p;
  int t0, t1, l0, l1;
};

__device__ __forceinline__ double wave_stripe_sum(double v) {
  // lanes holding the same column differ in lane-id bits 3..5
#pragma unroll
  for (int m = kRedCols; m < 64; m <<= 1) v += __shfl_xor(v, m);
  return v;
}

template <int NS>
__device__ __forceinline__ void slot_sums(const SlotSrc (&src)[NS], int k, int col, double (&out)[NS],
                                          double* lds /* [kRedWaves * NS * kRedCols] */) {
  const int j = threadIdx.x / kRedCols;
  double acc[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) acc[q] = 0.0;
  if (col < k) {
    int nt[NS], n[NS], nmax = 0;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      nt[q] = src[q].t1 - src[q].t0;
      n[q] = nt[q] + (src[q].l1 - src[q].l0);
      nmax = max(nmax, n[q]);
    }
    for (int i = j; i < nmax; i += kRedBurst * kRedStripes) {
      double x[NS][kRedBurst];
#pragma unroll
      for (int q = 0; q < NS; ++q)
#pragma unroll
        for (int u = 0; u < kRedBurst; ++u) {
          const int v = i + u * kRedStripes;
          const int slot = v < nt[q] ? src[q].t0 + v : src[q].l0 + (v - nt[q]);
          x[q][u] = v < n[q] ? src[q].p[int64_t(slot) * k + col] : 0.0;
        }
#pragma unroll
      for (int q = 0; q < NS; ++q) {
#pragma unroll
        for (int w = kRedBurst / 2; w >= 1; w >>= 1)
#pragma unroll
          for (int u = 0; u < w; ++u) x[q][u] += x[q][u + w];
        acc[q] += x[q][0];
      }
    }
  }
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    acc[q] = wave_stripe_sum(acc[q]);
    if (lane < kRedCols) lds[(wave * NS + q) * kRedCols + lane] = acc[q];
  }
  __syncthreads();
  if (wave == 0) {
    const int w2 = lane / kRedCols, l2 = lane % kRedCols;
#pragma unroll
    for (int q = 0; q < NS; ++q)
      out[q] = wave_stripe_sum(lds[(w2 * NS + q) * kRedCols + l2] + lds[((w2 + 8) * NS + q) * kRedCols + l2]);
  }
}

enum class RedOp { Init, Alpha, Beta, Check };

struct RedArgs {
  int G, k, n_slots;
  int32_t slots1[4], eslots1[4];  // the slot ranges when G == 1 (no loads)
  const int32_t* seg_slots;
  const double* part;   // r'r (Init, Beta, Check) or p'Mp (Alpha, not split)
  const double* part2;  // y'y (Init)
  const double* part3;  // r'z (Init, Beta, Check) when preconditioned
  const double* prec_rr;  // Beta after a periodic replacement: the recursive r'r
  // Alpha with p'Mp split as a p'p - b sum_e c_e |(H' S p)_e|^2 (eq. 1):
  // tile partials of p'p and edge-slot partials of the hyperedge sum
  const double* pp;     // null: p'Mp from part
  const double* epart;
  const int32_t* seg_eslots;
  const double* ab;     // [2G]: a_g = 1 + 1/lambda_g, then b_g = 1/lambda_g
  double tol;
  double claim;         // Beta: recursive relres at which a column stops for a check
  int iter;             // iteration index
  int periodic;         // Beta: the residual was recomputed in this iteration
  int has_prec;         // preconditioned: alpha, beta use r'z instead of r'r
};

// Flag words: cnt(it) = columns still iterating after iteration it (cnt(-1)
// after the start); chk(it) = columns still iterating after a check step run
// between iterations it-1 and it (the check adds them to cnt(it-1) as well,
// which gates iteration it).  One word per step, never reset inside the
// loop, so no launch can observe a word another launch is clearing.
struct Words {
  int32_t* base;
  int max_iter;
  __host__ __device__ int32_t* cnt(int it) const { return base + 1 + it; }
  __host__ __device__ int32_t* chk(int it) const { return base + (max_iter + 2) + it; }
  __host__ __device__ int32_t* err() const { return base + 2 * (max_iter + 2) + 1; }
  // largest recursive relative residual of the iterating columns after it
  // (FP64, updated with 64-bit atomics: the offset is kept 8-byte aligned;
  // base itself is 8-byte aligned)
  __host__ __device__ static int rmax_offset(int max_iter) { return (2 * (max_iter + 2) + 2 + 1) & ~1; }
  __host__ __device__ double* rmax(int it) const {
    return reinterpret_cast<double*>(base + rmax_offset(max_iter)) + it;
  }
  static size_t count(int max_iter) { return size_t(rmax_offset(max_iter)) + 2 * size_t(max_iter + 1); }
};

template <RedOp OP>
__global__ __launch_bounds__(kRedThreads) void k_cg_reduce(RedArgs ra, CgState st, Words wd) {
  const int it = ra.iter;
  // one workgroup per (graph, group of kRedCols columns); every load that
  // does not depend on the sums is issued first
  const int ngrp = (ra.k + kRedCols - 1) / kRedCols;
  const int g = blockIdx.x / ngrp;
  const int col = (blockIdx.x % ngrp) * kRedCols + threadIdx.x % kRedCols;
  const bool lead = threadIdx.x < kRedCols && col < ra.k;
  const int64_t id = int64_t(g) * ra.k + col;
  int gate = 1;
  if constexpr (OP == RedOp::Alpha || OP == RedOp::Beta) gate = *wd.cnt(it - 1);
  int32_t st0 = 0, it0 = 0;
  double rz0 = 0.0, yy0 = 0.0, rr0 = 0.0;
  if (lead && OP != RedOp::Init) {
    st0 = st.state[id];
    rz0 = st.rz[id];
    if constexpr (OP == RedOp::Beta || OP == RedOp::Check) yy0 = st.yy[id];
    if constexpr (OP == RedOp::Beta) it0 = st.iters[id];
    if constexpr (OP == RedOp::Check) rr0 = st.rr[id];
  }
  const bool split = OP == RedOp::Alpha && ra.pp != nullptr;
  double ag = 0.0, bg = 0.0;
  if (split) {
    ag = ra.ab[g];
    bg = ra.ab[ra.G + g];
  }
  // (the gate is tested after the sums: its load and the slot loads are in
  // flight together, and a gated-off launch, which reads valid slots it
  // then ignores, only happens after the last iteration)
  int sl[4], esl[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    sl[i] = ra.G == 1 ? ra.slots1[i] : ra.seg_slots[4 * g + i];
    esl[i] = ra.G == 1 ? ra.eslots1[i] : (split ? ra.seg_eslots[4 * g + i] : 0);
  }
  const SlotSrc all{nullptr, sl[0], sl[1], sl[2], sl[3]};
  __shared__ double lds[kRedWaves * 2 * kRedCols];
  double sum = 0.0, sum2 = 0.0, rz = 0.0;
  if constexpr (OP == RedOp::Alpha) {
    if (split) {
      // p'Mp = a p'p - b sum_e c_e |u_e|^2: p'p over the tiles only
      const SlotSrc src[2] = {{ra.pp, sl[0], sl[1], sl[2], sl[2]}, {ra.epart, esl[0], esl[1], esl[2], esl[3]}};
      double o[2];
      slot_sums<2>(src, ra.k, col, o, lds);
      sum = ag * o[0] - bg * o[1];
    } else {
      SlotSrc src[1] = {all};
      src[0].p = ra.part;
      double o[1];
      slot_sums<1>(src, ra.k, col, o, lds);
      sum = o[0];
    }
  } else if constexpr (OP == RedOp::Init) {
    SlotSrc src[2] = {all, all};
    src[0].p = ra.part;
    src[1].p = ra.part2;
    double o[2];
    slot_sums<2>(src, ra.k, col, o, lds);
    sum = o[0];
    sum2 = o[1];
  } else {
    if (ra.has_prec) {
      SlotSrc src[2] = {all, all};
      src[0].p = ra.part;
      src[1].p = ra.part3;
      double o[2];
      slot_sums<2>(src, ra.k, col, o, lds);
      sum = o[0];
      rz = o[1];
    } else {
      SlotSrc src[1] = {all};
      src[0].p = ra.part;
      double o[1];
      slot_sums<1>(src, ra.k, col, o, lds);
      sum = o[0];
    }
    if (OP == RedOp::Beta && ra.periodic) {
      // the recursive r'r of this iteration, set aside before the
      // replacement overwrote part
      SlotSrc src[1] = {all};
      src[0].p = ra.prec_rr;
      double o[1];
      __syncthreads();
      slot_sums<1>(src, ra.k, col, o, lds);
      rr0 = o[0];
    }
  }
  if (OP == RedOp::Init && ra.has_prec) {
    // r'z of the start: its own pass (three arrays)
    SlotSrc src[1] = {all};
    src[0].p = ra.part3;
    double o[1];
    __syncthreads();
    slot_sums<1>(src, ra.k, col, o, lds);
    rz = o[0];
  } else if (!ra.has_prec) {
    rz = sum;  // r'z = r'r without a preconditioner
  }
  if (gate == 0) return;  // uniform: no column iterates
  if (threadIdx.x >= kRedCols) return;
  // the per-column step: the counters it raises are added up over the
  // workgroup's columns first, so each flag word takes one atomic per
  // workgroup (lanes 0 .. kRedCols-1 of wave 0)
  int add_cnt = 0, add_chk = 0, add_err = 0;
  double rel_max = -1.0;
  if (col < ra.k) {
    do {
      if constexpr (OP == RedOp::Init) {
        st.yy[id] = sum2;
        st.rr[id] = sum;
        st.rz[id] = rz;
        st.iters[id] = 0;
        st.alpha[id] = 0.0;
        st.beta[id] = 0.0;
        const double rel = sum2 > 0.0 ? sqrt(sum / sum2) : sqrt(sum);
        st.relres[id] = rel;
        const bool done = sum2 == 0.0 || rel <= ra.tol;
        st.state[id] = done ? kDone : kActive;
        add_cnt = done ? 0 : 1;
      } else if constexpr (OP == RedOp::Alpha) {
        if (st0 == kRestart) {
          st.state[id] = kActive;  // its restart direction is in place
          st0 = kActive;
        }
        if (st0 != kActive || rz0 == 0.0) {
          st.alpha[id] = 0.0;
          break;
        }
        if (!(sum > 0.0) || !isfinite(sum) || !isfinite(rz0)) {
          st.alpha[id] = 0.0;
          st.state[id] = kBreakdown;
          add_err = 1;
          break;
        }
        st.alpha[id] = rz0 / sum;
      } else if constexpr (OP == RedOp::Beta) {
        if (st0 != kActive) {
          st.beta[id] = 0.0;
          break;
        }
        st.iters[id] = it0 + 1;
        const bool ran = ra.periodic != 0;  // sum is the recomputed true residual
        const double rel = sqrt(sum / yy0);
        if (ran) st.relres[id] = rel;
        if (ran && rel <= ra.tol) {  // a recomputed residual finishes the column
          st.state[id] = kDone;
          st.beta[id] = 0.0;
          st.rr[id] = sum;
          st.rz[id] = rz;
          break;
        }
        if (!isfinite(sum) || !isfinite(rz)) {
          st.state[id] = kBreakdown;
          st.beta[id] = 0.0;
          add_err = 1;
          break;
        }
        // after a periodic replacement the direction is kept only while the
        // true residual agrees with the recursive one (kKeepDir); else it
        // restarts in place (beta = 0: P = R, or the preconditioned R)
        st.beta[id] = (ran && sum > kKeepDir2 * rr0) ? 0.0 : rz / rz0;
        st.rr[id] = sum;
        st.rz[id] = rz;
        if (rel <= ra.claim * ra.tol) {  // stop for a check
          st.state[id] = kClaimed;
          break;
        }
        add_cnt = 1;
        rel_max = rel;
      } else {  // Check: sum is r'r of Y - M F recomputed in FP64
        if (st0 != kActive && st0 != kClaimed && st0 != kRestart) break;
        const double rel = yy0 > 0.0 ? sqrt(sum / yy0) : sqrt(sum);
        st.relres[id] = rel;
        // residual replacement: the recursion continues from the recomputed
        // residual
        st.rr[id] = sum;
        st.rz[id] = rz;
        if (rel <= ra.tol) {
          st.state[id] = kDone;
        } else if (st0 == kActive && sum <= kKeepDir2 * rr0) {
          add_chk = 1;  // still iterating, residuals agree: keeps its direction
        } else {
          // restart: the direction is rebuilt from the recomputed residual
          // (P = R, beta = 0), since the old one was scaled to a recursive
          // residual that has drifted from the true one
          st.state[id] = kRestart;
          st.beta[id] = 0.0;
          add_chk = 1;
        }
      }
    } while (false);
  }
#pragma unroll
  for (int off = kRedCols / 2; off >= 1; off >>= 1) {
    add_cnt += __shfl_xor(add_cnt, off, kRedCols);
    add_chk += __shfl_xor(add_chk, off, kRedCols);
    add_err |= __shfl_xor(add_err, off, kRedCols);
    rel_max = fmax(rel_max, __shfl_xor(rel_max, off, kRedCols));
  }
  if (threadIdx.x != 0) return;
  if (add_err) atomicOr(wd.err(), 1);
  if constexpr (OP == RedOp::Init) {
    if (add_cnt) atomicAdd(wd.cnt(-1), add_cnt);
  } else if constexpr (OP == RedOp::Beta) {
    if (add_cnt) {
      atomicAdd(wd.cnt(it), add_cnt);
      atomicMax(reinterpret_cast<unsigned long long*>(wd.rmax(it)),
                static_cast<unsigned long long>(__double_as_longlong(rel_max)));
    }
  } else if constexpr (OP == RedOp::Check) {
    if (add_chk) {
      atomicAdd(wd.chk(it), add_chk);
      atomicAdd(wd.cnt(it - 1), add_chk);  // iteration it runs for them
    }
  }
}

// ------------------------------------------------------------------ driver --

template <class T>
struct CgBuffers {
  T* R;
  T* P;
  T* Q;        // M P
  T* Z;        // E x k, type T
  double* Z64; // E x k FP64 (residual passes of the FP32 mode)
  double* part;
  double* part2;
  double* part3;
  T* Zp;       // preconditioned residual (PCG)
  double* pp;     // p'p tile partials (fused step)
  double* epart;  // edge-slot partials of sum_e c_e |(H' S p)_e|^2 (fused step)
  CgState st;
};

template <class T>
static int run_cg(hgl_handle* h, const double* lambdas, const hgl_cg_opts* o, const T* Y, int64_t ldy,
                  T* F, int64_t ldf, int k, int32_t* iters_host, double* relres_host, const Precond* prec,
                  hipStream_t s_user) {
  // the stream every launch below goes to (the capture stream while a chunk
  // of iterations is being recorded into a graph)
  hipStream_t s = s_user;
  const bool fp32 = sizeof(T) == 4;
  const bool has_prec = prec != nullptr;
  // Without a preconditioner the step is fused: p'Mp = a p'p - b sum_e c_e
  // |(H' S p)_e|^2 is reduced from the direction and edge-gather partials
  // before the vertex gather, which then applies F += alpha P, R -= alpha Q
  // with Q kept in registers (no Q round trip, no separate update pass).
  const bool fused = !has_prec;
  const int N = h->N, E = h->E, G = h->G;
  // Decoupled rows (s_v = 0) are solved at the start and skipped by the
  // iteration's row streams (fused step only; the preconditioned path keeps
  // every row).
  const T* sdec = nullptr;
  if (fused) {
    if constexpr (sizeof(T) == 4) sdec = h->s32;
    else sdec = h->s64;
  }
  const int64_t ld = k;  // internal vectors
  const int nsl = n_slots(h);
  // ---------------------------------------------------------- workspace
  const size_t vec = sizeof(T) * size_t(N) * ld;
  HGL_TRY(h->ws_vec.reserve((has_prec ? 4 : 3) * vec + 256));
  HGL_TRY(h->ws_z.reserve(sizeof(T) * size_t(std::max(E, 1)) * ld));
  if (fp32) HGL_TRY(h->ws_z64.reserve(sizeof(double) * size_t(std::max(E, 1)) * ld));
  HGL_TRY(h->ws_part.reserve(sizeof(double) * size_t(nsl) * k));
  HGL_TRY(h->ws_part2.reserve(sizeof(double) * size_t(nsl) * k));
  // part3 (r'z) with a preconditioner; p'p tile partials when fused
  HGL_TRY(h->ws_extra[0].reserve(sizeof(double) * size_t(nsl) * k));
  if (fused) HGL_TRY(h->ws_extra[5].reserve(sizeof(double) * size_t(std::max(n_eslots(h), 1)) * k));
  const size_t gk = size_t(G) * k;
  HGL_TRY(h->ws_state.reserve(sizeof(double) * 6 * gk + sizeof(int32_t) * (2 * gk + 2 + Words::count(o->max_iter))));
  HGL_TRY(ensure_pinned(h, 2 * gk + 8));
  if (h->n_chunks > 0) HGL_TRY(h->ws_chunk.reserve(sizeof(double) * size_t(h->n_chunks) * k));
  HGL_TRY(upload_ab(h, lambdas, s));
  const double* a_seg = h->ws_ab.as<double>();
  const double* b_seg = a_seg + G;

  CgBuffers<T> b;
  b.R = h->ws_vec.as<T>();
  b.P = b.R + size_t(N) * ld;
  b.Q = b.P + size_t(N) * ld;
  b.Z = h->ws_z.as<T>();
  b.Z64 = fp32 ? h->ws_z64.as<double>() : reinterpret_cast<double*>(b.Z);
  b.part = h->ws_part.as<double>();
  b.part2 = h->ws_part2.as<double>();
  b.part3 = has_prec ? h->ws_extra[0].as<double>() : nullptr;
  b.pp = fused ? h->ws_extra[0].as<double>() : nullptr;
  b.epart = fused ? h->ws_extra[5].as<double>() : nullptr;
  b.Zp = has_prec ? b.Q + size_t(N) * ld : nullptr;
  double* sd = h->ws_state.as<double>();
  b.st.yy = sd;
  b.st.rr = sd + gk;
  b.st.alpha = sd + 2 * gk;
  b.st.beta = sd + 3 * gk;
  b.st.relres = sd + 4 * gk;
  b.st.rz = sd + 5 * gk;
  b.st.state = reinterpret_cast<int32_t*>(sd + 6 * gk);
  b.st.iters = b.st.state + gk;
  // flag words start 8-byte aligned (they hold FP64 maxima)
  int32_t* words = b.st.iters + gk;
  if (reinterpret_cast<uintptr_t>(words) % 8 != 0) ++words;
  Words wd{words, o->max_iter};
  if (reinterpret_cast<uintptr_t>(wd.rmax(0)) % alignof(double) != 0) {
    set_error("internal: misaligned FP64 flag words");
    return HGL_EDEVICE;
  }
  HGL_HIP(hipMemsetAsync(wd.base, 0, Words::count(o->max_iter) * sizeof(int32_t), s));

  // row-streaming kernels: the widest-vector shape; operator gathers: the
  // autotuned one (the partial-sum layout does not depend on either)
  const ColShape cs = pick_shape(k, sizeof(T), {Y, F, b.R}, {ldy, ldf, ld});
  GatherShapes gs{cs, cs};
  if (o->tune) {
    // tuned on the solver's own launches, with alpha = 0 so that F (which
    // may hold x0) and R (rewritten by the start) keep their values
    HGL_HIP(hipMemsetAsync(b.st.alpha, 0, sizeof(double) * gk, s));
    gs = tune_shapes<T>(h, k, cs, Y, ldy, b.Z, UpdArgs<T>{F, ldf, b.R, ld, b.st.alpha}, b.epart, b.part, a_seg,
                        b_seg, s);
  }
  const ColShape cse = gs.edge, csv = gs.vertex;
  const int32_t shapes[6] = {cse.GL, cse.V, cse.slabs, csv.GL, csv.V, csv.slabs};
  std::copy(shapes, shapes + 6, h->last_shape);
  const ColShape cs64 = pick_shape(k, 8, {Y, F, b.R}, {ldy, ldf, ld});
  const int red_blocks = G * ((k + kRedCols - 1) / kRedCols);
  // claim < 1 in FP32 leaves room for the drift of the FP32 recursion from
  // the true residual
  const double claim = fp32 ? 0.5 : 1.0;
  // prec_rr: after a periodic replacement, the recursive r'r partials of the
  // iteration were written to part2 (free after the start)
  RedArgs ra{G,       k,      nsl,     {0, 0, 0, 0}, {0, 0, 0, 0}, h->seg_slots, b.part, b.part2,
             b.part3, b.part2, b.pp, b.epart, h->seg_eslots, a_seg, o->tol, claim, 0, 0, has_prec ? 1 : 0};
  if (G == 1)
    for (int i = 0; i < 4; ++i) {
      ra.slots1[i] = h->seg_slots_host[i];
      ra.eslots1[i] = h->seg_eslots_host[i];
    }

  // preconditioner: Zp = P^-1 R with partial r'z into part3 (or into part)
  auto precond = [&](const T* Rin, int64_t ldr, T* Zout, int64_t ldz, double* part, Gate gate) -> int {
    prof_begin(h, kProfPrecond, s);
    int st2;
    if constexpr (sizeof(T) == 4) st2 = prec->apply_f32(prec->ctx, Rin, ldr, Zout, ldz, part, k, gate, s);
    else st2 = prec->apply_f64(prec->ctx, Rin, ldr, Zout, ldz, part, k, gate, s);
    prof_end(h, s);
    return st2;
  };

  // residual pass R = Y - M F (FP64 accumulation), partial r'r into b.part
  auto resid = [&](Gate gate) -> int {
    prof_begin(h, kProfResidEdge, s);
    HGL_TRY(launch_spmm_edge<T, double>(h, F, ldf, b.Z64, ld, k, cs64, gate, s));
    prof_end(h, s);
    prof_begin(h, kProfResidVertex, s);
    HGL_TRY(launch_spmm_vertex<T, double>(h, VMode::Resid, F, ldf, b.Z64, ld, Y, ldy, b.R, ld, a_seg,
                                          b_seg, b.part, k, cs64, gate, s));
    prof_end(h, s);
    return HGL_OK;
  };

  // ------------------------------------------------------------- start
  // With a preconditioner and no start given, the start is F0 = P^-1 Y.
  const bool x0 = o->x0_given || has_prec;
  if (has_prec && !o->x0_given) HGL_TRY(precond(Y, ldy, F, ldf, nullptr, Gate{}));
  if (x0) HGL_TRY(resid(Gate{}));
  if (has_prec) HGL_TRY(precond(b.R, ld, b.Zp, ld, b.part3, Gate{}));
  prof_begin(h, kProfStart, s);
  int rc = HGL_DISPATCH_SHAPE(cs, sizeof(T), {
    dim3 grid(h->n_tiles, cs.slabs);
    launch(h, -1, k_cg_init<T, GL, V>, grid, dim3(kBlock), 0, s, h->n_tiles, h->tile_r0,
                       h->tile_r1, nsl, h->n_long, Y, ldy, F, ldf, b.R, b.P, ld, b.part, b.part2, k,
                       x0 ? 1 : 0, has_prec ? static_cast<const T*>(b.Zp) : nullptr, b.pp, sdec, h->tile_seg,
                       a_seg);
    HGL_HIP(hipGetLastError());
    return HGL_OK;
  });
  HGL_TRY(rc);
  ra.iter = -1;
  launch(h, -1, k_cg_reduce<RedOp::Init>, dim3(red_blocks), dim3(kRedThreads), 0, s, ra, b.st, wd);
  HGL_HIP(hipGetLastError());
  prof_end(h, s);

  // ---------------------------------------------------------- iterations
  auto iteration = [&](int it) -> int {
    Gate g_prev{wd.cnt(it - 1), nullptr, 1};
    RedArgs r = ra;
    r.iter = it;
    const int periodic = (o->rr_period > 0 && (it + 1) % o->rr_period == 0) ? 1 : 0;
    // partial r'r of the recursive residual: set aside in part2 when the
    // periodic replacement below overwrites part
    double* part_rr = periodic ? b.part2 : b.part;
    if (fused) {
      // edge gather + hyperedge half of p'Mp -> alpha -> vertex gather with
      // the update (partial r'r of the new R)
      prof_begin(h, kProfEdge, s);
      HGL_TRY(launch_spmm_edge<T, T>(h, b.P, ld, b.Z, ld, k, cse, g_prev, s, b.epart));
      prof_end(h, s);
      prof_begin(h, kProfReduce, s);
      launch(h, -1, k_cg_reduce<RedOp::Alpha>, dim3(red_blocks), dim3(kRedThreads), 0, s, r, b.st, wd);
      HGL_HIP(hipGetLastError());
      prof_end(h, s);
      prof_begin(h, kProfVertex, s);
      HGL_TRY(launch_spmm_vertex<T, T>(h, VMode::Step, b.P, ld, b.Z, ld, nullptr, 0, nullptr, 0, a_seg, b_seg,
                                       part_rr, k, csv, g_prev, s, UpdArgs<T>{F, ldf, b.R, ld, b.st.alpha}));
      prof_end(h, s);
    } else {
      prof_begin(h, kProfEdge, s);
      HGL_TRY(launch_spmm_edge<T, T>(h, b.P, ld, b.Z, ld, k, cse, g_prev, s));
      prof_end(h, s);
      prof_begin(h, kProfVertex, s);
      HGL_TRY(launch_spmm_vertex<T, T>(h, VMode::ApplyDot, b.P, ld, b.Z, ld, nullptr, 0, b.Q, ld, a_seg,
                                       b_seg, b.part, k, csv, g_prev, s));
      prof_end(h, s);
      prof_begin(h, kProfReduce, s);
      launch(h, -1, k_cg_reduce<RedOp::Alpha>, dim3(red_blocks), dim3(kRedThreads), 0, s, r, b.st, wd);
      HGL_HIP(hipGetLastError());
      prof_end(h, s);
      prof_begin(h, kProfUpdate, s);
      int rc2 = HGL_DISPATCH_SHAPE(cs, sizeof(T), {
        dim3 grid(h->n_tiles, cs.slabs);
        launch(h, -1, k_cg_update<T, GL, V>, grid, dim3(kBlock), 0, s, h->n_tiles, h->tile_r0,
                           h->tile_r1, h->tile_seg, nsl, h->n_long, F, ldf, b.R, b.P, b.Q, ld,
                           b.st.alpha, part_rr, k, g_prev);
        HGL_HIP(hipGetLastError());
        return HGL_OK;
      });
      HGL_TRY(rc2);
      prof_end(h, s);
    }
    if (periodic) HGL_TRY(resid(g_prev));
    if (has_prec) HGL_TRY(precond(b.R, ld, b.Zp, ld, b.part3, g_prev));
    r.periodic = periodic;
    prof_begin(h, kProfReduce, s);
    launch(h, -1, k_cg_reduce<RedOp::Beta>, dim3(red_blocks), dim3(kRedThreads), 0, s, r, b.st, wd);
    HGL_HIP(hipGetLastError());
    prof_end(h, s);
    Gate g_now{wd.cnt(it), nullptr, 1};
    prof_begin(h, kProfDirection, s);
    const T* dir_src = has_prec ? b.Zp : b.R;
    int rc3 = HGL_DISPATCH_SHAPE(cs, sizeof(T), {
      dim3 grid(h->n_tiles, cs.slabs);
      launch(h, -1, k_cg_direction<T, GL, V>, grid, dim3(kBlock), 0, s, h->tile_r0, h->tile_r1,
                         h->tile_seg, dir_src, b.P, ld, b.st.beta, static_cast<const int32_t*>(b.st.state), k,
                         g_now, b.pp, 0, sdec);
      HGL_HIP(hipGetLastError());
      return HGL_OK;
    });
    prof_end(h, s);
    return rc3;
  };

  // Check step between iterations it-1 and it: recompute R = Y - M F with
  // FP64 accumulation (residual replacement); columns whose recomputed
  // residual meets tol are done, the others restart from it (restart(): P =
  // R, or the preconditioned residual, since beta = 0 for them).
  auto check = [&](int it_next) -> int {
    HGL_TRY(resid(Gate{}));
    if (has_prec) HGL_TRY(precond(b.R, ld, b.Zp, ld, b.part3, Gate{}));
    RedArgs r = ra;
    r.iter = it_next;
    prof_begin(h, kProfReduce, s);
    launch(h, -1, k_cg_reduce<RedOp::Check>, dim3(red_blocks), dim3(kRedThreads), 0, s, r, b.st, wd);
    HGL_HIP(hipGetLastError());
    prof_end(h, s);
    return HGL_OK;
  };
  auto restart = [&]() -> int {
    prof_begin(h, kProfDirection, s);
    const T* dir_src = has_prec ? b.Zp : b.R;
    int rc4 = HGL_DISPATCH_SHAPE(cs, sizeof(T), {
      dim3 grid(h->n_tiles, cs.slabs);
      launch(h, -1, k_cg_direction<T, GL, V>, grid, dim3(kBlock), 0, s, h->tile_r0, h->tile_r1,
                         h->tile_seg, dir_src, b.P, ld, b.st.beta, static_cast<const int32_t*>(b.st.state), k,
                         Gate{}, b.pp, 1, sdec);
      HGL_HIP(hipGetLastError());
      return HGL_OK;
    });
    prof_end(h, s);
    return rc4;
  };

  // Iterations are enqueued in chunks; between chunks the host reads the
  // number of columns still iterating (neither claimed nor finished) and
  // their largest recursive relative residual.  When no column iterates, a
  // check step decides every claimed column on its recomputed residual.
  // Iterations enqueued after the last claim are gated no-ops, so a chunk may
  // overshoot cheaply: the first is sized from the CG bound with
  // kappa(M) <= 1 + 1/lambda (the spectrum of L lies in [0, 1]), later ones
  // from the observed contraction rate (chunk = 0), or fixed (chunk > 0).
  double lam_min = lambdas[0];
  for (int g = 1; g < G; ++g) lam_min = std::min(lam_min, lambdas[g]);
  const double kappa = 1.0 + 1.0 / lam_min;
  const double rho = (std::sqrt(kappa) - 1.0) / (std::sqrt(kappa) + 1.0);
  auto chunk_for = [&](double r_now, double rate) {
    if (!(rate < 0.999) || !(r_now > 0.0)) return 4;
    const double m = std::ceil(std::log(claim * o->tol / r_now) / std::log(rate));
    return int(std::min(64.0, std::max(1.0, m)));
  };
  // The first chunk as a HIP graph: recorded on first use, replayed while
  // every argument it bakes in (pointers, sizes, options) is unchanged.
  const bool use_graph = o->graph != 0 && !h->prof_on;
  auto graph_chunk = [&](int n) -> int {
    auto u = [](const void* p) { return uint64_t(reinterpret_cast<uintptr_t>(p)); };
    uint64_t tol_bits;
    std::memcpy(&tol_bits, &o->tol, sizeof(tol_bits));
    std::vector<uint64_t> key = {
        sizeof(T), uint64_t(k), uint64_t(G), uint64_t(n), uint64_t(ldy), uint64_t(ldf), u(Y), u(F),
        u(h->ws_vec.p), u(h->ws_z.p), u(h->ws_z64.p), u(h->ws_part.p), u(h->ws_part2.p), u(h->ws_extra[0].p),
        u(h->ws_state.p), u(h->ws_chunk.p), u(h->ws_ab.p), u(h->ws_extra[5].p), u(prec ? prec->ctx : nullptr), uint64_t(o->rr_period),
        tol_bits, uint64_t(cs.GL), uint64_t(cs.V), uint64_t(cs.slabs), uint64_t(cse.GL), uint64_t(cse.V),
        uint64_t(cse.slabs), uint64_t(csv.GL), uint64_t(csv.V), uint64_t(csv.slabs), u(wd.base),
        uint64_t(o->max_iter)};
    if (prec) for (uint64_t v : prec->key) key.push_back(v);
    if (!h->cg_graph || key != h->cg_graph_key) {
      if (h->cg_graph) {
        HGL_HIP(hipGraphExecDestroy(h->cg_graph));
        h->cg_graph = nullptr;
      }
      if (!h->capture_stream) HGL_HIP(hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking));
      hipGraph_t graph = nullptr;
      s = h->capture_stream;
      HGL_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      int rc = HGL_OK;
      for (int c = 0; c < n && rc == HGL_OK; ++c) rc = iteration(c);
      const hipError_t e = hipStreamEndCapture(s, &graph);
      s = s_user;
      if (rc != HGL_OK) {
        if (graph) hipGraphDestroy(graph);
        return rc;
      }
      HGL_HIP(e);
      const hipError_t e2 = hipGraphInstantiate(&h->cg_graph, graph, nullptr, nullptr, 0);
      hipGraphDestroy(graph);
      HGL_HIP(e2);
      h->cg_graph_key = key;
    }
    HGL_HIP(hipGraphLaunch(h->cg_graph, s));
    return HGL_OK;
  };

  int it = 0;
  int n_chunks = 0, n_checks = 0, n_resumed = 0;
  // per-column results (relres [gk] FP64, then state and iteration counts
  // [2 gk] int32) in pinned memory after the first 8 words, which hold the
  // readback of the loop
  double* res_d = h->pinned_d + 8;
  bool results_read = false;
  bool all_done = false;
  double r_ref = -1.0;
  int it_ref = 0;
  int checked_at = -1;
  int next = o->chunk > 0 ? o->chunk : std::max(2, chunk_for(2.0 * std::sqrt(kappa), rho));
  while (!all_done && it < o->max_iter) {
    const int n = std::min(next, o->max_iter - it);
    ++n_chunks;
    if (use_graph && it == 0) {
      HGL_TRY(graph_chunk(n));
      it += n;
    } else {
      for (int c = 0; c < n; ++c, ++it) HGL_TRY(iteration(it));
    }
    // A chunk sized to reach the claim level (chunk = 0) is followed at once
    // by a check, so that the usual solve needs one host synchronisation: a
    // column still iterating at the check only has its residual replaced.
    const bool speculate = o->chunk <= 0;
    if (speculate) HGL_TRY(check(it));
    HGL_HIP(hipMemcpyAsync(h->pinned_i, wd.cnt(it - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HGL_HIP(hipMemcpyAsync(h->pinned_d, wd.rmax(it - 1), sizeof(double), hipMemcpyDeviceToHost, s));
    if (speculate) {
      HGL_HIP(hipMemcpyAsync(h->pinned_i + 1, wd.chk(it), sizeof(int32_t), hipMemcpyDeviceToHost, s));
      // the per-column results too: when this check finishes every column,
      // the solve ends on this one synchronisation
      HGL_HIP(hipMemcpyAsync(res_d, b.st.relres, sizeof(double) * gk, hipMemcpyDeviceToHost, s));
      HGL_HIP(hipMemcpyAsync(res_d + gk, b.st.state, sizeof(int32_t) * 2 * gk, hipMemcpyDeviceToHost, s));
    }
    HGL_HIP(hipStreamSynchronize(s));
    const int iterating = h->pinned_i[0];
    if (iterating == 0 && !speculate) {  // every column claimed, finished or broken down
      HGL_TRY(check(it));
      HGL_HIP(hipMemcpyAsync(h->pinned_i + 1, wd.chk(it), sizeof(int32_t), hipMemcpyDeviceToHost, s));
      HGL_HIP(hipStreamSynchronize(s));
    }
    if (speculate || iterating == 0) {
      checked_at = it;
      ++n_checks;
      all_done = h->pinned_i[1] == 0;
      results_read = all_done && speculate;
      if (!all_done) {
        ++n_resumed;
        HGL_TRY(restart());  // P = R for the restarted columns only
      }
    }
    if (iterating == 0) {
      next = o->chunk > 0 ? o->chunk : 2;  // columns that go on are close to the end
      r_ref = -1.0;
      continue;
    }
    const double r_now = h->pinned_d[0];
    const double rate = (r_ref > 0.0 && r_now > 0.0 && it > it_ref)
                            ? std::pow(r_now / r_ref, 1.0 / double(it - it_ref)) : rho;
    if (o->chunk <= 0) next = chunk_for(r_now, rate);
    r_ref = r_now;
    it_ref = it;
  }
  if (!all_done && checked_at != it) {
    HGL_TRY(check(it));  // record the true residual of every unfinished column
    ++n_checks;
  }
  h->last_cg[0] = it;
  h->last_cg[1] = n_chunks;
  h->last_cg[2] = n_checks;
  h->last_cg[3] = n_resumed;
  // ---------------------------------------------------------- results
  double* pd = res_d;
  if (!results_read) {
    HGL_HIP(hipMemcpyAsync(pd, b.st.relres, sizeof(double) * gk, hipMemcpyDeviceToHost, s));
    HGL_HIP(hipMemcpyAsync(pd + gk, b.st.state, sizeof(int32_t) * 2 * gk, hipMemcpyDeviceToHost, s));
    HGL_HIP(hipStreamSynchronize(s));
  }
  const int32_t* state_h = reinterpret_cast<const int32_t*>(pd + gk);
  const int32_t* iters_h = state_h + gk;
  bool breakdown = false, unconverged = false;
  for (size_t i = 0; i < gk; ++i) {
    if (state_h[i] == kBreakdown) breakdown = true;
    if (state_h[i] == kActive || state_h[i] == kClaimed || state_h[i] == kRestart) unconverged = true;
    if (relres_host) relres_host[i] = pd[i];
    if (iters_host) iters_host[i] = iters_h[i];
  }
  if (breakdown) {
    set_error("CG breakdown: p'Mp <= 0 or a non-finite value (negative weight or NaN input?)");
    return HGL_EBREAKDOWN;
  }
  return unconverged ? HGL_NOT_CONVERGED : HGL_OK;
}

int cg_run(hgl_handle* h, const double* lambdas, const hgl_cg_opts* o, const void* Y, int64_t ldy, void* F,
           int64_t ldf, int k, int32_t* iters_host, double* relres_host, const Precond* prec, hipStream_t s) {
  HGL_CHECK_ARG(h != nullptr, "handle is NULL");
  HGL_CHECK_ARG(o != nullptr, "opts is NULL");
  HGL_CHECK_ARG(lambdas != nullptr, "lambdas is NULL");
  for (int g = 0; g < h->G; ++g)
    HGL_CHECK_ARG(lambdas[g] > 0.0 && std::isfinite(lambdas[g]), "lambda must be > 0 (graph %d: %g)", g,
                  lambdas[g]);
  HGL_CHECK_ARG(o->tol > 0.0 && std::isfinite(o->tol), "tol must be > 0");
  HGL_CHECK_ARG(o->max_iter >= 1, "max_iter must be >= 1");
  HGL_CHECK_ARG(k >= 1, "k must be >= 1");
  HGL_CHECK_ARG(Y && F, "Y and F must not be NULL");
  HGL_CHECK_ARG(ldy >= k && ldf >= k, "leading dimensions must be >= k");
  HGL_CHECK_ARG(o->rr_period >= 0, "rr_period must be >= 0");
  if (o->mode == HGL_CG_PLAIN_F64)
    return run_cg<double>(h, lambdas, o, static_cast<const double*>(Y), ldy, static_cast<double*>(F),
                          ldf, k, iters_host, relres_host, prec, s);
  if (o->mode == HGL_CG_F32_F64DOT_RR)
    return run_cg<float>(h, lambdas, o, static_cast<const float*>(Y), ldy, static_cast<float*>(F), ldf,
                         k, iters_host, relres_host, prec, s);
  set_error("unknown CG mode %d", o->mode);
  return HGL_EINVAL;
}

}  // namespace hgl

using namespace hgl;

extern "C" int hgl_cg_solve(hgl_handle* h, double lambda, const hgl_cg_opts* opts, const void* Y,
                            int64_t ldy, void* F, int64_t ldf, int32_t k, int32_t* iters_host,
                            double* relres_host, hipStream_t stream) {
  clear_error();
  enter(h, stream);
  HGL_CHECK_ARG(h != nullptr, "handle is NULL");
  std::vector<double> lams(h->G, lambda);
  return cg_run(h, lams.data(), opts, Y, ldy, F, ldf, k, iters_host, relres_host, nullptr, stream);
}

extern "C" int hgl_cg_solve_batched(hgl_handle* h, const double* lambdas_host, const hgl_cg_opts* opts,
                                    const void* Y, int64_t ldy, void* F, int64_t ldf, int32_t k,
                                    int32_t* iters_host, double* relres_host, hipStream_t stream) {
  clear_error();
  enter(h, stream);
  return cg_run(h, lambdas_host, opts, Y, ldy, F, ldf, k, iters_host, relres_host, nullptr, stream);
}
