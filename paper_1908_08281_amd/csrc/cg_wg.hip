// One-workgroup conjugate gradient: the latency path for small hypergraphs.
//
// The paper's experiments solve one query vector per test image on a graph
// of a few thousand vertices (section 4); a multi-kernel CG step there is
// bound by the per-launch latency of its six kernels, not by memory.  Here
// one workgroup of 1024 threads runs a column's whole solve, eqs. 16-20
// with M = I + L/lambda, in a single launch, and the columns of Y are
// independent workgroups (one launch solves many queries at once).
//
// Per workgroup (column j):
//   LDS:    Ps[N]  (FP32) = s o p, the scaled direction the edge gather reads;
//           Z[E]   (FP64) = c_e u_e with u_e = sum_{v in e} s_v p_v (eq. 1).
//   global: the column's F, R and P in column-contiguous workspaces (each row
//           is read and written by the thread that owns it).
// One iteration: edge gather Z and the FP64 partial sum_e c_e u_e^2; one
// workgroup reduction gives p'Mp = a p'p - b sum_e c_e u_e^2 (the split of
// p'Mp used by the multi-kernel path, a = 1 + 1/lambda, b = 1/lambda) and
// alpha; the vertex gather forms (Mp)_v = a p_v - b s_v (H Z)_v and applies
// f += alpha p, r -= alpha Mp; a second reduction gives r'r and beta; the
// direction update p = r + beta p.  Short rows and hyperedges are summed by
// one thread each, two at a time with their loads issued together; rows with
// more than kLongRow hyperedges are split into the handle's chunks of at
// most kChunk entries and hyperedges with more than kLongEdge members are
// taken whole, each by a group of 16 lanes with 8 loads in flight per lane.
// Every sum has a fixed order, so results are bitwise repeatable.
//
// Convergence follows the FP32 mode of the multi-kernel solver: when the
// recursive residual reaches claim * tol, the true residual Y - M F is
// recomputed with FP64 accumulation; the column finishes if it meets tol,
// and otherwise restarts from it (beta = 0).
#include <cmath>

#include "common.h"

namespace hgl {
namespace {

constexpr int kWg = 1024;
constexpr int kWgWaves = kWg / 64;
constexpr int kWgGather = 8;  // gathered entries in flight per thread and row
constexpr int kGrp = 16;      // lanes of a group summing one long row chunk or hyperedge
constexpr int kGroups = kWg / kGrp;
constexpr int kPerLane = kChunk / kGrp;  // entries in flight per lane of a group
// dynamic LDS of one workgroup (Ps and Z); the rest of the 160 KB holds the
// reduction scratch
constexpr size_t kWgLdsMax = 159 * 1024;

struct WgArgs {
  int32_t N, E;
  const int32_t* edge_ptr;
  const int32_t* edge_vtx;
  const int32_t* vtx_ptr;
  const int32_t* vtx_edge;
  const float* s;
  const float* c;
  const int32_t* long_edge;
  int32_t n_long_edge;
  const int32_t* long_row;
  int32_t n_long;
  const int32_t* long_chunk0;  // [n_long + 1] first chunk of each long row
  const int32_t* chunk_begin;  // [n_chunks] entry range in vtx_edge
  const int32_t* chunk_end;
  int32_t n_chunks;
  const float* Y;
  int64_t ldy;
  float* F;        // caller's F (row-major, ldf): x0 on entry when x0 != 0, result on exit
  int64_t ldf;
  float* Fw;       // workspaces [k][N], column j at j * N
  float* Rw;
  float* Pw;
  double a, b, tol2, claim2;
  int32_t max_iter, x0;
  int32_t* iters;
  double* relres;
  int32_t* status;
};

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
  return x;
}

// Sum over a group of kGrp consecutive lanes (fixed butterfly).
__device__ __forceinline__ double grp_sum(double x) {
#pragma unroll
  for (int m = kGrp / 2; m >= 1; m >>= 1) x += __shfl_xor(x, m);
  return x;
}

// Workgroup sums of x and y, identical in every thread (fixed order: a
// lane butterfly per wave, then the waves' sums in wave order).
__device__ __forceinline__ void wg_sum2(double& x, double& y, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  x = wave_sum(x);
  y = wave_sum(y);
  if (lane == 0) {
    red[wave] = x;
    red[kWgWaves + wave] = y;
  }
  __syncthreads();
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int w = 0; w < kWgWaves; ++w) {
    sx += red[w];
    sy += red[kWgWaves + w];
  }
  __syncthreads();  // red is reused by the next call
  x = sx;
  y = sy;
}

// Sum of val[idx[b + q]] over q in [q0, m), kWgGather entries in flight.
template <class TV>
__device__ __forceinline__ double row_tail(const int32_t* idx, const TV* val, int b, int q0, int m) {
  double acc = 0.0;
  for (int q = q0; q < m; q += kWgGather) {
    int j[kWgGather];
#pragma unroll
    for (int u = 0; u < kWgGather; ++u) j[u] = q + u < m ? idx[b + q + u] : -1;
#pragma unroll
    for (int u = 0; u < kWgGather; ++u) acc += j[u] >= 0 ? double(val[j[u]]) : 0.0;
  }
  return acc;
}

// Short CSR rows (at most `lim` entries), two rows per thread at a time
// (rows r and r + kWg): the offsets of both rows, then the first kWgGather
// entries of both, are issued before either is consumed, so a thread waits
// about twice per two rows instead of twice per row.  For each row r < n
// with at most lim entries, calls f(r, sum of val[idx[j]] over its entries,
// in entry order).
template <class TV, class Fn>
__device__ __forceinline__ void short_rows(int n, const int32_t* ptr, const int32_t* idx, const TV* val, int lim,
                                           Fn&& f) {
  for (int r0 = threadIdx.x; r0 < n; r0 += 2 * kWg) {
    const int r1 = r0 + kWg;
    const int b0 = ptr[r0];
    int m0 = ptr[r0 + 1] - b0;
    const int b1 = r1 < n ? ptr[r1] : 0;
    int m1 = r1 < n ? ptr[r1 + 1] - b1 : 0;
    if (m0 > lim) m0 = -1;  // a long row: done elsewhere
    if (m1 > lim) m1 = -1;
    int j0[kWgGather], j1[kWgGather];
#pragma unroll
    for (int u = 0; u < kWgGather; ++u) {
      j0[u] = u < m0 ? idx[b0 + u] : -1;
      j1[u] = u < m1 ? idx[b1 + u] : -1;
    }
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int u = 0; u < kWgGather; ++u) {
      a0 += j0[u] >= 0 ? double(val[j0[u]]) : 0.0;
      a1 += j1[u] >= 0 ? double(val[j1[u]]) : 0.0;
    }
    if (m0 > kWgGather) a0 += row_tail(idx, val, b0, kWgGather, m0);
    if (m1 > kWgGather) a1 += row_tail(idx, val, b1, kWgGather, m1);
    if (m0 >= 0) f(r0, a0);
    if (m1 >= 0 && r1 < n) f(r1, a1);
  }
}

// Sum of val[idx[j]] over j in [b, en) by a group of kGrp lanes: lane gl
// takes j = b + gl + kGrp u (kPerLane entries in flight per batch); the
// result is valid in every lane of the group.
template <class TV>
__device__ __forceinline__ double group_range(const int32_t* idx, const TV* val, int b, int en, int gl) {
  double acc = 0.0;
  for (int j0 = b; j0 < en; j0 += kGrp * kPerLane) {
    int j[kPerLane];
#pragma unroll
    for (int u = 0; u < kPerLane; ++u) {
      const int q = j0 + gl + kGrp * u;
      j[u] = q < en ? idx[q] : -1;
    }
#pragma unroll
    for (int u = 0; u < kPerLane; ++u) acc += j[u] >= 0 ? double(val[j[u]]) : 0.0;
  }
  return grp_sum(acc);
}

// Z_e = c_e u_e, u_e = sum_{v in e} Ps_v, for every hyperedge; returns this
// thread's share of sum_e c_e u_e^2.  Ends with a barrier (Z complete).
__device__ __forceinline__ double edge_phase(const WgArgs& A, const float* Ps, double* Z) {
  const int g = threadIdx.x / kGrp, gl = threadIdx.x % kGrp;
  double ep = 0.0;
  // hyperedges with more than kLongEdge members: a group each
  for (int i = g; i < A.n_long_edge; i += kGroups) {
    const int e = A.long_edge[i];
    const double u = group_range(A.edge_vtx, Ps, A.edge_ptr[e], A.edge_ptr[e + 1], gl);
    if (gl == 0) {
      const double z = double(A.c[e]) * u;
      Z[e] = z;
      ep += u * z;
    }
  }
  short_rows(A.E, A.edge_ptr, A.edge_vtx, Ps, kLongEdge, [&](int e, double u) {
    const double z = double(A.c[e]) * u;
    Z[e] = z;
    ep += u * z;
  });
  __syncthreads();
  return ep;
}

// Calls f(v, (H Z)_v) once for every row.  Rows with more than kLongRow
// hyperedges are split into the handle's chunks of at most kChunk entries:
// a group sums each chunk into cpart, and after a barrier thread i adds long
// row i's chunks in order.  Ends with the calls of the long rows (no barrier
// after them).
template <class Fn>
__device__ __forceinline__ void vertex_phase(const WgArgs& A, const double* Z, double* cpart, Fn&& f) {
  const int g = threadIdx.x / kGrp, gl = threadIdx.x % kGrp;
  for (int ch = g; ch < A.n_chunks; ch += kGroups) {
    const double hz = group_range(A.vtx_edge, Z, A.chunk_begin[ch], A.chunk_end[ch], gl);
    if (gl == 0) cpart[ch] = hz;
  }
  short_rows(A.N, A.vtx_ptr, A.vtx_edge, Z, kLongRow, f);
  __syncthreads();  // chunk sums complete
  for (int i = threadIdx.x; i < A.n_long; i += kWg) {
    double hz = 0.0;
    for (int c = A.long_chunk0[i]; c < A.long_chunk0[i + 1]; ++c) hz += cpart[c];
    f(A.long_row[i], hz);
  }
}

__global__ __launch_bounds__(kWg) void k_cg_wg(WgArgs A) {
  extern __shared__ __align__(16) unsigned char wg_lds[];
  __shared__ double red[2 * kWgWaves];
  const int tid = threadIdx.x;
  const int col = blockIdx.x;
  const int N = A.N;
  float* Ps = reinterpret_cast<float*>(wg_lds);
  double* Z = reinterpret_cast<double*>(wg_lds + ((size_t(N) * sizeof(float) + 15) & ~size_t(15)));
  double* cpart = Z + A.E;  // [n_chunks] chunk sums of the long rows
  float* Fw = A.Fw + int64_t(col) * N;
  float* Rw = A.Rw + int64_t(col) * N;
  float* Pw = A.Pw + int64_t(col) * N;
  const float* Y = A.Y + col;
  const double a = A.a, bb = A.b;

  // ||y||^2
  double yy = 0.0, unused = 0.0;
  for (int v = tid; v < N; v += kWg) {
    const double y = Y[int64_t(v) * A.ldy];
    yy += y * y;
  }
  wg_sum2(yy, unused, red);
  if (yy == 0.0) {  // zero column: f = 0 exactly
    for (int v = tid; v < N; v += kWg) A.F[int64_t(v) * A.ldf + col] = 0.f;
    if (tid == 0) {
      A.iters[col] = 0;
      A.relres[col] = 0.0;
      A.status[col] = 0;
    }
    return;
  }

  // True residual R = Y - M F with FP64 accumulation, then the restart
  // direction P = R; returns r'r (FP64 values) in rr and p'p in pp.
  auto check = [&](double& rr, double& pp) {
    for (int v = tid; v < N; v += kWg) Ps[v] = A.s[v] * Fw[v];
    __syncthreads();
    edge_phase(A, Ps, Z);
    double r2 = 0.0;
    vertex_phase(A, Z, cpart, [&](int v, double hz) {
      const double f = Fw[v];
      const double rt = double(Y[int64_t(v) * A.ldy]) - (a * f - bb * double(A.s[v]) * hz);
      Rw[v] = float(rt);
      r2 += rt * rt;
    });
    __syncthreads();  // R of the long rows (written by wave lanes) before the direction
    double p2 = 0.0;
    for (int v = tid; v < N; v += kWg) {
      const float p = Rw[v];
      Pw[v] = p;
      Ps[v] = A.s[v] * p;
      p2 += double(p) * double(p);
    }
    wg_sum2(r2, p2, red);  // its barriers also publish Ps
    rr = r2;
    pp = p2;
  };

  double rr, pp;
  if (A.x0) {
    for (int v = tid; v < N; v += kWg) Fw[v] = A.F[int64_t(v) * A.ldf + col];
    __syncthreads();
    check(rr, pp);
  } else {
    double p2 = 0.0;
    for (int v = tid; v < N; v += kWg) {
      const float y = Y[int64_t(v) * A.ldy];
      Fw[v] = 0.f;
      Rw[v] = y;
      Pw[v] = y;
      Ps[v] = A.s[v] * y;
      p2 += double(y) * double(y);
    }
    double r2 = p2;
    wg_sum2(r2, p2, red);
    rr = r2;
    pp = p2;
  }

  int it = 0, st = 1;
  double rel2 = rr / yy;
  bool fresh = A.x0 != 0;  // rr is a true residual (just checked)
  for (;;) {
    if (rr <= A.claim2 * yy || it >= A.max_iter) {
      double rt = rr, p2 = pp;
      if (!fresh) check(rt, p2);
      rel2 = rt / yy;
      if (rel2 <= A.tol2) {
        st = 0;
        break;
      }
      if (it >= A.max_iter || !(rel2 == rel2)) {
        st = rel2 == rel2 ? 1 : -4;
        break;
      }
      rr = rt;  // restart from the true residual (beta = 0); rt > tol^2 yy > claim^2 yy
      pp = p2;
      fresh = true;
    }
    fresh = false;
    // p'Mp = a p'p - b sum_e c_e u_e^2
    double ep = edge_phase(A, Ps, Z);
    double unused2 = 0.0;
    wg_sum2(ep, unused2, red);
    const double pmp = a * pp - bb * ep;
    if (!(pmp > 0.0) || !std::isfinite(pmp)) {
      st = -4;
      break;
    }
    const double alpha = rr / pmp;
    const float al = float(alpha);
    double r2 = 0.0;
    vertex_phase(A, Z, cpart, [&](int v, double hz) {
      const float p = Pw[v];
      const double q = a * double(p) - bb * double(A.s[v]) * hz;
      const float f = Fw[v] + al * p;
      const float r = Rw[v] - float(alpha * q);
      Fw[v] = f;
      Rw[v] = r;
      r2 += double(r) * double(r);
    });
    double unused3 = 0.0;
    wg_sum2(r2, unused3, red);  // also orders the long rows' R before the direction
    ++it;
    const double beta = r2 / rr;
    rr = r2;
    if (rr <= A.claim2 * yy || it >= A.max_iter) continue;  // the check restarts or finishes
    const float be = float(beta);
    double p2 = 0.0;
    for (int v = tid; v < N; v += kWg) {
      const float p = Rw[v] + be * Pw[v];
      Pw[v] = p;
      Ps[v] = A.s[v] * p;
      p2 += double(p) * double(p);
    }
    double unused4 = 0.0;
    wg_sum2(p2, unused4, red);  // its barriers publish Ps to the edge gather
    pp = p2;
  }

  for (int v = tid; v < N; v += kWg) A.F[int64_t(v) * A.ldf + col] = Fw[v];
  if (tid == 0) {
    A.iters[col] = it;
    A.relres[col] = std::sqrt(rel2);
    A.status[col] = st;
  }
}

}  // namespace

size_t cg_wg_lds_bytes(int N, int E, int n_chunks) {
  return ((size_t(N) * sizeof(float) + 15) & ~size_t(15)) + (size_t(E) + size_t(n_chunks)) * sizeof(double);
}

}  // namespace hgl

using namespace hgl;

extern "C" int hgl_cg_solve_wg(hgl_handle* h, double lambda, const hgl_cg_opts* o, const float* Y, int64_t ldy,
                               float* F, int64_t ldf, int32_t k, int32_t* iters_host, double* relres_host,
                               hipStream_t s) {
  clear_error();
  HGL_CHECK_ARG(h != nullptr && o != nullptr, "handle and opts must not be NULL");
  HGL_CHECK_ARG(h->G == 1, "the one-workgroup solver needs a single-graph handle");
  HGL_CHECK_ARG(lambda > 0.0 && std::isfinite(lambda), "lambda must be > 0 (%g)", lambda);
  HGL_CHECK_ARG(o->tol > 0.0 && std::isfinite(o->tol), "tol must be > 0");
  HGL_CHECK_ARG(o->max_iter >= 1, "max_iter must be >= 1");
  HGL_CHECK_ARG(k >= 1, "k must be >= 1");
  HGL_CHECK_ARG(Y && F, "Y and F must not be NULL");
  HGL_CHECK_ARG(ldy >= k && ldf >= k, "leading dimensions must be >= k");
  if (o->mode != HGL_CG_F32_F64DOT_RR) {
    set_error("the one-workgroup solver runs the FP32 mode only (mode %d)", o->mode);
    return HGL_EUNSUPPORTED;
  }
  const size_t lds = cg_wg_lds_bytes(h->N, h->E, h->n_chunks);
  if (lds > kWgLdsMax) {
    set_error("graph too large for the one-workgroup solver: N = %d, E = %d need %zu B of LDS (at most %zu)",
              h->N, h->E, lds, kWgLdsMax);
    return HGL_EUNSUPPORTED;
  }
  const size_t vec = sizeof(float) * size_t(h->N) * k;
  HGL_TRY(h->ws_vec.reserve(3 * vec + 256));
  HGL_TRY(h->ws_state.reserve(size_t(k) * (sizeof(double) + 2 * sizeof(int32_t)) + 64));
  HGL_TRY(ensure_pinned(h, 2 * size_t(k)));
  float* base = h->ws_vec.as<float>();
  double* relres_d = h->ws_state.as<double>();
  int32_t* iters_d = reinterpret_cast<int32_t*>(relres_d + k);
  int32_t* status_d = iters_d + k;
  WgArgs A;
  A.N = h->N;
  A.E = h->E;
  A.edge_ptr = h->edge_ptr;
  A.edge_vtx = h->edge_vtx;
  A.vtx_ptr = h->vtx_ptr;
  A.vtx_edge = h->vtx_edge;
  A.s = h->s32;
  A.c = h->c32;
  A.long_edge = h->long_edge;
  A.n_long_edge = h->n_long_edge;
  A.long_row = h->long_row;
  A.n_long = h->n_long;
  A.long_chunk0 = h->long_chunk0;
  A.chunk_begin = h->chunk_begin;
  A.chunk_end = h->chunk_end;
  A.n_chunks = h->n_chunks;
  A.Y = Y;
  A.ldy = ldy;
  A.F = F;
  A.ldf = ldf;
  A.Fw = base;
  A.Rw = base + size_t(h->N) * k;
  A.Pw = base + 2 * size_t(h->N) * k;
  A.a = 1.0 + 1.0 / lambda;
  A.b = 1.0 / lambda;
  A.tol2 = o->tol * o->tol;
  A.claim2 = 0.25 * A.tol2;  // claims at tol / 2, as the multi-kernel FP32 mode
  A.max_iter = o->max_iter;
  A.x0 = o->x0_given ? 1 : 0;
  A.iters = iters_d;
  A.relres = relres_d;
  A.status = status_d;
  if (lds > 64 * 1024)
    HGL_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_cg_wg), hipFuncAttributeMaxDynamicSharedMemorySize,
                                int(lds)));
  launch(h, -1, k_cg_wg, dim3(k), dim3(kWg), uint32_t(lds), s, A);
  HGL_HIP(hipGetLastError());
  double* pd = h->pinned_d;
  HGL_HIP(hipMemcpyAsync(pd, relres_d, sizeof(double) * k + 2 * sizeof(int32_t) * k, hipMemcpyDeviceToHost, s));
  HGL_HIP(hipStreamSynchronize(s));
  const int32_t* pi = reinterpret_cast<const int32_t*>(pd + k);
  int rc = HGL_OK;
  for (int j = 0; j < k; ++j) {
    if (relres_host) relres_host[j] = pd[j];
    if (iters_host) iters_host[j] = pi[j];
    const int32_t st = pi[k + j];
    if (st == -4) rc = HGL_EBREAKDOWN;
    else if (st == 1 && rc == HGL_OK) rc = HGL_NOT_CONVERGED;
  }
  if (rc == HGL_EBREAKDOWN) set_error("CG breakdown (p'Mp <= 0 or not finite) in a column");
  return rc;
}
