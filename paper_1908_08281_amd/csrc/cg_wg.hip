// One-workgroup conjugate gradient: the latency path for small hypergraphs.
//
// The paper's experiments solve one query vector per test image on a graph
// of a few thousand vertices (section 4); a multi-kernel CG step there is
// bound by the per-launch latency of its six kernels, not by memory.  Here
// one workgroup of 1024 threads runs a column's whole solve, eqs. 16-20
// with M = I + L/lambda, in a single launch, and the columns of Y are
// independent workgroups (one launch solves many queries at once).
//
// Each thread owns an even share (at most kSlots entries) of each CSR of H,
// edge-major and vertex-major: 16-bit indices, a bitmask of the entries that
// end a row, the length of a leading run that continues a row begun in an
// earlier thread's share, the ordinal of its first row that starts in the
// share, and the number of following threads that its last row runs into.
// A gather loads its thread's share (19 independent words from a table that
// stays in L2) and then works from LDS only.  The vectors f, r, p and the
// scale s of a thread's kRowsPT vertex rows (v = thread + i * 1024) and c of
// its kEdgesPT hyperedges stay in registers for the whole solve.
// LDS holds Ps = s o p (FP64), U / Z over the hyperedges (FP64), H Z over the
// vertex rows that have hyperedges (FP64), one carry word per thread and the
// column of Y (FP32, read again by the residual checks).
//
// One iteration: the edge gather u_e = sum_{v in e} s_v p_v (each thread
// sums its share; rows that cross shares are finished by adding the
// following threads' leading partial sums, in thread order), Z_e = c_e u_e
// and the FP64 partial sum_e c_e u_e^2 by the hyperedge owners; one
// workgroup reduction gives p'Mp = a p'p - b sum_e c_e u_e^2 (the split of
// p'Mp used by the multi-kernel path, a = 1 + 1/lambda, b = 1/lambda) and
// alpha; the vertex gather (H Z)_v the same way; the row owners form
// (Mp)_v = a p_v - b s_v (H Z)_v and apply f += alpha p, r -= alpha Mp; a
// second reduction gives r'r and beta; the owners update p = r + beta p.
// Every sum has a fixed order, so results are bitwise repeatable.
//
// Convergence follows the FP32 mode of the multi-kernel solver: when the
// recursive residual reaches tol/2, the true residual Y - M F is recomputed
// with FP64 accumulation (s o f in FP64); the column finishes if it meets
// tol, and otherwise restarts from it (beta = 0).
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "common.h"

namespace hgl {
namespace {

constexpr int kWg = 1024;
constexpr int kWgWaves = kWg / 64;
constexpr int kSlots = 32;             // CSR entries per thread (per CSR)
constexpr int kSlotW = kSlots / 2;     // words of packed 16-bit indices
constexpr int kTabCsr = kSlotW + 3;    // table words per thread and CSR
constexpr int kRowsPT = 6;             // vertex rows owned per thread (N <= 6144)
constexpr int kEdgesPT = 6;            // hyperedges owned per thread (E <= 6144)
constexpr size_t kWgLdsMax = 159 * 1024;

struct WgArgs {
  int32_t N, E, nq;
  const uint32_t* tab_e;  // edge-major CSR share table [kTabCsr][kWg]
  const uint32_t* tab_v;  // vertex-major CSR share table [kTabCsr][kWg]
  const int32_t* rowq;    // [kRowsPT][kWg] ordinal of row (thread + i kWg) among rows with hyperedges, or -1
  const float* s;
  const float* c;
  const float* Y;
  int64_t ldy;
  float* F;  // x0 on entry when x0 != 0, the result on exit (row-major, ldf)
  int64_t ldf;
  double a, b, tol2, claim2;
  int32_t max_iter, x0;
  int32_t* iters;
  double* relres;
  int32_t* status;
};

// A thread's share of one CSR (see the table layout in share_table).
struct Share {
  uint32_t w[kSlotW];
  uint32_t q0;    // ordinal of the first row that starts in the share
  uint32_t hm;    // head | cnt << 6 | span << 12
  uint32_t mask;  // bit i: entry i ends its row
};

__device__ __forceinline__ void load_share(const uint32_t* tab, Share& sh) {
  const int t = threadIdx.x;
#pragma unroll
  for (int w = 0; w < kSlotW; ++w) sh.w[w] = tab[w * kWg + t];
  sh.q0 = tab[kSlotW * kWg + t];
  sh.hm = tab[(kSlotW + 1) * kWg + t];
  sh.mask = tab[(kSlotW + 2) * kWg + t];
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
  return x;
}

// Workgroup sums of x and y, identical in every thread, in a fixed order:
// a lane butterfly per wave, then wave 0's first kWgWaves lanes add the
// waves' sums by a butterfly of their own and broadcast the two totals.
// red: 2 * kWgWaves + 2 doubles.
__device__ __forceinline__ void wg_sum2(double& x, double& y, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  x = wave_sum(x);
  y = wave_sum(y);
  if (lane == 0) {
    red[wave] = x;
    red[kWgWaves + wave] = y;
  }
  __syncthreads();
  if (wave == 0) {
    double sx = lane < kWgWaves ? red[lane] : 0.0;
    double sy = lane < kWgWaves ? red[kWgWaves + lane] : 0.0;
#pragma unroll
    for (int m = kWgWaves / 2; m >= 1; m >>= 1) {
      sx += __shfl_xor(sx, m);
      sy += __shfl_xor(sy, m);
    }
    if (lane == 0) {
      red[2 * kWgWaves] = sx;
      red[2 * kWgWaves + 1] = sy;
    }
  }
  __syncthreads();
  x = red[2 * kWgWaves];
  y = red[2 * kWgWaves + 1];
  __syncthreads();  // red is reused by the next call
}

// Row sums of val over one CSR: out[q] = sum of val[idx] over row q's
// entries, in entry order.  A thread sums its share (tab: the CSR's share
// table); a row that starts in it and runs on is finished, after a barrier,
// by adding the leading partial sums (carry) of the following `span` threads
// in thread order.  Ends with a barrier (out complete).
template <class TV, class TO>
__device__ __attribute__((noinline)) void share_gather(const uint32_t* tab, const TV* val, TO* out, double* carry) {
  Share sh;
  load_share(tab, sh);
  const int head = int(sh.hm & 63u), cnt = int((sh.hm >> 6) & 63u), span = int(sh.hm >> 12);
  double acc = 0.0, lead = 0.0;
  int q = int(sh.q0);
#pragma unroll
  for (int i = 0; i < kSlots; ++i) {
    if (i < cnt) {
      acc += double(val[(sh.w[i >> 1] >> ((i & 1) * 16)) & 0xffffu]);
      if ((sh.mask >> i) & 1u) {
        if (i < head) {
          lead = acc;  // the end of a row begun in an earlier share
        } else {
          out[q] = TO(acc);
          ++q;
        }
        acc = 0.0;
      }
    }
    // at most 8 LDS loads in flight: the whole share at once would need 64
    // registers for its values and spill the solver's vectors
    if ((i & 7) == 7) __builtin_amdgcn_sched_barrier(0);
  }
  const bool open = cnt > 0 && !((sh.mask >> (cnt - 1)) & 1u);  // the last row runs on
  if (open && head == cnt) lead = acc;                          // the whole share is inside one row
  carry[threadIdx.x] = lead;
  __syncthreads();
  if (open && head < cnt) {
    // four interleaved partial sums (a fixed order), so the loads of a long
    // span overlap
    double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
    const double* cs = carry + threadIdx.x + 1;
    int u = 0;
    for (; u + 4 <= span; u += 4) {
      t0 += cs[u];
      t1 += cs[u + 1];
      t2 += cs[u + 2];
      t3 += cs[u + 3];
    }
    for (; u < span; ++u) t0 += cs[u];
    out[q] = TO(acc + ((t0 + t1) + (t2 + t3)));
  }
  __syncthreads();
}

__global__ __launch_bounds__(kWg) void k_cg_wg(WgArgs A) {
  extern __shared__ __align__(16) double wg_lds[];
  __shared__ double red[2 * kWgWaves + 2];
  const int tid = threadIdx.x, col = blockIdx.x;
  const int N = A.N, E = A.E;
  // Ps and U hold FP32 values during the iterations and FP64 values in the
  // residual checks (the same bytes; FP64 needs the full regions)
  double* Psd = wg_lds;       // [N]  s o f (checks)
  double* Ud = Psd + N;       // [E]  u_e, then Z_e = c_e u_e (checks)
  float* Psf = reinterpret_cast<float*>(Psd);  // s o p (iterations)
  float* Uf = reinterpret_cast<float*>(Ud);    // u_e, then Z_e (iterations)
  double* HZ = Ud + E;        // [nq]
  double* carry = HZ + A.nq;  // [kWg]
  float* Ys = reinterpret_cast<float*>(carry + kWg);  // [N]
  float s[kRowsPT], f[kRowsPT], r[kRowsPT], p[kRowsPT], ce[kEdgesPT];
  int qv[kRowsPT];
#pragma unroll
  for (int i = 0; i < kRowsPT; ++i) {
    const int v = tid + i * kWg;
    s[i] = v < N ? A.s[v] : 0.f;
    qv[i] = A.rowq[i * kWg + tid];
    f[i] = r[i] = p[i] = 0.f;
  }
#pragma unroll
  for (int i = 0; i < kEdgesPT; ++i) {
    const int e = tid + i * kWg;
    ce[i] = e < E ? A.c[e] : 0.f;
  }
  const float* Y = A.Y + col;
  const double a = A.a, bb = A.b;

  // ||y||^2; the column of Y into LDS
  double yy = 0.0, unused = 0.0;
#pragma unroll
  for (int i = 0; i < kRowsPT; ++i) {
    const int v = tid + i * kWg;
    if (v < N) {
      const float y = Y[int64_t(v) * A.ldy];
      Ys[v] = y;
      yy += double(y) * double(y);
    }
  }
  wg_sum2(yy, unused, red);
  if (yy == 0.0) {  // zero column: f = 0 exactly
#pragma unroll
    for (int i = 0; i < kRowsPT; ++i) {
      const int v = tid + i * kWg;
      if (v < N) A.F[int64_t(v) * A.ldf + col] = 0.f;
    }
    if (tid == 0) {
      A.iters[col] = 0;
      A.relres[col] = 0.0;
      A.status[col] = 0;
    }
    return;
  }

  // Edge gather from Ps (complete on entry; T = float in the iterations,
  // double in the checks): Z in U; returns this thread's share of
  // sum_e c_e u_e^2.  Z is complete after the caller's next barrier.
  auto edge_phase = [&](auto* Ps, auto* U) __attribute__((always_inline)) -> double {
    using T = std::remove_pointer_t<decltype(U)>;
    share_gather(A.tab_e, Ps, U, carry);
    double ep = 0.0;
#pragma unroll
    for (int i = 0; i < kEdgesPT; ++i) {
      const int e = tid + i * kWg;
      if (e < E) {
        const double u = U[e];
        const double z = double(ce[i]) * u;
        U[e] = T(z);
        ep += u * z;
      }
    }
    return ep;
  };
  // Vertex gather from Z (complete on entry); fn(i, v, (H Z)_v) per owned row.
  auto vertex_phase = [&](auto* U, auto&& fn) __attribute__((always_inline)) {
    share_gather(A.tab_v, U, HZ, carry);
#pragma unroll
    for (int i = 0; i < kRowsPT; ++i) {
      const int v = tid + i * kWg;
      if (v < N) fn(i, v, qv[i] >= 0 ? HZ[qv[i]] : 0.0);
    }
  };
  // True residual r = y - M f with FP64 accumulation, then the restart
  // direction p = r; returns r'r (FP64 values) in rr and p'p in pp.
  auto check = [&](double& rr, double& pp) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < kRowsPT; ++i) {
      const int v = tid + i * kWg;
      if (v < N) Psd[v] = double(s[i]) * double(f[i]);
    }
    __syncthreads();
    edge_phase(Psd, Ud);
    __syncthreads();  // Z complete
    double r2 = 0.0, p2 = 0.0;
    vertex_phase(Ud, [&](int i, int v, double hz) __attribute__((always_inline)) {
      const double rt = double(Ys[v]) - (a * double(f[i]) - bb * double(s[i]) * hz);
      r[i] = float(rt);
      p[i] = r[i];
      Psf[v] = float(double(s[i]) * double(p[i]));  // Psd is no longer read
      r2 += rt * rt;
      p2 += double(p[i]) * double(p[i]);
    });
    wg_sum2(r2, p2, red);  // its barriers publish Ps
    rr = r2;
    pp = p2;
  };

  double rr = 0.0, pp = 0.0;
  bool need_check = A.x0 != 0;  // a given start is checked (and restarted from) first
  if (A.x0) {
#pragma unroll
    for (int i = 0; i < kRowsPT; ++i) {
      const int v = tid + i * kWg;
      if (v < N) f[i] = A.F[int64_t(v) * A.ldf + col];
    }
  } else {
    double p2 = 0.0;
#pragma unroll
    for (int i = 0; i < kRowsPT; ++i) {
      const int v = tid + i * kWg;
      if (v < N) {
        const float y = Ys[v];
        r[i] = p[i] = y;
        Psf[v] = float(double(s[i]) * double(y));
        p2 += double(y) * double(y);
      }
    }
    double r2 = p2;
    wg_sum2(r2, p2, red);
    rr = r2;
    pp = p2;
  }

  int it = 0, st = 1;
  double rel2 = 1.0;
  for (;;) {
    if (need_check || rr <= A.claim2 * yy || it >= A.max_iter) {
      double rt, p2;
      check(rt, p2);
      need_check = false;
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
    }
    // p'Mp = a p'p - b sum_e c_e u_e^2
    double ep = edge_phase(Psf, Uf);
    double unused2 = 0.0;
    wg_sum2(ep, unused2, red);  // its barriers complete Z
    const double pmp = a * pp - bb * ep;
    if (!(pmp > 0.0) || !std::isfinite(pmp)) {
      st = -4;
      break;
    }
    const double alpha = rr / pmp;
    const float al = float(alpha);
    double r2 = 0.0;
    vertex_phase(Uf, [&](int i, int, double hz) __attribute__((always_inline)) {
      const double q = a * double(p[i]) - bb * double(s[i]) * hz;
      f[i] += al * p[i];
      r[i] -= float(alpha * q);
      r2 += double(r[i]) * double(r[i]);
    });
    double unused3 = 0.0;
    wg_sum2(r2, unused3, red);
    ++it;
    const double beta = r2 / rr;
    rr = r2;
    if (rr <= A.claim2 * yy || it >= A.max_iter) continue;  // the check restarts or finishes
    const float be = float(beta);
    double p2 = 0.0;
#pragma unroll
    for (int i = 0; i < kRowsPT; ++i) {
      const int v = tid + i * kWg;
      if (v < N) {
        p[i] = r[i] + be * p[i];
        Psf[v] = float(double(s[i]) * double(p[i]));
        p2 += double(p[i]) * double(p[i]);
      }
    }
    double unused4 = 0.0;
    wg_sum2(p2, unused4, red);  // its barriers publish Ps to the edge gather
    pp = p2;
  }

#pragma unroll
  for (int i = 0; i < kRowsPT; ++i) {
    const int v = tid + i * kWg;
    if (v < N) A.F[int64_t(v) * A.ldf + col] = f[i];
  }
  if (tid == 0) {
    A.iters[col] = it;
    A.relres[col] = std::sqrt(rel2);
    A.status[col] = st;
  }
}

// Share table of one CSR with `rows` rows (ptr [rows+1], idx [nnz]) into
// out [kTabCsr][kWg]: thread t takes entries [t nnz / kWg, (t+1) nnz / kWg).
// Word layout per thread: kSlotW words of 16-bit index pairs (entry 2w in
// the low half), q0 = ordinal (ord[row]) of the first row that starts in the
// share, hm = head | cnt << 6 | span << 12 (head: leading entries that end or
// continue a row begun earlier; cnt: entries; span: following threads that
// the share's last row runs into), mask: bit i when entry i ends its row.
// Returns false if a share exceeds kSlots entries or an index 16 bits.
bool share_table(int rows, const std::vector<int32_t>& ptr, const std::vector<int32_t>& idx,
                 const std::vector<int32_t>& ord, uint32_t* out) {
  const int64_t nnz = ptr[rows];
  std::vector<int32_t> rowof(static_cast<size_t>(nnz));
  for (int r = 0; r < rows; ++r)
    for (int32_t j = ptr[r]; j < ptr[r + 1]; ++j) rowof[j] = r;
  auto lo = [&](int t) { return int64_t(t) * nnz / kWg; };
  for (int t = 0; t < kWg; ++t) {
    const int64_t s0 = lo(t), s1 = lo(t + 1);
    const int cnt = int(s1 - s0);
    if (cnt > kSlots) return false;
    uint32_t mask = 0;
    for (int i = 0; i < cnt; ++i) {
      const int32_t x = idx[size_t(s0 + i)];
      if (x < 0 || x > 0xffff) return false;
      out[size_t(i / 2) * kWg + t] |= uint32_t(x) << (16 * (i & 1));
      if (s0 + i == ptr[rowof[size_t(s0 + i)] + 1] - 1) mask |= 1u << i;
    }
    int head = 0;
    if (cnt > 0 && ptr[rowof[size_t(s0)]] < s0)
      head = int(std::min<int64_t>(cnt, ptr[rowof[size_t(s0)] + 1] - s0));
    const uint32_t q0 = head < cnt ? uint32_t(ord[rowof[size_t(s0 + head)]]) : 0u;
    int span = 0;
    if (cnt > 0 && !((mask >> (cnt - 1)) & 1u)) {
      const int64_t last = ptr[rowof[size_t(s1 - 1)] + 1] - 1;
      int t2 = t + 1;
      while (lo(t2 + 1) <= last) ++t2;
      span = t2 - t;
    }
    out[size_t(kSlotW) * kWg + t] = q0;
    out[size_t(kSlotW + 1) * kWg + t] = uint32_t(head) | uint32_t(cnt) << 6 | uint32_t(span) << 12;
    out[size_t(kSlotW + 2) * kWg + t] = mask;
  }
  return true;
}

// Builds the share tables of both CSRs and the owned-row ordinals once per
// handle (the structure of H never changes after the build).
int build_tables(hgl_handle* h, hipStream_t s) {
  if (h->wg_nq >= 0) return HGL_OK;
  if (h->wg_nq == -2) {  // refused before: the structure of H does not change
    set_error("hypergraph too large for the one-workgroup solver (more than %d incidences per thread)", kSlots);
    return HGL_EUNSUPPORTED;
  }
  const int N = h->N, E = h->E;
  const int64_t nnz = h->nnz;
  std::vector<int32_t> ep(static_cast<size_t>(E) + 1), ev(static_cast<size_t>(nnz)), vp(static_cast<size_t>(N) + 1),
      ve(static_cast<size_t>(nnz));
  HGL_HIP(hipMemcpyAsync(ep.data(), h->edge_ptr, sizeof(int32_t) * ep.size(), hipMemcpyDeviceToHost, s));
  HGL_HIP(hipMemcpyAsync(vp.data(), h->vtx_ptr, sizeof(int32_t) * vp.size(), hipMemcpyDeviceToHost, s));
  if (nnz > 0) {
    HGL_HIP(hipMemcpyAsync(ev.data(), h->edge_vtx, sizeof(int32_t) * ev.size(), hipMemcpyDeviceToHost, s));
    HGL_HIP(hipMemcpyAsync(ve.data(), h->vtx_edge, sizeof(int32_t) * ve.size(), hipMemcpyDeviceToHost, s));
  }
  HGL_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> ord_e(size_t(E) + 1), ord_v(size_t(N) + 1, -1);
  for (int e = 0; e < E; ++e) ord_e[e] = e;
  int nq = 0;
  for (int v = 0; v < N; ++v)
    if (vp[v + 1] > vp[v]) ord_v[v] = nq++;
  const size_t words = size_t(2 * kTabCsr + kRowsPT) * kWg;
  std::vector<uint32_t> tab(words, 0u);
  if (!share_table(E, ep, ev, ord_e, tab.data()) ||
      !share_table(N, vp, ve, ord_v, tab.data() + size_t(kTabCsr) * kWg)) {
    h->wg_nq = -2;
    set_error("hypergraph too large for the one-workgroup solver (more than %d incidences per thread)", kSlots);
    return HGL_EUNSUPPORTED;
  }
  int32_t* rowq = reinterpret_cast<int32_t*>(tab.data() + size_t(2 * kTabCsr) * kWg);
  for (int i = 0; i < kRowsPT; ++i)
    for (int t = 0; t < kWg; ++t) {
      const int v = t + i * kWg;
      rowq[size_t(i) * kWg + t] = v < N ? ord_v[v] : -1;
    }
  HGL_TRY(h->wg_tab.reserve(sizeof(uint32_t) * words));
  HGL_HIP(hipMemcpyAsync(h->wg_tab.p, tab.data(), sizeof(uint32_t) * words, hipMemcpyHostToDevice, s));
  HGL_HIP(hipStreamSynchronize(s));
  h->wg_nq = nq;
  return HGL_OK;
}

}  // namespace
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
  if (h->N > kRowsPT * kWg || h->E > kEdgesPT * kWg) {
    set_error("graph too large for the one-workgroup solver: N = %d, E = %d (at most %d each)", h->N, h->E,
              kRowsPT * kWg);
    return HGL_EUNSUPPORTED;
  }
  HGL_TRY(build_tables(h, s));
  const size_t lds = sizeof(double) * (size_t(h->N) + size_t(h->E) + size_t(h->wg_nq) + kWg) +
                     sizeof(float) * size_t(h->N);
  if (lds > kWgLdsMax) {
    set_error("graph too large for the one-workgroup solver: N = %d, E = %d need %zu B of LDS (at most %zu)",
              h->N, h->E, lds, kWgLdsMax);
    return HGL_EUNSUPPORTED;
  }
  HGL_TRY(h->ws_state.reserve(size_t(k) * (sizeof(double) + 2 * sizeof(int32_t)) + 64));
  HGL_TRY(ensure_pinned(h, 2 * size_t(k)));
  double* relres_d = h->ws_state.as<double>();
  int32_t* iters_d = reinterpret_cast<int32_t*>(relres_d + k);
  int32_t* status_d = iters_d + k;
  const uint32_t* tab = h->wg_tab.as<uint32_t>();
  WgArgs A;
  A.N = h->N;
  A.E = h->E;
  A.nq = h->wg_nq;
  A.tab_e = tab;
  A.tab_v = tab + size_t(kTabCsr) * kWg;
  A.rowq = reinterpret_cast<const int32_t*>(tab + size_t(2 * kTabCsr) * kWg);
  A.s = h->s32;
  A.c = h->c32;
  A.Y = Y;
  A.ldy = ldy;
  A.F = F;
  A.ldf = ldf;
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
