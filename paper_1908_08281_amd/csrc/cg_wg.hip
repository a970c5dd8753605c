// One-workgroup conjugate gradient: the latency path for small hypergraphs.
//
// The paper's experiments solve one query vector per test image on a graph
// of a few thousand vertices (section 4); a multi-kernel CG step there is
// bound by the per-launch latency of its six kernels, not by memory.  Here
// one workgroup of 1024 threads runs a column's whole solve, eqs. 16-20
// with M = I + L/lambda, in a single launch, and the columns of Y (and the
// graphs of a batched handle) are independent workgroups (one launch solves
// many queries at once).
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
// LDS holds Ps = s o p and U / Z over the hyperedges (FP32 values during the
// iterations, FP64 in the residual checks, in the same bytes), H Z over the
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

#include "kernels.h"

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

constexpr size_t kTabWords = size_t(2 * kTabCsr + kRowsPT) * kWg;  // one graph's tables
constexpr int kDesc = 5;                                             // N, E, N', vertex and edge offsets

// Per graph g (of a batched handle; one graph otherwise) the table holds
// kTabWords words at g kTabWords: the edge-major share table [kTabCsr][kWg],
// the vertex-major one, and [kRowsPT][kWg] ordinals of the owned rows among
// the graph's rows with hyperedges (-1: none or past N_g).  desc[kDesc g ..]
// gives N_g, E_g, N'_g (rows with hyperedges) and the graph's first vertex
// and hyperedge; its CSR shares use graph-local ids.
struct WgArgs {
  const uint32_t* tab;
  const int32_t* desc;
  const double* ab;  // [2 G]: a_g = 1 + 1/lambda_g at g, b_g = 1/lambda_g at G + g
  int32_t G, k;
  const float* s;
  const float* c;
  const float* Y;
  int64_t ldy;
  float* F;  // x0 on entry when x0 != 0, the result on exit (row-major, ldf)
  int64_t ldf;
  double tol2, claim2;
  int32_t max_iter, x0;
  int32_t* iters;  // [G k], graph-major
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

// Workgroup sums of x and y, identical in every thread, in a fixed order:
// each wave's sum by DPP row sums and four lane reads, then every thread
// adds the waves' sums in wave order.  red: 4 * kWgWaves doubles, two
// halves used by alternate calls (par), so the one barrier both publishes
// this call's sums and orders the last-but-one call's reads of the half
// before this call's writes.  To the caller the call is one barrier.
__device__ __forceinline__ void wg_sum2(double& x, double& y, double* red, int& par) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  x = wave_sum_dpp(x);
  y = wave_sum_dpp(y);
  double* const half = red + par * 2 * kWgWaves;
  par ^= 1;
  if (lane == 0) {
    half[wave] = x;
    half[kWgWaves + wave] = y;
  }
  __syncthreads();
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int w = 0; w < kWgWaves; ++w) {
    sx += half[w];
    sy += half[kWgWaves + w];
  }
  x = sx;
  y = sy;
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
  __shared__ double red[4 * kWgWaves];
  int par = 0;   // the half of red the next wg_sum2 writes
  const int tid = threadIdx.x, col = blockIdx.x, g = blockIdx.y;
  const int32_t* dg = A.desc + kDesc * g;
  const int N = dg[0], E = dg[1], nq = dg[2], voff = dg[3], eoff = dg[4];
  const uint32_t* tab_e = A.tab + size_t(g) * kTabWords;
  const uint32_t* tab_v = tab_e + size_t(kTabCsr) * kWg;
  const int32_t* rowq = reinterpret_cast<const int32_t*>(tab_e + size_t(2 * kTabCsr) * kWg);
  const float* sg = A.s + voff;
  const float* cg = A.c + eoff;
  float* Fo = A.F + int64_t(voff) * A.ldf + col;
  const int o = g * A.k + col;  // this (graph, column)'s output slot
  // Ps and U hold FP32 values during the iterations and FP64 values in the
  // residual checks (the same bytes; FP64 needs the full regions)
  double* Psd = wg_lds;       // [N]  s o f (checks)
  double* Ud = Psd + N;       // [E]  u_e, then Z_e = c_e u_e (checks)
  float* Psf = reinterpret_cast<float*>(Psd);  // s o p (iterations)
  float* Uf = reinterpret_cast<float*>(Ud);    // u_e, then Z_e (iterations)
  double* HZ = Ud + E;        // [nq]
  double* carry = HZ + nq;    // [kWg]
  float* Ys = reinterpret_cast<float*>(carry + kWg);  // [N]
  float s[kRowsPT], f[kRowsPT], r[kRowsPT], p[kRowsPT], ce[kEdgesPT];
  int qv[kRowsPT];
#pragma unroll
  for (int i = 0; i < kRowsPT; ++i) {
    const int v = tid + i * kWg;
    s[i] = v < N ? sg[v] : 0.f;
    qv[i] = rowq[i * kWg + tid];
    f[i] = r[i] = p[i] = 0.f;
  }
#pragma unroll
  for (int i = 0; i < kEdgesPT; ++i) {
    const int e = tid + i * kWg;
    ce[i] = e < E ? cg[e] : 0.f;
  }
  const float* Y = A.Y + int64_t(voff) * A.ldy + col;
  const double a = A.ab[g], bb = A.ab[A.G + g];

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
  wg_sum2(yy, unused, red, par);
  if (yy == 0.0) {  // zero column: f = 0 exactly
#pragma unroll
    for (int i = 0; i < kRowsPT; ++i) {
      const int v = tid + i * kWg;
      if (v < N) Fo[int64_t(v) * A.ldf] = 0.f;
    }
    if (tid == 0) {
      A.iters[o] = 0;
      A.relres[o] = 0.0;
      A.status[o] = 0;
    }
    return;
  }

  // Edge gather from Ps (complete on entry; T = float in the iterations,
  // double in the checks): Z in U; returns this thread's share of
  // sum_e c_e u_e^2.  Z is complete after the caller's next barrier.
  auto edge_phase = [&](auto* Ps, auto* U) __attribute__((always_inline)) -> double {
    using T = std::remove_pointer_t<decltype(U)>;
    share_gather(tab_e, Ps, U, carry);
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
    share_gather(tab_v, U, HZ, carry);
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
    wg_sum2(r2, p2, red, par);  // its barrier publishes Ps
    rr = r2;
    pp = p2;
  };

  double rr = 0.0, pp = 0.0;
  bool need_check = A.x0 != 0;  // a given start is checked (and restarted from) first
  if (A.x0) {
#pragma unroll
    for (int i = 0; i < kRowsPT; ++i) {
      const int v = tid + i * kWg;
      if (v < N) f[i] = Fo[int64_t(v) * A.ldf];
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
    wg_sum2(r2, p2, red, par);
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
    wg_sum2(ep, unused2, red, par);  // its barrier completes Z
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
    wg_sum2(r2, unused3, red, par);
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
    wg_sum2(p2, unused4, red, par);  // its barrier publishes Ps to the edge gather
    pp = p2;
  }

#pragma unroll
  for (int i = 0; i < kRowsPT; ++i) {
    const int v = tid + i * kWg;
    if (v < N) Fo[int64_t(v) * A.ldf] = f[i];
  }
  if (tid == 0) {
    A.iters[o] = it;
    A.relres[o] = std::sqrt(rel2);
    A.status[o] = st;
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

// Builds, once per handle, every graph's share tables (graph-local ids),
// owned-row ordinals and descriptor, and the LDS size of the largest graph
// (the structure of H never changes after the build).
int build_tables(hgl_handle* h, hipStream_t s) {
  if (h->wg_lds >= 0) return HGL_OK;
  if (h->wg_lds == -2) {  // refused before
    set_error("a graph is too large for the one-workgroup solver (N, E <= %d, at most %d incidences per "
              "thread and CSR)", kRowsPT * kWg, kSlots);
    return HGL_EUNSUPPORTED;
  }
  const int N = h->N, E = h->E, G = h->G;
  const int64_t nnz = h->nnz;
  std::vector<int32_t> ep(static_cast<size_t>(E) + 1), ev(static_cast<size_t>(nnz)),
      vp(static_cast<size_t>(N) + 1), ve(static_cast<size_t>(nnz));
  HGL_HIP(hipMemcpyAsync(ep.data(), h->edge_ptr, sizeof(int32_t) * ep.size(), hipMemcpyDeviceToHost, s));
  HGL_HIP(hipMemcpyAsync(vp.data(), h->vtx_ptr, sizeof(int32_t) * vp.size(), hipMemcpyDeviceToHost, s));
  if (nnz > 0) {
    HGL_HIP(hipMemcpyAsync(ev.data(), h->edge_vtx, sizeof(int32_t) * ev.size(), hipMemcpyDeviceToHost, s));
    HGL_HIP(hipMemcpyAsync(ve.data(), h->vtx_edge, sizeof(int32_t) * ve.size(), hipMemcpyDeviceToHost, s));
  }
  HGL_HIP(hipStreamSynchronize(s));
  const size_t desc_words = size_t(kDesc) * G;
  std::vector<uint32_t> tab(size_t(G) * kTabWords + desc_words, 0u);
  int32_t* desc = reinterpret_cast<int32_t*>(tab.data() + size_t(G) * kTabWords);
  size_t lds_max = 0;
  bool ok = true;
  for (int g = 0; g < G && ok; ++g) {
    const int v0 = h->vtx_off[g], v1 = h->vtx_off[g + 1], e0 = h->edge_off[g], e1 = h->edge_off[g + 1];
    const int Ng = v1 - v0, Eg = e1 - e0;
    if (Ng > kRowsPT * kWg || Eg > kEdgesPT * kWg) {
      ok = false;
      break;
    }
    // the graph's CSRs with local ids
    std::vector<int32_t> lep(size_t(Eg) + 1), lev, lvp(size_t(Ng) + 1), lve;
    for (int e = 0; e <= Eg; ++e) lep[e] = ep[e0 + e] - ep[e0];
    lev.reserve(size_t(lep[Eg]));
    for (int32_t j = ep[e0]; j < ep[e1]; ++j) lev.push_back(ev[j] - v0);
    for (int v = 0; v <= Ng; ++v) lvp[v] = vp[v0 + v] - vp[v0];
    lve.reserve(size_t(lvp[Ng]));
    for (int32_t j = vp[v0]; j < vp[v1]; ++j) lve.push_back(ve[j] - e0);
    std::vector<int32_t> ord_e(size_t(Eg) + 1), ord_v(size_t(Ng) + 1, -1);
    for (int e = 0; e < Eg; ++e) ord_e[e] = e;
    int nq = 0;
    for (int v = 0; v < Ng; ++v)
      if (lvp[v + 1] > lvp[v]) ord_v[v] = nq++;
    uint32_t* tg = tab.data() + size_t(g) * kTabWords;
    if (!share_table(Eg, lep, lev, ord_e, tg) || !share_table(Ng, lvp, lve, ord_v, tg + size_t(kTabCsr) * kWg)) {
      ok = false;
      break;
    }
    int32_t* rowq = reinterpret_cast<int32_t*>(tg + size_t(2 * kTabCsr) * kWg);
    for (int i = 0; i < kRowsPT; ++i)
      for (int t = 0; t < kWg; ++t) {
        const int v = t + i * kWg;
        rowq[size_t(i) * kWg + t] = v < Ng ? ord_v[v] : -1;
      }
    desc[kDesc * g + 0] = Ng;
    desc[kDesc * g + 1] = Eg;
    desc[kDesc * g + 2] = nq;
    desc[kDesc * g + 3] = v0;
    desc[kDesc * g + 4] = e0;
    lds_max = std::max(lds_max, sizeof(double) * (size_t(Ng) + size_t(Eg) + size_t(nq) + kWg) +
                                    sizeof(float) * size_t(Ng));
  }
  if (!ok || lds_max > kWgLdsMax) {
    h->wg_lds = -2;
    set_error("a graph is too large for the one-workgroup solver (N, E <= %d, at most %d incidences per "
              "thread and CSR, %zu B of LDS)", kRowsPT * kWg, kSlots, kWgLdsMax);
    return HGL_EUNSUPPORTED;
  }
  HGL_TRY(h->wg_tab.reserve(sizeof(uint32_t) * tab.size()));
  HGL_HIP(hipMemcpyAsync(h->wg_tab.p, tab.data(), sizeof(uint32_t) * tab.size(), hipMemcpyHostToDevice, s));
  HGL_HIP(hipStreamSynchronize(s));
  h->wg_lds = int32_t(lds_max);
  return HGL_OK;
}

int run_wg(hgl_handle* h, const double* lambdas, const hgl_cg_opts* o, const float* Y, int64_t ldy, float* F,
           int64_t ldf, int32_t k, int32_t* iters_host, double* relres_host, hipStream_t s) {
  HGL_CHECK_ARG(h != nullptr && o != nullptr && lambdas != nullptr, "handle, opts and lambdas must not be NULL");
  for (int g = 0; g < h->G; ++g)
    HGL_CHECK_ARG(lambdas[g] > 0.0 && std::isfinite(lambdas[g]), "lambda must be > 0 (graph %d: %g)", g,
                  lambdas[g]);
  HGL_CHECK_ARG(o->tol > 0.0 && std::isfinite(o->tol), "tol must be > 0");
  HGL_CHECK_ARG(o->max_iter >= 1, "max_iter must be >= 1");
  HGL_CHECK_ARG(k >= 1, "k must be >= 1");
  HGL_CHECK_ARG(Y && F, "Y and F must not be NULL");
  HGL_CHECK_ARG(ldy >= k && ldf >= k, "leading dimensions must be >= k");
  if (o->mode != HGL_CG_F32_F64DOT_RR) {
    set_error("the one-workgroup solver runs the FP32 mode only (mode %d)", o->mode);
    return HGL_EUNSUPPORTED;
  }
  HGL_TRY(build_tables(h, s));
  HGL_TRY(upload_ab(h, lambdas, s));
  const size_t gk = size_t(h->G) * k;
  HGL_TRY(h->ws_state.reserve(gk * (sizeof(double) + 2 * sizeof(int32_t)) + 64));
  HGL_TRY(ensure_pinned(h, 2 * gk));
  double* relres_d = h->ws_state.as<double>();
  int32_t* iters_d = reinterpret_cast<int32_t*>(relres_d + gk);
  int32_t* status_d = iters_d + gk;
  const uint32_t* tab = h->wg_tab.as<uint32_t>();
  WgArgs A;
  A.tab = tab;
  A.desc = reinterpret_cast<const int32_t*>(tab + size_t(h->G) * kTabWords);
  A.ab = h->ws_ab.as<double>();
  A.G = h->G;
  A.k = k;
  A.s = h->s32;
  A.c = h->c32;
  A.Y = Y;
  A.ldy = ldy;
  A.F = F;
  A.ldf = ldf;
  A.tol2 = o->tol * o->tol;
  A.claim2 = 0.25 * A.tol2;  // claims at tol / 2, as the multi-kernel FP32 mode
  A.max_iter = o->max_iter;
  A.x0 = o->x0_given ? 1 : 0;
  A.iters = iters_d;
  A.relres = relres_d;
  A.status = status_d;
  const size_t lds = size_t(h->wg_lds);
  if (lds > 64 * 1024)
    HGL_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_cg_wg), hipFuncAttributeMaxDynamicSharedMemorySize,
                                int(lds)));
  launch(h, -1, k_cg_wg, dim3(k, h->G), dim3(kWg), uint32_t(lds), s, A);
  HGL_HIP(hipGetLastError());
  double* pd = h->pinned_d;
  HGL_HIP(hipMemcpyAsync(pd, relres_d, sizeof(double) * gk + 2 * sizeof(int32_t) * gk, hipMemcpyDeviceToHost, s));
  HGL_HIP(hipStreamSynchronize(s));
  const int32_t* pi = reinterpret_cast<const int32_t*>(pd + gk);
  int rc = HGL_OK;
  for (size_t j = 0; j < gk; ++j) {
    if (relres_host) relres_host[j] = pd[j];
    if (iters_host) iters_host[j] = pi[j];
    const int32_t st = pi[gk + j];
    if (st == -4) rc = HGL_EBREAKDOWN;
    else if (st == 1 && rc == HGL_OK) rc = HGL_NOT_CONVERGED;
  }
  if (rc == HGL_EBREAKDOWN) set_error("CG breakdown (p'Mp <= 0 or not finite) in a column");
  return rc;
}

}  // namespace
}  // namespace hgl

using namespace hgl;

extern "C" int hgl_cg_solve_wg(hgl_handle* h, double lambda, const hgl_cg_opts* o, const float* Y, int64_t ldy,
                               float* F, int64_t ldf, int32_t k, int32_t* iters_host, double* relres_host,
                               hipStream_t s) {
  clear_error();
  enter(h, s);
  HGL_CHECK_ARG(h != nullptr, "handle is NULL");
  std::vector<double> lams(h->G, lambda);
  return run_wg(h, lams.data(), o, Y, ldy, F, ldf, k, iters_host, relres_host, s);
}

extern "C" int hgl_cg_solve_wg_batched(hgl_handle* h, const double* lambdas_host, const hgl_cg_opts* o,
                                       const float* Y, int64_t ldy, float* F, int64_t ldf, int32_t k,
                                       int32_t* iters_host, double* relres_host, hipStream_t s) {
  clear_error();
  enter(h, s);
  return run_wg(h, lambdas_host, o, Y, ldy, F, ldf, k, iters_host, relres_host, s);
}
