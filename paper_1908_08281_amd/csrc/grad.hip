// Derivatives with respect to the hyperedge weights (paper, section 2:
// P(w) of eq. 4 and the steepest-descent weight update) and the projection
// onto the constraint set {w >= 0, 1'w = 1} of eq. (4).
//
// With s_v = delta(v)^-1/2, c_e = w_e/delta(e) and A = S H C H' S (eq. 1),
//   dA/dw_e = (1/delta(e)) (S h_e)(S h_e)' - 1/2 (D_e A + A D_e),
//   D_e = diag(s_v^2 [v in e]),
// so for N x k matrices P, Q
//   Gamma_e(P, Q) = <P, dA/dw_e Q> = <u_e(P), u_e(Q)>/delta(e) - 1/2 sum_{v in e} t_v,
//   u_e(P) = sum_{v in e} s_v P_v,  t_v = s_v^2 (<P_v, (AQ)_v> + <(AP)_v, Q_v>).
// F = M^-1 Y, M = I + L/lambda, gives dF/dw_e = M^-1 (dA/dw_e) F / lambda; a
// loss with upstream G = dl/dF has dl/dw_e = Gamma_e(Z, F)/lambda with the
// adjoint Z = M^-1 G (M is symmetric, so the same CG solves it) and
// dl/dY = Z.  The adaptive-weight objective
//   J(w) = tr(F'LF) + lambda ||F - Y||^2 + mu ||w||^2
// has dJ/dw_e = -Gamma_e(F, F) + Gamma_e(Z, F)/lambda + 2 mu w_e with
// Z = M^-1 (2 lambda (M F - Y)) (total derivative; Dv depends on w).
// All contractions accumulate in FP64, each edge and vertex in a fixed order.
#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace hgl {

// Per-vertex contractions (FP64, k-wide rows, one 64-lane wave per vertex):
//   t1_v = s_v^2 * 2 <F_v, (AF)_v>                       (for Gamma(F, F))
//   t2_v = s_v^2 (<Z_v, (AF)_v> + <(AZ)_v, F_v>)         (for Gamma(Z, F))
// F and Z in the caller's type TF (row strides ldf, ldz), AF and AZ FP64.
template <class TF>
__global__ __launch_bounds__(kBlock) void k_vertex_terms(int32_t N, int k, const double* __restrict__ s,
                                                         const TF* __restrict__ F, int64_t ldf,
                                                         const double* __restrict__ AF, const TF* __restrict__ Z,
                                                         int64_t ldz, const double* __restrict__ AZ,
                                                         double* __restrict__ t1, double* __restrict__ t2) {
  const int v = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (v >= N) return;
  const int64_t o = int64_t(v) * k;
  double a = 0.0, b = 0.0;
  for (int c = lane; c < k; c += kWave) {
    const double f = double(F[int64_t(v) * ldf + c]), af = AF[o + c];
    a += f * af;
    if (Z) b += double(Z[int64_t(v) * ldz + c]) * af + AZ[o + c] * f;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a += __shfl_xor(a, off, kWave);
    b += __shfl_xor(b, off, kWave);
  }
  if (lane == 0) {
    const double s2 = s[v] * s[v];
    t1[v] = s2 * 2.0 * a;
    t2[v] = s2 * b;
  }
}

// Per-edge gradient (one wave per hyperedge):
//   g1 = <u_e(F), u_e(F)>/delta(e) - 1/2 sum_{v in e} t1_v    (= Gamma_e(F, F))
//   g2 = <u_e(Z), u_e(F)>/delta(e) - 1/2 sum_{v in e} t2_v    (= Gamma_e(Z, F))
//   grad_e = cf * g1 + cz * g2 + 2 mu w_e
// F and Z in the caller's type TF (row strides ldf, ldz), accumulated in FP64.
template <class TF>
__global__ __launch_bounds__(kBlock) void k_edge_grad(int32_t E, int k, const int32_t* __restrict__ edge_ptr,
                                                      const int32_t* __restrict__ edge_vtx,
                                                      const double* __restrict__ s, const TF* __restrict__ F,
                                                      int64_t ldf, const TF* __restrict__ Z, int64_t ldz,
                                                      const double* __restrict__ t1, const double* __restrict__ t2,
                                                      const double* __restrict__ w, double cf, double cz, double mu,
                                                      double* __restrict__ grad) {
  const int e = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (e >= E) return;
  const int b = edge_ptr[e], en = edge_ptr[e + 1];
  double ff = 0.0, zf = 0.0;
  for (int c = lane; c < k; c += kWave) {
    double uf = 0.0, uz = 0.0;
    for (int j = b; j < en; ++j) {
      const int v = edge_vtx[j];
      const double sv = s[v];
      uf += sv * double(F[int64_t(v) * ldf + c]);
      if (Z) uz += sv * double(Z[int64_t(v) * ldz + c]);
    }
    ff += uf * uf;
    zf += uz * uf;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    ff += __shfl_xor(ff, off, kWave);
    zf += __shfl_xor(zf, off, kWave);
  }
  if (lane == 0) {
    double s1 = 0.0, s2 = 0.0;
    for (int j = b; j < en; ++j) {
      s1 += t1[edge_vtx[j]];
      s2 += t2[edge_vtx[j]];
    }
    const double de = double(en - b);
    const double g1 = ff / de - 0.5 * s1;
    const double g2 = zf / de - 0.5 * s2;
    grad[e] = cf * g1 + cz * g2 + 2.0 * mu * w[e];
  }
}

template <class T>
__global__ void k_scale(int64_t rows, int k, T* __restrict__ X, int64_t ldx, double a) {
  const int64_t total = rows * k;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    T& x = X[(i / k) * ldx + i % k];
    x = T(a * double(x));
  }
}

// ------------------------------------------------------ simplex projection --

// Euclidean projection of v onto {w >= 0, sum w = 1} in one workgroup of
// kProj threads.  tau solves f(tau) = sum max(v - tau, 0) = 1 (f decreases
// in tau): each pass over v evaluates f at kSect points splitting the
// bracket [lo, hi] evenly and keeps the sub-interval where f crosses 1, then
// the exact tau of the support found, (sum_{v_i > tau} v_i - 1)/|support|,
// is recomputed until the support is stable.  Per-thread sums in a fixed
// stride order and fixed-order block reductions: deterministic.
constexpr int kProj = 512, kProjWaves = kProj / kWave, kSect = 8;

// Sums over the workgroup of x[0 .. n-1] (n <= kSect), returned to every thread.
template <int n>
__device__ void block_sums(double (&x)[n], double* lds /* [kProjWaves * kSect] */) {
#pragma unroll
  for (int m = 0; m < n; ++m)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x[m] += __shfl_xor(x[m], off, kWave);
  if (threadIdx.x % kWave == 0)
#pragma unroll
    for (int m = 0; m < n; ++m) lds[(threadIdx.x / kWave) * kSect + m] = x[m];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < n; ++m) {
    double t = 0.0;
    for (int w = 0; w < kProjWaves; ++w) t += lds[w * kSect + m];
    x[m] = t;
  }
  __syncthreads();
}

// The point projected: v_i, or (g given) the gradient step w_i - eta g_i,
// with eta read from *eta_in when it is given; *eta_out (nullable) receives
// the eta used.  The step is evaluated without contraction, so every pass
// sees the same value.
struct StepPoint {
  const double* v;
  const double* g;
  const double* eta_in;
  double* eta_out;
  double eta;
  __device__ __forceinline__ double operator()(int i) const {
#pragma clang fp contract(off)
    return g ? v[i] - eta * g[i] : v[i];
  }
};

__global__ __launch_bounds__(kProj) void k_project_simplex(int32_t E, StepPoint pt, double* __restrict__ w) {
  __shared__ double lds[kProjWaves * kSect];
  if (pt.g && pt.eta_in) pt.eta = *pt.eta_in;
  if (pt.eta_out && threadIdx.x == 0) *pt.eta_out = pt.eta;
  const StepPoint& v = pt;
  // max v and sum v: tau lies in [max(vmax - 1, (sum v - 1)/E), vmax] (the
  // largest entry alone gives at most 1; tau = (sum v - 1)/E would give
  // every entry, so f there is >= 1)
  double mx = -INFINITY, sm[1] = {0.0};
  for (int i = threadIdx.x; i < E; i += kProj) {
    mx = fmax(mx, v(i));
    sm[0] += v(i);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, kWave));
  if (threadIdx.x % kWave == 0) lds[(threadIdx.x / kWave) * kSect + 1] = mx;
  __syncthreads();
  mx = -INFINITY;
  for (int wv = 0; wv < kProjWaves; ++wv) mx = fmax(mx, lds[wv * kSect + 1]);
  __syncthreads();
  block_sums<1>(sm, lds);
  double lo = fmax(mx - 1.0, (sm[0] - 1.0) / double(E)), hi = mx;
  // sectioning narrows the bracket by (kSect + 1) per pass; seven passes
  // leave about 2e-7 of it, after which the support iteration below needs a
  // round or two
  for (int pass = 0; pass < 7 && hi > lo; ++pass) {
    double tau[kSect], f[kSect];
#pragma unroll
    for (int m = 0; m < kSect; ++m) {
      tau[m] = lo + (hi - lo) * double(m + 1) / double(kSect + 1);
      f[m] = 0.0;
    }
    // eight loads in flight per round; entries past E read as -inf (adding 0)
    for (int i0 = threadIdx.x; i0 < E; i0 += 8 * kProj) {
      double vi[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) vi[u] = i0 + u * kProj < E ? v(i0 + u * kProj) : -INFINITY;
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int m = 0; m < kSect; ++m) f[m] += fmax(vi[u] - tau[m], 0.0);
    }
    block_sums<kSect>(f, lds);
    // f is decreasing: the crossing lies after the last point with f >= 1
    double nlo = lo, nhi = hi;
#pragma unroll
    for (int m = 0; m < kSect; ++m) {
      if (f[m] >= 1.0) nlo = tau[m];
      else if (nhi == hi) nhi = tau[m];
    }
    lo = nlo;
    hi = nhi;
  }
  // support iteration from below (f(lo) >= 1, so lo <= tau*): tau <- (sum
  // of the entries above tau - 1)/their count increases to tau* and stops
  // there once the support is stable
  double tau = lo;
  for (int round = 0; round < 64; ++round) {
    double sc[2] = {0.0, 0.0};  // sum and count of the support
    for (int i = threadIdx.x; i < E; i += kProj)
      if (v(i) > tau) {
        sc[0] += v(i);
        sc[1] += 1.0;
      }
    block_sums<2>(sc, lds);
    const double t2 = sc[1] > 0.0 ? (sc[0] - 1.0) / sc[1] : tau;
    if (!(t2 > tau)) break;
    tau = t2;
  }
  for (int i = threadIdx.x; i < E; i += kProj) w[i] = fmax(v(i) - tau, 0.0);
}

// The fixed step of the weight update, set from the first gradient:
// eta = 0.5 max|w| / max|g - mean(g)| (0 when g is constant), written to
// *eta_out.  One workgroup, fixed-order sums: deterministic.
__global__ __launch_bounds__(kProj) void k_step_size(int32_t E, const double* __restrict__ w,
                                                     const double* __restrict__ g, double* __restrict__ eta_out) {
  __shared__ double lds[kProjWaves * kSect];
  double sm[2] = {0.0, 0.0};  // sum g, max |w| (as a sum slot after the max reduction)
  double wmax = 0.0;
  for (int i = threadIdx.x; i < E; i += kProj) {
    sm[0] += g[i];
    wmax = fmax(wmax, fabs(w[i]));
  }
  double sg[1] = {sm[0]};
  block_sums<1>(sg, lds);
  const double mean = sg[0] / double(E);
  double dmax = 0.0;
  for (int i = threadIdx.x; i < E; i += kProj) dmax = fmax(dmax, fabs(g[i] - mean));
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    wmax = fmax(wmax, __shfl_xor(wmax, off, kWave));
    dmax = fmax(dmax, __shfl_xor(dmax, off, kWave));
  }
  if (threadIdx.x % kWave == 0) {
    lds[(threadIdx.x / kWave) * kSect] = wmax;
    lds[(threadIdx.x / kWave) * kSect + 1] = dmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int wv = 0; wv < kProjWaves; ++wv) {
      a = fmax(a, lds[wv * kSect]);
      b = fmax(b, lds[wv * kSect + 1]);
    }
    *eta_out = b > 0.0 ? 0.5 * a / b : 0.0;
  }
}

// ------------------------------------------------ active-set step (eq. 5) --

// Minimum over the workgroup, returned to every thread (fixed order).
__device__ double block_min(double x, double* lds /* [kProjWaves * kSect] */) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = fmin(x, __shfl_xor(x, off, kWave));
  if (threadIdx.x % kWave == 0) lds[(threadIdx.x / kWave) * kSect] = x;
  __syncthreads();
  double m = INFINITY;
  for (int w = 0; w < kProjWaves; ++w) m = fmin(m, lds[w * kSect]);
  __syncthreads();
  return m;
}

// Steepest descent on the Lagrangian of eq. 5 in one workgroup of kProj
// threads.  The direction is the projection of -g onto the constraints that
// stay active: d_i = nu - g_i where w_i > 0, max(nu - g_i, 0) where w_i = 0,
// with nu the root of phi(nu) = sum d_i = 0 (phi increases, with slope at
// least the number of positive weights, so the root is unique and lies in
// [min g, max g]).  Sectioning passes narrow the bracket as in the
// projection; then, from the upper end (phi >= 0), nu <- the mean of g over
// the positive weights and the zero weights with g_i < nu decreases to the
// root and stops once that set is stable.  The step mu_eff = min(mu, min
// over d_i < 0 of w_i / -d_i) keeps w >= 0; the entries at the bound get
// exactly 0.  info = {nu, mu_eff, released zero weights, active zero
// weights}; nu = NaN when w has no positive entry (then w_out = w).
__global__ __launch_bounds__(kProj) void k_active_set_step(int32_t E, const double* __restrict__ w,
                                                           const double* __restrict__ g, double mu,
                                                           double* w_out, double* __restrict__ d_out,
                                                           double* __restrict__ info) {
  __shared__ double lds[kProjWaves * kSect];
  double mn = INFINITY, mx = -INFINITY, np_[1] = {0.0};
  for (int i = threadIdx.x; i < E; i += kProj) {
    mn = fmin(mn, g[i]);
    mx = fmax(mx, g[i]);
    if (w[i] > 0.0) np_[0] += 1.0;
  }
  mn = block_min(mn, lds);
  mx = -block_min(-mx, lds);
  block_sums<1>(np_, lds);
  if (np_[0] == 0.0) {
    for (int i = threadIdx.x; i < E; i += kProj) {
      w_out[i] = w[i];
      if (d_out) d_out[i] = 0.0;
    }
    if (threadIdx.x == 0) {
      info[0] = NAN;
      info[1] = 0.0;
      info[2] = 0.0;
      info[3] = double(E);
    }
    return;
  }
  double lo = mn, hi = mx;
  for (int pass = 0; pass < 7 && hi > lo; ++pass) {
    double t[kSect], f[kSect];
#pragma unroll
    for (int m = 0; m < kSect; ++m) {
      t[m] = lo + (hi - lo) * double(m + 1) / double(kSect + 1);
      f[m] = 0.0;
    }
    for (int i = threadIdx.x; i < E; i += kProj) {
      const double gi = g[i];
      const bool pos = w[i] > 0.0;
#pragma unroll
      for (int m = 0; m < kSect; ++m) f[m] += pos ? t[m] - gi : fmax(t[m] - gi, 0.0);
    }
    block_sums<kSect>(f, lds);
    // phi increases: the root lies after the last point with phi < 0
    double nlo = lo, nhi = hi;
#pragma unroll
    for (int m = 0; m < kSect; ++m) {
      if (f[m] < 0.0) nlo = t[m];
      else if (nhi == hi) nhi = t[m];
    }
    lo = nlo;
    hi = nhi;
  }
  double nu = hi;
  for (int round = 0; round < 64; ++round) {
    double sc[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < E; i += kProj)
      if (w[i] > 0.0 || g[i] < nu) {
        sc[0] += g[i];
        sc[1] += 1.0;
      }
    block_sums<2>(sc, lds);
    const double n2 = sc[0] / sc[1];
    if (!(n2 < nu)) break;
    nu = n2;
  }
  double rmin = INFINITY, cnt[2] = {0.0, 0.0};
  for (int i = threadIdx.x; i < E; i += kProj) {
    const double wi = w[i], gi = g[i];
    const double di = wi > 0.0 ? nu - gi : fmax(nu - gi, 0.0);
    if (di < 0.0) rmin = fmin(rmin, wi / -di);
    if (!(wi > 0.0)) cnt[di > 0.0 ? 0 : 1] += 1.0;
  }
  rmin = block_min(rmin, lds);
  block_sums<2>(cnt, lds);
  const double me = fmin(mu, rmin);
  for (int i = threadIdx.x; i < E; i += kProj) {
    const double wi = w[i], gi = g[i];
    const double di = wi > 0.0 ? nu - gi : fmax(nu - gi, 0.0);
    const bool hit = di < 0.0 && wi / -di <= me;
    w_out[i] = hit ? 0.0 : wi + me * di;
    if (d_out) d_out[i] = di;
  }
  if (threadIdx.x == 0) {
    info[0] = nu;
    info[1] = me;
    info[2] = cnt[0];
    info[3] = cnt[1];
  }
}

// ------------------------------------------------------------------ driver --

template <class T>
static int run_grad(hgl_handle* h, double lam, double mu, const T* F, int64_t ldf, const T* G, int64_t ldg,
                    const T* Y, int64_t ldy, int k, const hgl_cg_opts* adj, double* grad, T* Zout, int64_t ldz,
                    int32_t* iters_host, double* relres_host, hipStream_t s) {
  const int N = h->N, E = h->E;
  const bool objective = G == nullptr;
  const size_t nk = size_t(N) * k;
  // buffers: AF, AZ (N x k FP64), rhs/Z in T (N x k), t1, t2 (N)
  DevBuf& buf = h->ws_extra[1];
  DevBuf& bufT = h->ws_extra[2];
  HGL_TRY(buf.reserve(sizeof(double) * (2 * nk + 2 * size_t(N)) + 256));
  HGL_TRY(bufT.reserve(sizeof(T) * 2 * nk + 256));
  double* AF = buf.as<double>();
  double* AZ = AF + nk;
  double* t1 = AZ + nk;
  double* t2 = t1 + N;
  T* rhs = bufT.as<T>();
  T* Zt = rhs + nk;
  HGL_TRY(h->ws_z64.reserve(sizeof(double) * size_t(std::max(E, 1)) * k));
  double* Zedge = h->ws_z64.as<double>();
  const int blocks = int(std::min<int64_t>((int64_t(nk) + 255) / 256, 65535));

  prof_begin(h, kProfGrad, s);
  // (a, b) pairs for the products: A X = 0 X - (-1) S H Z; M X = (1+1/lam) X - (1/lam) S H Z
  DevBuf& abA = h->ws_extra[3];
  DevBuf& abM = h->ws_extra[4];
  HGL_TRY(abA.reserve(16 * size_t(h->G)));
  HGL_TRY(abM.reserve(16 * size_t(h->G)));
  {
    std::vector<double> a(2 * h->G), m(2 * h->G);
    for (int g = 0; g < h->G; ++g) {
      a[g] = 0.0;
      a[h->G + g] = -1.0;
      m[g] = 1.0 + 1.0 / lam;
      m[h->G + g] = 1.0 / lam;
    }
    HGL_TRY(ensure_pinned(h, 4 * h->G + 8));
    std::copy(a.begin(), a.end(), h->pinned_d);
    std::copy(m.begin(), m.end(), h->pinned_d + 2 * h->G);
    HGL_HIP(hipMemcpyAsync(abA.p, h->pinned_d, 16 * size_t(h->G), hipMemcpyHostToDevice, s));
    HGL_HIP(hipMemcpyAsync(abM.p, h->pinned_d + 2 * h->G, 16 * size_t(h->G), hipMemcpyHostToDevice, s));
    HGL_HIP(hipStreamSynchronize(s));
  }
  // A X in FP64 from X in the caller's type: the edge gather accumulates in
  // FP64 (exact products of the stored values), the vertex gather takes no
  // X (a = 0 for A)
  auto applyA = [&](const T* X, int64_t ldx, double* Out) -> int {
    const ColShape csa = pick_shape(k, 8, {X, Zedge, Out}, {ldx, int64_t(k)});
    HGL_TRY((launch_spmm_edge<T, double>(h, X, ldx, Zedge, k, k, csa, Gate{}, s)));
    return launch_spmm_vertex<double, double>(h, VMode::Apply, nullptr, 0, Zedge, k, nullptr, 0, Out, k,
                                               abA.as<double>(), abA.as<double>() + h->G, nullptr, k, csa, Gate{},
                                               s);
  };
  HGL_TRY(applyA(F, ldf, AF));
  // adjoint right-hand side: G, or for the objective R = Y - M F from the FP64
  // residual pass (accumulated in FP64, so the small difference keeps its
  // digits); then Z' = M^-1 R and Z = -2 lambda Z' (M^-1 is linear), so the
  // adjoint term Gamma(Z, F)/lambda = -2 Gamma(Z', F)
  const T* rhs_ptr = G;
  int64_t ld_rhs = ldg;
  if (objective) {
    HGL_TRY(h->ws_part.reserve(sizeof(double) * size_t(n_slots(h)) * k));
    const ColShape csr = pick_shape(k, 8, {F, Y, rhs, Zedge}, {ldf, ldy, int64_t(k)});
    HGL_TRY((launch_spmm_edge<T, double>(h, F, ldf, Zedge, k, k, csr, Gate{}, s)));
    HGL_TRY((launch_spmm_vertex<T, double>(h, VMode::Resid, F, ldf, Zedge, k, Y, ldy, rhs, k, abM.as<double>(),
                                           abM.as<double>() + h->G, h->ws_part.as<double>(), k, csr, Gate{}, s)));
    rhs_ptr = rhs;
    ld_rhs = k;
  }
  prof_end(h, s);
  // adjoint solve Z = M^-1 rhs (same operator: M is symmetric)
  T* Zdst = Zout ? Zout : Zt;
  const int64_t ldzd = Zout ? ldz : k;
  std::vector<double> lams(h->G, lam);
  int st = cg_run(h, lams.data(), adj, rhs_ptr, ld_rhs, Zdst, ldzd, k, iters_host, relres_host, nullptr, s);
  if (st < 0) return st;
  prof_begin(h, kProfGrad, s);
  HGL_TRY(applyA(Zdst, ldzd, AZ));
  // the contractions read F and Z in the caller's type (FP32 -> FP64 is exact)
  launch(h, -1, k_vertex_terms<T>, dim3((N + 3) / 4), dim3(kBlock), 0, s, N, k, h->s64, F, ldf,
         static_cast<const double*>(AF), static_cast<const T*>(Zdst), ldzd, static_cast<const double*>(AZ), t1, t2);
  HGL_HIP(hipGetLastError());
  if (E > 0) {
    const double cf = objective ? -1.0 : 0.0;
    const double cz = objective ? -2.0 : 1.0 / lam;
    launch(h, -1, k_edge_grad<T>, dim3((E + 3) / 4), dim3(kBlock), 0, s, E, k, h->edge_ptr, h->edge_vtx, h->s64,
           F, ldf, static_cast<const T*>(Zdst), ldzd, static_cast<const double*>(t1), static_cast<const double*>(t2),
           static_cast<const double*>(h->w), cf, cz, objective ? mu : 0.0, grad);
    HGL_HIP(hipGetLastError());
  }
  if (objective && Zout) {
    // the caller's Z = -2 lambda Z'
    launch(h, -1, k_scale<T>, dim3(blocks), dim3(256), 0, s, int64_t(N), k, Zout, ldz, -2.0 * lam);
    HGL_HIP(hipGetLastError());
  }
  prof_end(h, s);
  HGL_HIP(hipStreamSynchronize(s));
  return st;
}

}  // namespace hgl

using namespace hgl;

extern "C" int hgl_weight_grad(hgl_handle* h, double lambda, double mu, const void* F, int64_t ldf, const void* G,
                               int64_t ldg, const void* Y, int64_t ldy, int32_t k, const hgl_cg_opts* adj,
                               double* grad_w, void* Z_out, int64_t ldz, int32_t* iters_host,
                               double* relres_host, hipStream_t s) {
  clear_error();
  enter(h, s);
  HGL_CHECK_ARG(h != nullptr && adj != nullptr, "handle and adjoint options must not be NULL");
  HGL_CHECK_ARG(h->G == 1, "the weight gradient needs a single-graph handle");
  HGL_CHECK_ARG(lambda > 0.0 && std::isfinite(lambda), "lambda must be > 0");
  HGL_CHECK_ARG(std::isfinite(mu), "mu must be finite");
  HGL_CHECK_ARG(k >= 1 && F && grad_w, "need k >= 1, F and grad_w");
  HGL_CHECK_ARG(ldf >= k && (G == nullptr || ldg >= k) && (Z_out == nullptr || ldz >= k), "bad leading dimension");
  HGL_CHECK_ARG(G != nullptr || (Y != nullptr && ldy >= k), "the objective gradient (G = NULL) needs Y");
  if (adj->mode == HGL_CG_F32_F64DOT_RR)
    return run_grad<float>(h, lambda, mu, static_cast<const float*>(F), ldf, static_cast<const float*>(G), ldg,
                           static_cast<const float*>(Y), ldy, k, adj, grad_w, static_cast<float*>(Z_out), ldz,
                           iters_host, relres_host, s);
  if (adj->mode == HGL_CG_PLAIN_F64)
    return run_grad<double>(h, lambda, mu, static_cast<const double*>(F), ldf, static_cast<const double*>(G), ldg,
                            static_cast<const double*>(Y), ldy, k, adj, grad_w, static_cast<double*>(Z_out), ldz,
                            iters_host, relres_host, s);
  set_error("unknown CG mode %d", adj->mode);
  return HGL_EINVAL;
}

extern "C" int hgl_project_simplex(const double* v, double* w, int32_t E, hipStream_t s) {
  clear_error();
  HGL_CHECK_ARG(E >= 1 && v && w, "need E >= 1 and v, w");
  hipLaunchKernelGGL(k_project_simplex, dim3(1), dim3(kProj), 0, s, E, StepPoint{v, nullptr, nullptr, nullptr, 0.0},
                     w);
  HGL_HIP(hipGetLastError());
  return HGL_OK;
}

extern "C" int hgl_projected_gradient_step(const double* w, const double* g, double eta, int32_t E, double* w_out,
                                           double* eta_dev, hipStream_t s) {
  clear_error();
  HGL_CHECK_ARG(E >= 1 && w && g && w_out, "need E >= 1 and w, g, w_out");
  HGL_CHECK_ARG(std::isfinite(eta), "eta must be finite");
  HGL_CHECK_ARG(eta > 0.0 || eta_dev, "eta <= 0 asks for the step from the gradient: eta_dev must be given");
  HGL_CHECK_ARG(w_out != w && w_out != g, "w_out must not alias w or g");
  if (eta > 0.0) {
    hipLaunchKernelGGL(k_project_simplex, dim3(1), dim3(kProj), 0, s, E, StepPoint{w, g, nullptr, eta_dev, eta},
                       w_out);
  } else {
    hipLaunchKernelGGL(k_step_size, dim3(1), dim3(kProj), 0, s, E, w, g, eta_dev);
    HGL_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_project_simplex, dim3(1), dim3(kProj), 0, s, E, StepPoint{w, g, eta_dev, nullptr, 0.0},
                       w_out);
  }
  HGL_HIP(hipGetLastError());
  return HGL_OK;
}

extern "C" int hgl_active_set_step(const double* w, const double* g, double mu, int32_t E, double* w_out,
                                   double* d_out, double* info_dev, double* info_host, hipStream_t s) {
  clear_error();
  HGL_CHECK_ARG(E >= 1 && w && g && w_out && info_dev, "need E >= 1 and w, g, w_out, info_dev");
  HGL_CHECK_ARG(mu > 0.0 && std::isfinite(mu), "mu must be > 0 and finite");
  hipLaunchKernelGGL(k_active_set_step, dim3(1), dim3(kProj), 0, s, E, w, g, mu, w_out, d_out, info_dev);
  HGL_HIP(hipGetLastError());
  if (info_host) {
    HGL_HIP(hipMemcpyAsync(info_host, info_dev, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    HGL_HIP(hipStreamSynchronize(s));
    HGL_CHECK_ARG(!std::isnan(info_host[0]), "w has no positive entry (it is not on the simplex)");
  }
  return HGL_OK;
}
