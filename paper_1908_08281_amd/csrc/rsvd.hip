// Block randomized SVD by subspace iteration (paper, section 3, Algorithm 1)
// on the diagonal blocks of the tessellated operator (eq. 11), and the block
// inverse built from it (eq. 15, in identity-plus-low-rank form).
//
// For every diagonal block b (vertex range [o_b, o_b + n_b)) the dense block
// A_bb of the normalised adjacency (eq. 1) is extracted once.  Then, for all
// blocks at once (one launch per step, blocks of uneven size batched):
//   Y = A_bb Omega                      (BF16 MFMA, FP32 accumulation)
//   S = orth(Y)                         (CholQR2: FP64 Gram, FP64 Cholesky)
//   q times: S~ = orth(A_bb' S) = orth(A_bb S)   (A_bb is symmetric)
//            S  = orth(A_bb S~)
//   W = A_bb S,  B B' = S' A A' S = W'W (FP64 Gram)
//   B B' = U~ diag(sigma^2) U~'          (FP64 parallel cyclic Jacobi)
//   U = S U~, keep the leading k columns.
// The block inverse M_bb^-1 ~ lambda/(1+lambda) [I + U diag(sigma/(1+lambda-sigma)) U']
// preconditions CG on the full system.
//
// Storage per block: n_b padded to nbp (multiple of 64) rows and columns;
// l = k + p sketch columns padded to LP (multiple of 16, at most 96).
//   A_bb      nbp x nbp row-major (BF16 or FP64), zero padding
//   Y, S      nbp x LP  row-major FP32/FP64 (FP64 in the FP64 sketch mode)
//   ST        LP x nbp  row-major = S transposed, the GEMM operand (BF16/FP64)
//   Gram, L^-1  LP x LP FP64
#include <algorithm>
#include <cmath>
#include <cstring>

#include "kernels.h"

namespace hgl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kMaxLP = 96;

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

struct BlockMeta {
  int32_t nb;            // blocks
  int32_t l, LP, kk;     // sketch width, padded width, kept rank
  const int32_t* off;    // [nb+1] vertex offsets
  const int32_t* nbp;    // [nb] padded sizes
  const int64_t* aoff;   // [nb] offset of A_bb (elements)
  const int64_t* yoff;   // [nb] offset of Y/S/ST (elements)
  const int32_t* item_b; // [n_items] block of a 64-row tile
  const int32_t* item_t; // [n_items] tile index within the block
};

// ------------------------------------------------------------ extraction --

// A_bb[u][v] = s_u s_v sum_{e containing u and v} c_e for u, v in block b.
// One wave per row u: the row is accumulated in LDS, hyperedges of u in
// increasing id order, members of one hyperedge on distinct lanes (a vertex
// set has no repeats), so no two lanes update one entry at once.
template <class TA>
__global__ __launch_bounds__(kBlock) void k_extract_blocks(BlockMeta bm, const int32_t* __restrict__ vtx_ptr,
                                                           const int32_t* __restrict__ vtx_edge,
                                                           const int32_t* __restrict__ edge_ptr,
                                                           const int32_t* __restrict__ edge_vtx,
                                                           const double* __restrict__ s,
                                                           const double* __restrict__ c, TA* __restrict__ A,
                                                           int max_nbp) {
  extern __shared__ double srow[];  // [4][max_nbp]
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int b = blockIdx.y;
  const int o = bm.off[b], n = bm.off[b + 1] - o, nbp = bm.nbp[b];
  const int ur = blockIdx.x * 4 + wave;  // row within the padded block
  if (blockIdx.x * 4 >= nbp) return;
  double* row = srow + int64_t(wave) * max_nbp;
  for (int j = lane; j < nbp; j += kWave) row[j] = 0.0;
  __syncthreads();
  if (ur < n) {
    const int u = o + ur;
    for (int q = vtx_ptr[u]; q < vtx_ptr[u + 1]; ++q) {
      const int e = vtx_edge[q];
      const double ce = c[e];
      for (int m = edge_ptr[e] + lane; m < edge_ptr[e + 1]; m += kWave) {
        const int v = edge_vtx[m];
        if (v >= o && v < o + n) row[v - o] += ce * s[v];
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    }
  }
  __syncthreads();
  if (ur < nbp) {
    const double su = ur < n ? s[o + ur] : 0.0;
    TA* dst = A + bm.aoff[b] + int64_t(ur) * nbp;
    for (int j = lane; j < nbp; j += kWave) {
      const double v = su * row[j];
      if constexpr (sizeof(TA) == 2) dst[j] = f32_to_bf16_rne(float(v));
      else dst[j] = v;
    }
  }
}

// -------------------------------------------------------------- sketch --

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the
// multiply-xor round function on a 128-bit counter with a 64-bit key bumped
// by the Weyl constants each round.
__device__ __forceinline__ void philox4x32_10(uint32_t ctr[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(M0, ctr[0]), lo0 = M0 * ctr[0];
    const uint32_t hi1 = __umulhi(M1, ctr[2]), lo1 = M1 * ctr[2];
    const uint32_t n0 = hi1 ^ ctr[1] ^ k0, n2 = hi0 ^ ctr[3] ^ k1;
    ctr[0] = n0;
    ctr[1] = lo1;
    ctr[2] = n2;
    ctr[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

// Standard normal pair from two uniforms in (0, 1] (Box-Muller).
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& z0, double& z1) {
  const double u1 = (double(a) + 1.0) * (1.0 / 4294967296.0);
  const double u2 = double(b) * (1.0 / 4294967296.0);
  const double r = sqrt(-2.0 * log(u1));
  const double t = 6.283185307179586476925286766559 * u2;
  z0 = r * cos(t);
  z1 = r * sin(t);
}

// Omega[g][j] (g = global vertex row, j < l) from counter (g*l + j) / 4 of
// the Philox stream: each counter gives four 32-bit words = two normals.
__global__ void k_philox_sketch(int64_t rows, int l, uint64_t seed, uint16_t* __restrict__ out) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;  // one counter = 2 normals
  const int64_t total = rows * l;
  if (2 * idx >= total) return;
  uint32_t ctr[4] = {uint32_t(idx), uint32_t(uint64_t(idx) >> 32), 0u, 0u};
  philox4x32_10(ctr, uint32_t(seed), uint32_t(seed >> 32));
  double z0, z1;
  box_muller(ctr[0], ctr[1], z0, z1);
  out[2 * idx] = f32_to_bf16_rne(float(z0));
  if (2 * idx + 1 < total) out[2 * idx + 1] = f32_to_bf16_rne(float(z1));
}

// ST_b[j][r] = Omega[o_b + r][j] for j < l, r < n_b; zero elsewhere.
template <class TS>
__global__ void k_sketch_to_st(BlockMeta bm, const uint16_t* __restrict__ omega, TS* __restrict__ ST,
                               int64_t lo_off) {
  const int b = blockIdx.y;
  const int o = bm.off[b], n = bm.off[b + 1] - o, nbp = bm.nbp[b];
  const int64_t total = int64_t(bm.LP) * nbp;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    const int j = int(i / nbp), r = int(i % nbp);
    uint16_t v = 0;
    if (j < bm.l && r < n) v = omega[int64_t(o + r) * bm.l + j];
    if constexpr (sizeof(TS) == 2) {
      ST[bm.yoff[b] + i] = v;
      ST[lo_off + bm.yoff[b] + i] = 0;  // Omega is exactly BF16: no lo part
    } else {
      ST[bm.yoff[b] + i] = double(bf16_to_f32(v));
    }
  }
}

// ---------------------------------------------------------------- GEMMs --

// Y_b = A_bb S_b for one 64-row tile: 4 waves x 16 rows, LP/16 MFMA tiles of
// 16x16 per wave, K in steps of 32 (v_mfma_f32_16x16x32_bf16).  Lane l holds
// A rows (l % 16), k = 8*(l/16) .. +7 and S columns (l % 16), same k; the
// result holds rows 4*(l/16) .. +3 of column l % 16.
// S is carried as a pair of BF16 matrices S = S_hi + S_lo (S_lo = the BF16
// rounding of S - S_hi), so each loaded A fragment feeds two MFMAs and the
// product keeps about 16 significant bits of S while A_bb stays in BF16.
template <int LP>
__global__ __launch_bounds__(kBlock) void k_gemm_bf16(BlockMeta bm, const uint16_t* __restrict__ A,
                                                      const uint16_t* __restrict__ ST, int64_t lo_off,
                                                      float* __restrict__ Y) {
  constexpr int NT = LP / 16;
  const int b = bm.item_b[blockIdx.x], t = bm.item_t[blockIdx.x];
  const int nbp = bm.nbp[b];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int r0 = t * 64 + wave * 16;
  const int li = lane % 16, kq = lane / 16;
  const uint16_t* Ab = A + bm.aoff[b] + int64_t(r0 + li) * nbp + kq * 8;
  const uint16_t* Sb = ST + bm.yoff[b] + int64_t(li) * nbp + kq * 8;
  floatx4 acc[NT];
#pragma unroll
  for (int n = 0; n < NT; ++n) acc[n] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < nbp; k0 += 32) {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(Ab + k0);
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      const uint16_t* sp = Sb + int64_t(n) * 16 * nbp + k0;
      const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(sp);
      const bf16x8 blo = *reinterpret_cast<const bf16x8*>(sp + lo_off);
      acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bhi, acc[n], 0, 0, 0);
      acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, blo, acc[n], 0, 0, 0);
    }
  }
  float* Yb = Y + bm.yoff[b];
#pragma unroll
  for (int n = 0; n < NT; ++n)
#pragma unroll
    for (int i = 0; i < 4; ++i) Yb[int64_t(r0 + kq * 4 + i) * LP + n * 16 + li] = acc[n][i];
}

// FP64 reference-precision variant: Y_b = A_bb S_b, plain FMA, one thread per
// (row, 4 columns) of a 64-row tile.
__global__ __launch_bounds__(kBlock) void k_gemm_f64(BlockMeta bm, const double* __restrict__ A,
                                                     const double* __restrict__ ST, double* __restrict__ Y) {
  const int b = bm.item_b[blockIdx.x], t = bm.item_t[blockIdx.x];
  const int nbp = bm.nbp[b], LP = bm.LP;
  const double* Ab = A + bm.aoff[b];
  const double* Sb = ST + bm.yoff[b];
  double* Yb = Y + bm.yoff[b];
  for (int o = threadIdx.x; o < 64 * LP; o += kBlock) {
    const int r = t * 64 + o / LP, j = o % LP;
    const double* ar = Ab + int64_t(r) * nbp;
    const double* sj = Sb + int64_t(j) * nbp;
    double acc = 0.0;
    for (int q = 0; q < nbp; ++q) acc += ar[q] * sj[q];
    Yb[int64_t(r) * LP + j] = acc;
  }
}

// ----------------------------------------------------------------- Gram --

// G_b = Y_b' Y_b over the first l columns (FP64 accumulation), rows staged
// through LDS 32 at a time; thread t owns the upper-triangle pairs t, t+256, ...
constexpr int kGramPairsPerThread = (kMaxLP * (kMaxLP + 1) / 2 + kBlock - 1) / kBlock;

template <class TY>
__global__ __launch_bounds__(kBlock) void k_gram(BlockMeta bm, const TY* __restrict__ Y, double* __restrict__ G) {
  __shared__ double tile[32 * kMaxLP];
  const int b = blockIdx.x;
  const int n = bm.off[b + 1] - bm.off[b];
  const int l = bm.l, LP = bm.LP;
  const int npairs = l * (l + 1) / 2;
  int pi[kGramPairsPerThread], pj[kGramPairsPerThread];
  double acc[kGramPairsPerThread];
  int np = 0;
  for (int p = threadIdx.x; p < npairs; p += kBlock) {
    int i = 0, rem = p;
    while (rem >= l - i) {
      rem -= l - i;
      ++i;
    }
    pi[np] = i;
    pj[np] = i + rem;
    acc[np] = 0.0;
    ++np;
  }
  const TY* Yb = Y + bm.yoff[b];
  for (int r0 = 0; r0 < n; r0 += 32) {
    const int rows = min(32, n - r0);
    __syncthreads();
    for (int q = threadIdx.x; q < rows * l; q += kBlock) {
      const int rr = q / l, cc = q % l;
      tile[rr * kMaxLP + cc] = double(Yb[int64_t(r0 + rr) * LP + cc]);
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < kGramPairsPerThread; ++a) {
      if (a < np) {
        double sacc = acc[a];
        for (int rr = 0; rr < rows; ++rr) sacc += tile[rr * kMaxLP + pi[a]] * tile[rr * kMaxLP + pj[a]];
        acc[a] = sacc;
      }
    }
  }
  double* Gb = G + int64_t(b) * LP * LP;
#pragma unroll
  for (int a = 0; a < kGramPairsPerThread; ++a) {
    if (a < np) {
      Gb[pi[a] * LP + pj[a]] = acc[a];
      Gb[pj[a] * LP + pi[a]] = acc[a];
    }
  }
}

// ------------------------------------------------------ Cholesky, inverse --

// In LDS: L = chol(G) (lower), then Linv = L^-1 (lower), written to Li.
// A non-positive or non-finite pivot triggers one retry with the shift
// 11 (n l + l (l+1)) u trace(G) (shifted CholQR, Fukaya et al. 2020); a
// second failure sets fail[b].
__global__ __launch_bounds__(kBlock) void k_chol_inv(BlockMeta bm, const double* __restrict__ G,
                                                     double* __restrict__ Li, int32_t* __restrict__ fail) {
  extern __shared__ double sm[];
  const int b = blockIdx.x;
  const int l = bm.l, LP = bm.LP;
  const int n = bm.off[b + 1] - bm.off[b];
  double* L = sm;             // l x l
  double* X = sm + l * l;     // l x l
  __shared__ int s_bad;
  __shared__ double s_tr;
  const double* Gb = G + int64_t(b) * LP * LP;
  for (int attempt = 0; attempt < 2; ++attempt) {
    if (threadIdx.x == 0) {
      double tr = 0.0;
      for (int i = 0; i < l; ++i) tr += Gb[i * LP + i];
      s_tr = tr;
      s_bad = 0;
    }
    __syncthreads();
    const double shift = attempt == 0 ? 0.0 : 11.0 * (double(n) * l + double(l) * (l + 1)) * 1.1102230246251565e-16 * s_tr;
    for (int q = threadIdx.x; q < l * l; q += kBlock) {
      const int i = q / l, j = q % l;
      L[q] = Gb[i * LP + j] + (i == j ? shift : 0.0);
    }
    __syncthreads();
    for (int j = 0; j < l; ++j) {
      if (threadIdx.x == 0) {
        const double piv = L[j * l + j];
        if (!(piv > 0.0) || !isfinite(piv)) s_bad = 1;
        L[j * l + j] = sqrt(fmax(piv, 0.0));
      }
      __syncthreads();
      if (s_bad) break;
      const double d = L[j * l + j];
      for (int i = j + 1 + threadIdx.x; i < l; i += kBlock) L[i * l + j] /= d;
      __syncthreads();
      const int m = l - j - 1;  // trailing (m x m) lower triangle
      for (int q = threadIdx.x; q < m * m; q += kBlock) {
        const int i = j + 1 + q / m, c = j + 1 + q % m;
        if (c <= i) L[i * l + c] -= L[i * l + j] * L[c * l + j];
      }
      __syncthreads();
    }
    __syncthreads();
    if (!s_bad) break;
    __syncthreads();
  }
  if (s_bad) {
    if (threadIdx.x == 0) fail[b] = 1;
    return;
  }
  // X = L^-1 by forward substitution, one column per thread
  for (int cidx = threadIdx.x; cidx < l; cidx += kBlock) {
    for (int i = 0; i < l; ++i) X[i * l + cidx] = 0.0;
    for (int i = cidx; i < l; ++i) {
      double sacc = (i == cidx) ? 1.0 : 0.0;
      for (int m2 = cidx; m2 < i; ++m2) sacc -= L[i * l + m2] * X[m2 * l + cidx];
      X[i * l + cidx] = sacc / L[i * l + i];
    }
  }
  __syncthreads();
  double* Lb = Li + int64_t(b) * LP * LP;
  for (int q = threadIdx.x; q < LP * LP; q += kBlock) {
    const int i = q / LP, j = q % LP;
    Lb[q] = (i < l && j < l) ? X[i * l + j] : 0.0;
  }
}

// S = Y L^-T on a 64-row tile: S[r][j] = sum_{i<=j} Y[r][i] Linv[j][i] (j < l),
// zero for j >= l and rows >= n_b.  Writes S (row-major) and ST (transposed,
// the next GEMM operand: BF16 in the BF16 mode).
template <class TY, class TST>
__global__ __launch_bounds__(kBlock) void k_apply_rinv(BlockMeta bm, const TY* __restrict__ Y,
                                                       const double* __restrict__ Li, TY* __restrict__ S,
                                                       TST* __restrict__ ST, int64_t lo_off) {
  extern __shared__ double sm[];
  const int b = bm.item_b[blockIdx.x], t = bm.item_t[blockIdx.x];
  const int n = bm.off[b + 1] - bm.off[b], nbp = bm.nbp[b];
  const int l = bm.l, LP = bm.LP;
  double* Lt = sm;                  // l x l
  double* Yt = sm + l * l;          // 64 x l
  const double* Lb = Li + int64_t(b) * LP * LP;
  for (int q = threadIdx.x; q < l * l; q += kBlock) Lt[q] = Lb[(q / l) * LP + q % l];
  const TY* Yb = Y + bm.yoff[b];
  for (int q = threadIdx.x; q < 64 * l; q += kBlock) {
    const int r = t * 64 + q / l;
    Yt[q] = r < n ? double(Yb[int64_t(r) * LP + q % l]) : 0.0;
  }
  __syncthreads();
  TY* Sb = S + bm.yoff[b];
  TST* STb = ST + bm.yoff[b];
  for (int q = threadIdx.x; q < 64 * LP; q += kBlock) {
    const int rr = q % 64, j = q / 64;  // consecutive threads: consecutive rows (coalesced ST)
    const int r = t * 64 + rr;
    double acc = 0.0;
    if (j < l && r < n) {
      const double* yr = Yt + rr * l;
      const double* lj = Lt + j * l;
      for (int i = 0; i <= j; ++i) acc += yr[i] * lj[i];
    }
    Sb[int64_t(r) * LP + j] = TY(acc);
    if constexpr (sizeof(TST) == 2) {
      // hi + lo BF16 pair (the lo half lives y_elems further on)
      const float f = float(acc);
      const uint16_t hi = f32_to_bf16_rne(f);
      STb[int64_t(j) * nbp + r] = hi;
      STb[lo_off + int64_t(j) * nbp + r] = f32_to_bf16_rne(f - bf16_to_f32(hi));
    } else {
      STb[int64_t(j) * nbp + r] = acc;
    }
  }
}

// --------------------------------------------------------------- Jacobi --

// Eigen-decomposition of the symmetric l x l matrix G_b (= B B') by parallel
// cyclic Jacobi (round-robin pairing: l/2 disjoint rotations per round, l-1
// rounds per sweep; rotation of Golub & Van Loan, sym.schur2).  Writes the k
// largest eigenvalues' square roots (singular values of B, decreasing) and
// the matching eigenvectors (columns of Ut, l x k).
__global__ __launch_bounds__(kBlock) void k_jacobi(BlockMeta bm, const double* __restrict__ G,
                                                   double* __restrict__ sig, double* __restrict__ Ut,
                                                   int max_sweeps) {
  extern __shared__ double sm[];
  const int b = blockIdx.x;
  const int l = bm.l, LP = bm.LP, kk = bm.kk;
  const int ne = l + (l & 1);  // even count (a dummy index pairs with the odd one out)
  const int half = ne / 2;
  double* A = sm;              // l x l
  double* V = sm + l * l;      // l x l
  double* cs = sm + 2 * l * l; // [half][2]
  int* pp = reinterpret_cast<int*>(cs + 2 * half);  // [half][2]
  __shared__ double s_off[4], s_diag[4];
  const double* Gb = G + int64_t(b) * LP * LP;
  for (int q = threadIdx.x; q < l * l; q += kBlock) {
    const int i = q / l, j = q % l;
    A[q] = Gb[i * LP + j];
    V[q] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // convergence: off-diagonal mass against the diagonal (fixed-order sums)
    double off = 0.0, dg = 0.0;
    for (int q = threadIdx.x; q < l * l; q += kBlock) {
      const int i = q / l, j = q % l;
      if (i != j) off += A[q] * A[q]; else dg += A[q] * A[q];
    }
    for (int o2 = 32; o2 >= 1; o2 >>= 1) {
      off += __shfl_xor(off, o2, kWave);
      dg += __shfl_xor(dg, o2, kWave);
    }
    if (threadIdx.x % kWave == 0) {
      s_off[threadIdx.x / kWave] = off;
      s_diag[threadIdx.x / kWave] = dg;
    }
    __syncthreads();
    const double off_t = ((s_off[0] + s_off[1]) + s_off[2]) + s_off[3];
    const double dg_t = ((s_diag[0] + s_diag[1]) + s_diag[2]) + s_diag[3];
    __syncthreads();
    if (off_t <= 1e-30 * dg_t) break;
    for (int round = 0; round < ne - 1; ++round) {
      for (int pr = threadIdx.x; pr < half; pr += kBlock) {
        // circle method: slot 0 fixed, the others rotate
        auto at = [&](int slot) { return slot == 0 ? 0 : 1 + ((slot - 1 + round) % (ne - 1)); };
        int p = at(pr), q = at(ne - 1 - pr);
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        double c = 1.0, s = 0.0;
        if (q < l) {
          const double apq = A[p * l + q];
          if (fabs(apq) > 1e-300) {
            const double tau = (A[q * l + q] - A[p * l + p]) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
        pp[2 * pr] = p;
        pp[2 * pr + 1] = q;
        cs[2 * pr] = c;
        cs[2 * pr + 1] = s;
      }
      __syncthreads();
      // rows: A <- J' A
      for (int w = threadIdx.x; w < half * l; w += kBlock) {
        const int pr = w / l, col = w % l;
        const int p = pp[2 * pr], q = pp[2 * pr + 1];
        if (q >= l) continue;
        const double c = cs[2 * pr], s = cs[2 * pr + 1];
        const double ap = A[p * l + col], aq = A[q * l + col];
        A[p * l + col] = c * ap - s * aq;
        A[q * l + col] = s * ap + c * aq;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int w = threadIdx.x; w < half * l; w += kBlock) {
        const int pr = w / l, row = w % l;
        const int p = pp[2 * pr], q = pp[2 * pr + 1];
        if (q >= l) continue;
        const double c = cs[2 * pr], s = cs[2 * pr + 1];
        const double ap = A[row * l + p], aq = A[row * l + q];
        A[row * l + p] = c * ap - s * aq;
        A[row * l + q] = s * ap + c * aq;
        const double vp = V[row * l + p], vq = V[row * l + q];
        V[row * l + p] = c * vp - s * vq;
        V[row * l + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  // rank by decreasing eigenvalue (ties by index): output the leading kk
  for (int i = threadIdx.x; i < l; i += kBlock) {
    const double li = A[i * l + i];
    int rank = 0;
    for (int j = 0; j < l; ++j) {
      const double lj = A[j * l + j];
      rank += (lj > li) || (lj == li && j < i);
    }
    if (rank < kk) {
      sig[int64_t(b) * kk + rank] = sqrt(fmax(li, 0.0));
      for (int r = 0; r < l; ++r) Ut[int64_t(b) * LP * kk + int64_t(r) * kk + rank] = V[r * l + i];
    }
  }
}

// U[o_b + r][c] = sum_{i<l} S_b[r][i] Ut_b[i][c], c < kk (global N x kk, FP32).
template <class TY>
__global__ __launch_bounds__(kBlock) void k_basis(BlockMeta bm, const TY* __restrict__ S,
                                                  const double* __restrict__ Ut, float* __restrict__ U) {
  const int b = bm.item_b[blockIdx.x], t = bm.item_t[blockIdx.x];
  const int o = bm.off[b], n = bm.off[b + 1] - o;
  const int l = bm.l, LP = bm.LP, kk = bm.kk;
  const double* Ub = Ut + int64_t(b) * LP * kk;
  const TY* Sb = S + bm.yoff[b];
  for (int q = threadIdx.x; q < 64 * kk; q += kBlock) {
    const int r = t * 64 + q / kk, c = q % kk;
    if (r >= n) continue;
    double acc = 0.0;
    for (int i = 0; i < l; ++i) acc += double(Sb[int64_t(r) * LP + i]) * Ub[int64_t(i) * kk + c];
    U[int64_t(o + r) * kk + c] = float(acc);
  }
}

// ------------------------------------------------ block preconditioner --

// dT_b = diag(d_b) U_b' R_b for 64 columns of R per launch column slab:
// d_i = sigma_i / (1 + lambda - sigma_i).  One workgroup per (block, slab).
constexpr int kPrecT = 24;  // outputs per thread: kk * 64 <= 256 * kPrecT
template <class T>
__global__ __launch_bounds__(kBlock) void k_prec_t(BlockMeta bm, const float* __restrict__ U,
                                                   const double* __restrict__ sig, double lam,
                                                   const T* __restrict__ R, int64_t ldr, int nrhs,
                                                   double* __restrict__ dT) {
  __shared__ float su[32 * kMaxLP];
  __shared__ double sr[32 * 64];
  const int b = blockIdx.x, c0 = blockIdx.y * 64;
  const int o = bm.off[b], n = bm.off[b + 1] - o, kk = bm.kk;
  const int nc = min(64, nrhs - c0);
  double acc[kPrecT];
#pragma unroll
  for (int a = 0; a < kPrecT; ++a) acc[a] = 0.0;
  for (int r0 = 0; r0 < n; r0 += 32) {
    const int rows = min(32, n - r0);
    __syncthreads();
    for (int q = threadIdx.x; q < rows * kk; q += kBlock) su[q] = U[int64_t(o + r0 + q / kk) * kk + q % kk];
    for (int q = threadIdx.x; q < rows * 64; q += kBlock) {
      const int rr = q / 64, cc = q % 64;
      sr[q] = cc < nc ? double(R[int64_t(o + r0 + rr) * ldr + c0 + cc]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < kPrecT; ++a) {
      const int w = threadIdx.x + a * kBlock;
      if (w < kk * 64) {
        const int i = w / 64, cc = w % 64;
        double sacc = acc[a];
        for (int rr = 0; rr < rows; ++rr) sacc += double(su[rr * kk + i]) * sr[rr * 64 + cc];
        acc[a] = sacc;
      }
    }
  }
#pragma unroll
  for (int a = 0; a < kPrecT; ++a) {
    const int w = threadIdx.x + a * kBlock;
    if (w < kk * 64) {
      const int i = w / 64, cc = w % 64;
      if (cc < nc) {
        const double si = sig[int64_t(b) * kk + i];
        dT[(int64_t(b) * kk + i) * nrhs + c0 + cc] = acc[a] * si / (1.0 + lam - si);
      }
    }
  }
}

// Z = lambda/(1+lambda) (R + U dT_b) row by row over the CG tiles, with the
// partial inner products <R_j, Z_j> per tile (long-row slots zeroed).
template <class T, int GL, int V>
__global__ __launch_bounds__(kBlock) void k_prec_z(BlockMeta bm, int32_t n_tiles, const int32_t* __restrict__ tile_r0,
                                                   const int32_t* __restrict__ tile_r1, int n_slots, int n_long,
                                                   const float* __restrict__ U, const double* __restrict__ dT,
                                                   double g, const T* __restrict__ R, int64_t ldr,
                                                   T* __restrict__ Z, int64_t ldz, int nrhs,
                                                   double* __restrict__ part, Gate gate) {
  if (gate.skip()) return;
  constexpr int GPB = kBlock / GL, W = GL * V;
  __shared__ double lds[4 * W];
  const int grp = threadIdx.x / GL, lane = threadIdx.x % GL;
  const int col = blockIdx.y * W + lane * V;
  const int t = blockIdx.x;
  const int kk = bm.kk;
  double dot[V];
#pragma unroll
  for (int i = 0; i < V; ++i) dot[i] = 0.0;
  if (col < nrhs) {
    for (int r = tile_r0[t] + grp; r < tile_r1[t]; r += GPB) {
      // block of row r: largest b with off[b] <= r
      int lo = 0, hi = bm.nb - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bm.off[mid] <= r) lo = mid; else hi = mid - 1;
      }
      const double* dTb = dT + int64_t(lo) * kk * nrhs;
      const float* ur = U + int64_t(r) * kk;
      double acc[V];
      T rv[V], zv[V];
      load_row<V>(R + int64_t(r) * ldr + col, rv);
#pragma unroll
      for (int i = 0; i < V; ++i) acc[i] = double(rv[i]);
      for (int i = 0; i < kk; ++i) {
        const double ui = double(ur[i]);
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] += ui * dTb[int64_t(i) * nrhs + col + v];
      }
#pragma unroll
      for (int i = 0; i < V; ++i) {
        zv[i] = T(g * acc[i]);
        dot[i] += double(rv[i]) * double(zv[i]);
      }
      store_row<V>(Z + int64_t(r) * ldz + col, zv);
    }
  }
  if (part) {
    double s = block_colsum<GL, V>(dot, lds);
    const int c = blockIdx.y * W + threadIdx.x;
    if (threadIdx.x < W && c < nrhs) part[int64_t(c) * n_slots + t] = s;
    if (blockIdx.y == 0) {
      const int64_t total = int64_t(n_long) * nrhs;
      for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
           i += int64_t(gridDim.x) * blockDim.x)
        part[(i / n_long) * n_slots + n_tiles + i % n_long] = 0.0;
    }
  }
}

// -------------------------------------------------------------- driver --

struct Rsvd {
  int nb = 0, l = 0, LP = 0, kk = 0;
  bool f64 = false;
  std::vector<int32_t> off, nbp, item_b, item_t;
  std::vector<int64_t> aoff, yoff;
  int64_t a_elems = 0, y_elems = 0;
  int max_nbp = 0;
  // device
  DevBuf meta, A, Y, S, ST, G, Li, Ut, sig, fail, omega;
  BlockMeta bm{};
};

static int rsvd_setup(hgl_handle* h, Rsvd& R, int n_blocks, const int32_t* offs, const hgl_rsvd_opts* o,
                      hipStream_t s) {
  R.nb = n_blocks;
  R.l = o->k + o->p;
  R.kk = o->k;
  R.LP = (R.l + 15) / 16 * 16;
  R.f64 = o->sketch == HGL_SKETCH_F64;
  R.off.assign(offs, offs + n_blocks + 1);
  R.nbp.resize(n_blocks);
  R.aoff.resize(n_blocks);
  R.yoff.resize(n_blocks);
  int64_t a = 0, y = 0;
  for (int b = 0; b < n_blocks; ++b) {
    const int n = offs[b + 1] - offs[b];
    const int p = (n + 63) / 64 * 64;
    R.nbp[b] = p;
    R.max_nbp = std::max(R.max_nbp, p);
    R.aoff[b] = a;
    R.yoff[b] = y;
    a += int64_t(p) * p;
    y += int64_t(p) * R.LP;
    for (int t = 0; t < p / 64; ++t) {
      R.item_b.push_back(b);
      R.item_t.push_back(t);
    }
  }
  R.a_elems = a;
  R.y_elems = y;
  const size_t nI = R.item_b.size();
  const size_t meta_bytes = 4 * (n_blocks + 1) + 4 * n_blocks + 8 * 2 * n_blocks + 4 * 2 * nI + 64;
  HGL_TRY(R.meta.reserve(meta_bytes));
  std::vector<char> host(meta_bytes, 0);
  size_t pos = 0;
  auto put = [&](const void* src, size_t bytes, size_t align) {
    pos = (pos + align - 1) / align * align;
    std::memcpy(host.data() + pos, src, bytes);
    const size_t at = pos;
    pos += bytes;
    return at;
  };
  const size_t p_aoff = put(R.aoff.data(), 8 * n_blocks, 8);
  const size_t p_yoff = put(R.yoff.data(), 8 * n_blocks, 8);
  const size_t p_off = put(R.off.data(), 4 * (n_blocks + 1), 4);
  const size_t p_nbp = put(R.nbp.data(), 4 * n_blocks, 4);
  const size_t p_ib = put(R.item_b.data(), 4 * nI, 4);
  const size_t p_it = put(R.item_t.data(), 4 * nI, 4);
  HGL_TRY(ensure_pinned(h, (pos + 7) / 8 + 8));
  std::memcpy(h->pinned_d, host.data(), pos);
  HGL_HIP(hipMemcpyAsync(R.meta.p, h->pinned_d, pos, hipMemcpyHostToDevice, s));
  HGL_HIP(hipStreamSynchronize(s));
  char* base = static_cast<char*>(R.meta.p);
  R.bm = BlockMeta{n_blocks, R.l, R.LP, R.kk,
                   reinterpret_cast<const int32_t*>(base + p_off), reinterpret_cast<const int32_t*>(base + p_nbp),
                   reinterpret_cast<const int64_t*>(base + p_aoff), reinterpret_cast<const int64_t*>(base + p_yoff),
                   reinterpret_cast<const int32_t*>(base + p_ib), reinterpret_cast<const int32_t*>(base + p_it)};
  const size_t ea = R.f64 ? 8 : 2, ey = R.f64 ? 8 : 4;
  HGL_TRY(R.A.reserve(ea * R.a_elems));
  HGL_TRY(R.Y.reserve(ey * R.y_elems));
  HGL_TRY(R.S.reserve(ey * R.y_elems));
  HGL_TRY(R.ST.reserve(ea * R.y_elems * (R.f64 ? 1 : 2)));  // BF16: hi and lo halves
  HGL_TRY(R.G.reserve(8 * size_t(n_blocks) * R.LP * R.LP));
  HGL_TRY(R.Li.reserve(8 * size_t(n_blocks) * R.LP * R.LP));
  HGL_TRY(R.Ut.reserve(8 * size_t(n_blocks) * R.LP * R.kk));
  HGL_TRY(R.sig.reserve(8 * size_t(n_blocks) * R.kk));
  HGL_TRY(R.fail.reserve(4 * size_t(n_blocks)));
  HGL_HIP(hipMemsetAsync(R.fail.p, 0, 4 * size_t(n_blocks), s));
  return HGL_OK;
}

// Kernels whose dynamic LDS exceeds the default 64 KiB must opt in (gfx950
// has 160 KiB of LDS per CU).
template <class K>
static int allow_lds(K kernel, size_t bytes) {
  if (bytes > 160 * 1024) {
    set_error("kernel needs %zu bytes of LDS", bytes);
    return HGL_EUNSUPPORTED;
  }
  if (bytes > 64 * 1024)
    HGL_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
  return HGL_OK;
}

static int launch_gemm(Rsvd& R, hipStream_t s) {
  const int n_items = int(R.item_b.size());
  if (R.f64) {
    hipLaunchKernelGGL(k_gemm_f64, dim3(n_items), dim3(kBlock), 0, s, R.bm, R.A.as<double>(),
                       R.ST.as<double>(), R.Y.as<double>());
  } else {
    const uint16_t* A = R.A.as<uint16_t>();
    const uint16_t* ST = R.ST.as<uint16_t>();
    float* Y = R.Y.as<float>();
    const int64_t lo = R.y_elems;
    const dim3 g(n_items), blk(kBlock);
    switch (R.LP) {
      case 16: hipLaunchKernelGGL(k_gemm_bf16<16>, g, blk, 0, s, R.bm, A, ST, lo, Y); break;
      case 32: hipLaunchKernelGGL(k_gemm_bf16<32>, g, blk, 0, s, R.bm, A, ST, lo, Y); break;
      case 48: hipLaunchKernelGGL(k_gemm_bf16<48>, g, blk, 0, s, R.bm, A, ST, lo, Y); break;
      case 64: hipLaunchKernelGGL(k_gemm_bf16<64>, g, blk, 0, s, R.bm, A, ST, lo, Y); break;
      case 80: hipLaunchKernelGGL(k_gemm_bf16<80>, g, blk, 0, s, R.bm, A, ST, lo, Y); break;
      case 96: hipLaunchKernelGGL(k_gemm_bf16<96>, g, blk, 0, s, R.bm, A, ST, lo, Y); break;
      default: set_error("unsupported padded sketch width %d", R.LP); return HGL_EUNSUPPORTED;
    }
  }
  HGL_HIP(hipGetLastError());
  return HGL_OK;
}

template <class TY>
static int launch_gram(Rsvd& R, const DevBuf& Yb, hipStream_t s) {
  hipLaunchKernelGGL((k_gram<TY>), dim3(R.nb), dim3(kBlock), 0, s, R.bm, Yb.as<TY>(), R.G.as<double>());
  HGL_HIP(hipGetLastError());
  return HGL_OK;
}

// S, ST <- orth(Y) by CholQR2 (Y is overwritten by the first pass).
template <class TY, class TST>
static int cholqr2(hgl_handle* h, Rsvd& R, hipStream_t s) {
  const int n_items = int(R.item_b.size());
  const size_t lds_chol = sizeof(double) * 2 * R.l * R.l;
  const size_t lds_rinv = sizeof(double) * (R.l * R.l + 64 * R.l);
  HGL_TRY(allow_lds(k_chol_inv, lds_chol));
  HGL_TRY(allow_lds(k_apply_rinv<TY, TST>, lds_rinv));
  prof_begin(h, kProfQr, s);
  for (int pass = 0; pass < 2; ++pass) {
    DevBuf& in = pass == 0 ? R.Y : R.S;
    DevBuf& out = pass == 0 ? R.S : R.Y;
    HGL_TRY(launch_gram<TY>(R, in, s));
    hipLaunchKernelGGL(k_chol_inv, dim3(R.nb), dim3(kBlock), lds_chol, s, R.bm, R.G.as<double>(),
                       R.Li.as<double>(), R.fail.as<int32_t>());
    hipLaunchKernelGGL((k_apply_rinv<TY, TST>), dim3(n_items), dim3(kBlock), lds_rinv, s, R.bm, in.as<TY>(),
                       R.Li.as<double>(), out.as<TY>(), R.ST.as<TST>(), R.y_elems);
    HGL_HIP(hipGetLastError());
  }
  prof_end(h, s);
  // after two passes the basis is in R.Y; keep it in R.S
  std::swap(R.Y, R.S);
  return HGL_OK;
}

template <class TY, class TST>
static int run_rsvd(hgl_handle* h, Rsvd& R, const hgl_rsvd_opts* o, const uint16_t* omega, hipStream_t s) {
  // 1. dense diagonal blocks A_bb
  const size_t lds_ex = sizeof(double) * 4 * R.max_nbp;
  if (lds_ex > 160 * 1024) {
    set_error("diagonal block too large for LDS staging (%d rows)", R.max_nbp);
    return HGL_EUNSUPPORTED;
  }
  {
    dim3 grid((R.max_nbp + 3) / 4, R.nb);
    prof_begin(h, kProfExtract, s);
    if (R.f64) {
      HGL_TRY(allow_lds(k_extract_blocks<double>, lds_ex));
      hipLaunchKernelGGL((k_extract_blocks<double>), grid, dim3(kBlock), lds_ex, s, R.bm, h->vtx_ptr, h->vtx_edge,
                         h->edge_ptr, h->edge_vtx, h->s64, h->c64, R.A.as<double>(), R.max_nbp);
    } else {
      HGL_TRY(allow_lds(k_extract_blocks<uint16_t>, lds_ex));
      hipLaunchKernelGGL((k_extract_blocks<uint16_t>), grid, dim3(kBlock), lds_ex, s, R.bm, h->vtx_ptr, h->vtx_edge,
                         h->edge_ptr, h->edge_vtx, h->s64, h->c64, R.A.as<uint16_t>(), R.max_nbp);
    }
    HGL_HIP(hipGetLastError());
    prof_end(h, s);
  }
  // 2. sketch Omega (caller's, or Philox from the seed) into ST
  const uint16_t* om = omega;
  if (!om) {
    HGL_TRY(R.omega.reserve(sizeof(uint16_t) * size_t(h->N) * R.l + 16));
    const int64_t pairs = (int64_t(h->N) * R.l + 1) / 2;
    hipLaunchKernelGGL(k_philox_sketch, dim3(int((pairs + 255) / 256)), dim3(256), 0, s, int64_t(h->N), R.l,
                       o->seed, R.omega.as<uint16_t>());
    om = R.omega.as<uint16_t>();
  }
  hipLaunchKernelGGL((k_sketch_to_st<TST>), dim3(64, R.nb), dim3(256), 0, s, R.bm, om, R.ST.as<TST>(),
                     R.y_elems);
  HGL_HIP(hipGetLastError());
  // 3. Y = A Omega, S = orth(Y); q subspace iterations
  auto gemm = [&]() -> int {
    prof_begin(h, kProfGemm, s);
    const int st = launch_gemm(R, s);
    prof_end(h, s);
    return st;
  };
  HGL_TRY(gemm());
  HGL_TRY((cholqr2<TY, TST>(h, R, s)));
  for (int i = 0; i < 2 * o->q; ++i) {
    HGL_TRY(gemm());
    HGL_TRY((cholqr2<TY, TST>(h, R, s)));
  }
  // 4. W = A S; B B' = W'W; Jacobi; U = S U~
  HGL_TRY(gemm());  // W in R.Y, basis S in R.S
  prof_begin(h, kProfEig, s);
  HGL_TRY(launch_gram<TY>(R, R.Y, s));
  const int half = (R.l + (R.l & 1)) / 2;
  const size_t lds_j = sizeof(double) * (2 * R.l * R.l + 2 * half) + sizeof(int) * 2 * half + 16;
  HGL_TRY(allow_lds(k_jacobi, lds_j));
  hipLaunchKernelGGL(k_jacobi, dim3(R.nb), dim3(kBlock), lds_j, s, R.bm, R.G.as<double>(), R.sig.as<double>(),
                     R.Ut.as<double>(), 30);
  HGL_HIP(hipGetLastError());
  prof_end(h, s);
  return HGL_OK;
}

static int check_opts(hgl_handle* h, int n_blocks, const int32_t* offs, const hgl_rsvd_opts* o) {
  HGL_CHECK_ARG(h != nullptr && o != nullptr, "handle and opts must not be NULL");
  HGL_CHECK_ARG(h->G == 1, "block rSVD needs a single-graph handle");
  HGL_CHECK_ARG(n_blocks >= 1 && offs != nullptr, "need at least one block");
  HGL_CHECK_ARG(offs[0] == 0 && offs[n_blocks] == h->N, "block offsets must cover [0, N)");
  for (int b = 0; b < n_blocks; ++b)
    HGL_CHECK_ARG(offs[b + 1] > offs[b], "block %d is empty or offsets decrease", b);
  HGL_CHECK_ARG(o->k >= 1 && o->p >= 0 && o->q >= 0, "need k >= 1, p >= 0, q >= 0");
  HGL_CHECK_ARG(o->k + o->p <= kMaxLP, "k + p must be <= %d", kMaxLP);
  HGL_CHECK_ARG(o->sketch == HGL_SKETCH_BF16 || o->sketch == HGL_SKETCH_F64, "unknown sketch precision");
  for (int b = 0; b < n_blocks; ++b)
    HGL_CHECK_ARG(offs[b + 1] - offs[b] >= o->k + o->p,
                  "block %d has %d rows, fewer than k + p = %d", b, offs[b + 1] - offs[b], o->k + o->p);
  return HGL_OK;
}

static int finish_rsvd(hgl_handle* h, Rsvd& R, float* U_out, double* sigma_out, hipStream_t s) {
  const int n_items = int(R.item_b.size());
  if (R.f64)
    hipLaunchKernelGGL((k_basis<double>), dim3(n_items), dim3(kBlock), 0, s, R.bm, R.S.as<double>(),
                       R.Ut.as<double>(), U_out);
  else
    hipLaunchKernelGGL((k_basis<float>), dim3(n_items), dim3(kBlock), 0, s, R.bm, R.S.as<float>(),
                       R.Ut.as<double>(), U_out);
  HGL_HIP(hipGetLastError());
  if (sigma_out)
    HGL_HIP(hipMemcpyAsync(sigma_out, R.sig.p, sizeof(double) * R.nb * R.kk, hipMemcpyDeviceToDevice, s));
  HGL_HIP(hipMemcpyAsync(h->pinned_i, R.fail.p, sizeof(int32_t) * std::min(R.nb, 32), hipMemcpyDeviceToHost, s));
  HGL_HIP(hipStreamSynchronize(s));
  // any block: reduce the flags on the host in chunks of 32
  for (int b0 = 0; b0 < R.nb; b0 += 32) {
    if (b0 > 0) {
      HGL_HIP(hipMemcpyAsync(h->pinned_i, R.fail.as<int32_t>() + b0, sizeof(int32_t) * std::min(R.nb - b0, 32),
                             hipMemcpyDeviceToHost, s));
      HGL_HIP(hipStreamSynchronize(s));
    }
    for (int i = 0; i < std::min(R.nb - b0, 32); ++i)
      if (h->pinned_i[i]) {
        set_error("CholQR failed on diagonal block %d (rank-deficient sketch)", b0 + i);
        return HGL_ECHOLQR;
      }
  }
  return HGL_OK;
}

static int rsvd_any(hgl_handle* h, Rsvd& R, const hgl_rsvd_opts* o, const uint16_t* omega, hipStream_t s) {
  if (R.f64) return run_rsvd<double, double>(h, R, o, omega, s);
  return run_rsvd<float, uint16_t>(h, R, o, omega, s);
}

// Block preconditioner for CG: Z = blockdiag(M_bb^-1 approx) R.
struct BlockPrec {
  hgl_handle* h;
  Rsvd* R;
  const float* U;
  double lam;
  DevBuf* dT;
};

template <class T>
static int prec_apply(void* ctx, const T* Rm, int64_t ldr, T* Z, int64_t ldz, double* part, int nrhs, Gate gate,
                      hipStream_t s) {
  BlockPrec* P = static_cast<BlockPrec*>(ctx);
  Rsvd& R = *P->R;
  hgl_handle* h = P->h;
  hipLaunchKernelGGL((k_prec_t<T>), dim3(R.nb, (nrhs + 63) / 64), dim3(kBlock), 0, s, R.bm, P->U,
                     R.sig.as<double>(), P->lam, Rm, ldr, nrhs, P->dT->as<double>());
  HGL_HIP(hipGetLastError());
  const ColShape cs = pick_shape(nrhs, sizeof(T), {Rm, Z}, {ldr, ldz});
  const double g = P->lam / (1.0 + P->lam);
  return HGL_DISPATCH_SHAPE(cs, sizeof(T), {
    hipLaunchKernelGGL((k_prec_z<T, GL, V>), dim3(h->n_tiles, cs.slabs), dim3(kBlock), 0, s, R.bm, h->n_tiles,
                       h->tile_r0, h->tile_r1, n_slots(h), h->n_long, P->U, P->dT->as<double>(), g, Rm, ldr, Z,
                       ldz, nrhs, part, gate);
    HGL_HIP(hipGetLastError());
    return HGL_OK;
  });
}

}  // namespace hgl

using namespace hgl;

extern "C" int hgl_block_rsvd(hgl_handle* h, int32_t n_blocks, const int32_t* block_offsets_host,
                              const hgl_rsvd_opts* o, const uint16_t* omega_bf16, float* U_out,
                              double* sigma_out, hipStream_t s) {
  clear_error();
  HGL_TRY(check_opts(h, n_blocks, block_offsets_host, o));
  HGL_CHECK_ARG(U_out != nullptr, "U_out must not be NULL");
  Rsvd R;
  HGL_TRY(rsvd_setup(h, R, n_blocks, block_offsets_host, o, s));
  HGL_TRY(rsvd_any(h, R, o, omega_bf16, s));
  return finish_rsvd(h, R, U_out, sigma_out, s);
}

extern "C" int hgl_block_rsvd_invert(hgl_handle* h, double lambda, int32_t n_blocks,
                                     const int32_t* block_offsets_host, const hgl_rsvd_opts* o,
                                     const uint16_t* omega_bf16, const float* Y, int64_t ldy, float* F,
                                     int64_t ldf, int32_t nrhs, double* sigma_out, int32_t* iters_host,
                                     double* relres_host, hipStream_t s) {
  clear_error();
  HGL_TRY(check_opts(h, n_blocks, block_offsets_host, o));
  HGL_CHECK_ARG(lambda > 0.0 && std::isfinite(lambda), "lambda must be > 0");
  HGL_CHECK_ARG(Y && F && nrhs >= 1 && ldy >= nrhs && ldf >= nrhs, "bad Y/F/nrhs/leading dimensions");
  HGL_CHECK_ARG(o->refine_tol > 0.0, "refine_tol must be > 0");
  Rsvd R;
  HGL_TRY(rsvd_setup(h, R, n_blocks, block_offsets_host, o, s));
  HGL_TRY(rsvd_any(h, R, o, omega_bf16, s));
  DevBuf U, dT;
  HGL_TRY(U.reserve(sizeof(float) * size_t(h->N) * R.kk));
  HGL_TRY(dT.reserve(sizeof(double) * size_t(n_blocks) * R.kk * nrhs));
  int st = finish_rsvd(h, R, U.as<float>(), sigma_out, s);
  if (st < 0) {
    U.release();
    dT.release();
    return st;
  }
  BlockPrec bp{h, &R, U.as<float>(), lambda, &dT};
  Precond pc;
  pc.ctx = &bp;
  pc.apply_f32 = &prec_apply<float>;
  pc.apply_f64 = &prec_apply<double>;
  hgl_cg_opts co{};
  co.mode = HGL_CG_F32_F64DOT_RR;
  co.tol = o->refine_tol;
  co.max_iter = o->max_refine;
  co.x0_given = 0;
  co.rr_period = 0;
  co.chunk = o->chunk;
  std::vector<double> lams(h->G, lambda);
  st = cg_run(h, lams.data(), &co, Y, ldy, F, ldf, nrhs, iters_host, relres_host, &pc, s);
  HGL_HIP(hipStreamSynchronize(s));
  U.release();
  dT.release();
  return st;
}

extern "C" int hgl_sketch_gaussian(int64_t rows, int32_t l, uint64_t seed, uint16_t* out_bf16, hipStream_t s) {
  clear_error();
  HGL_CHECK_ARG(rows >= 1 && l >= 1 && out_bf16 != nullptr, "bad sketch arguments");
  const int64_t pairs = (rows * l + 1) / 2;
  hipLaunchKernelGGL(k_philox_sketch, dim3(int((pairs + 255) / 256)), dim3(256), 0, s, rows, l, seed, out_bf16);
  HGL_HIP(hipGetLastError());
  return HGL_OK;
}
