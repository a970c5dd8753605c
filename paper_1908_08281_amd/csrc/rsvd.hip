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
#include <functional>
#include <type_traits>

#include "kernels.h"

namespace hgl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kMaxLP = 96;
constexpr int kGroups = 2;   // concurrent chains of blocks (see Grp)

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
  const int32_t* pair_b; // [n_pairs] block of a 128-row item (two tiles, or the block's last one)
  const int32_t* pair_t; // [n_pairs] its first tile index
  const int32_t* gemm_b; // [n_gemm] the 128-row items in XCD order (block -1: none)
  const int32_t* gemm_t;
  // a launch over a group of blocks adds these to its workgroup index: the
  // first block (per-block kernels), 128-row item (per-item kernels), 64-row
  // item and GEMM-list entry of the group
  int32_t b0 = 0, p0 = 0, i0 = 0, g0 = 0;
};

// Lane src's value of v (src uniform), both halves by v_readlane.
__device__ __forceinline__ double lane_read(double v, int src) {
  const uint64_t u = __double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readlane(uint32_t(u), src);
  const uint32_t hi = __builtin_amdgcn_readlane(uint32_t(u >> 32), src);
  return __longlong_as_double((int64_t(hi) << 32) | lo);
}

// A wave's LDS accesses complete in issue order; this keeps the compiler
// from moving them across the point either.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------ extraction --

// A_bb[u][v] = s_u s_v sum_{e containing u and v} c_e for u, v in block b.
// One wave per row u, 8 rows per workgroup; the row is accumulated in LDS
// (FP32 for a BF16 block, FP64 otherwise).  Lane i loads the metadata of
// u's i-th hyperedge of a 64-hyperedge chunk (id, c_e, member range); the
// member loads of four hyperedges at a time are issued together; the row
// updates are LDS atomic adds issued in hyperedge order, which a wave's LDS
// applies in issue order, so the sums are deterministic (members of one
// hyperedge are distinct, so no two lanes of one add touch one entry).
constexpr int kExW = 8;
template <class TA>
__global__ __launch_bounds__(kExW * kWave) void k_extract_blocks(BlockMeta bm, const int32_t* __restrict__ vtx_ptr,
                                                                 const int32_t* __restrict__ vtx_edge,
                                                                 const int32_t* __restrict__ edge_ptr,
                                                                 const int32_t* __restrict__ edge_vtx,
                                                                 const double* __restrict__ s,
                                                                 const double* __restrict__ c, TA* __restrict__ A,
                                                                 int max_nbp) {
  using TC = std::conditional_t<sizeof(TA) == 2, float, double>;
  extern __shared__ double srow_raw[];
  TC* const srow = reinterpret_cast<TC*>(srow_raw);   // [kExW][max_nbp]
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int b = bm.b0 + blockIdx.y;
  const int o = bm.off[b], n = bm.off[b + 1] - o, nbp = bm.nbp[b];
  const int ur = blockIdx.x * kExW + wave;  // row within the padded block
  if (blockIdx.x * kExW >= nbp) return;
  TC* row = srow + int64_t(wave) * max_nbp;
  for (int j = lane; j < nbp; j += kWave) row[j] = TC(0);
  wave_sync();
  if (ur < n) {
    const int u = o + ur;
    const int q0 = vtx_ptr[u], q1 = vtx_ptr[u + 1];
    for (int qb = q0; qb < q1; qb += kWave) {
      int eb = 0, en = 0;
      TC ce = TC(0);
      if (qb + lane < q1) {
        const int e = vtx_edge[qb + lane];
        ce = TC(c[e]);
        eb = edge_ptr[e];
        en = edge_ptr[e + 1];
      }
      const int cnt = min(kWave, q1 - qb);
      for (int i0 = 0; i0 < cnt; i0 += 4) {
        int vv[4], beg[4], end[4];
        TC cc[4], sv[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int i = min(i0 + g, cnt - 1);
          const bool ok = i0 + g < cnt;
          beg[g] = ok ? __builtin_amdgcn_readlane(eb, i) : 0;
          end[g] = ok ? __builtin_amdgcn_readlane(en, i) : 0;
          if constexpr (sizeof(TC) == 4) {
            cc[g] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ce), i));
          } else {
            cc[g] = lane_read(ce, i);
          }
          const int m = beg[g] + lane;
          vv[g] = m < min(end[g], beg[g] + kWave) ? edge_vtx[m] : -1;
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) sv[g] = (vv[g] >= o && vv[g] < o + n) ? TC(s[vv[g]]) : TC(0);
#pragma unroll
        for (int g = 0; g < 4; ++g)
          if (vv[g] >= o && vv[g] < o + n) atomicAdd(&row[vv[g] - o], cc[g] * sv[g]);
        // members past the first 64 (large hyperedges), in hyperedge order
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          for (int m = beg[g] + kWave + lane; m < end[g]; m += kWave) {
            const int v = edge_vtx[m];
            if (v >= o && v < o + n) atomicAdd(&row[v - o], cc[g] * TC(s[v]));
          }
        }
      }
    }
  }
  wave_sync();
  if (ur < nbp) {
    const double su = ur < n ? s[o + ur] : 0.0;
    TA* dst = A + bm.aoff[b] + int64_t(ur) * nbp;
    for (int j = lane; j < nbp; j += kWave) {
      const double v = su * double(row[j]);
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

// out[4i .. 4i+3] = Philox4x32-10 of counter ctr[4i .. 4i+3] under key.
__global__ void k_philox_words(int64_t n, const uint32_t* __restrict__ ctr, uint64_t key,
                               uint32_t* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t c[4] = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
  philox4x32_10(c, uint32_t(key), uint32_t(key >> 32));
#pragma unroll
  for (int j = 0; j < 4; ++j) out[4 * i + j] = c[j];
}

// ST_b[j][r] = Omega[o_b + r][j] for j < l, r < n_b; zero elsewhere.
template <class TS>
__global__ void k_sketch_to_st(BlockMeta bm, const uint16_t* __restrict__ omega, TS* __restrict__ ST,
                               int64_t lo_off) {
  const int b = bm.b0 + blockIdx.y;
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
constexpr int kGemmT = 256;   // 4 waves of 32 rows: one 128-row item
template <int LP>
__global__ __launch_bounds__(kGemmT) void k_gemm_bf16(BlockMeta bm, const uint16_t* __restrict__ A,
                                                      const uint16_t* __restrict__ ST, int64_t lo_off,
                                                      float* __restrict__ Y) {
  constexpr int NT = LP / 16;
  const int b = bm.gemm_b[bm.g0 + blockIdx.x], t = bm.gemm_t[bm.g0 + blockIdx.x];
  if (b < 0) return;   // padding of the XCD order
  const int nbp = bm.nbp[b];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int r0 = t * 64 + wave * 32;
  // a block's last tile may be alone in its item: the waves past it only
  // help stage S'
  const bool live = r0 < nbp;
  const int li = lane % 16, kq = lane / 16;
  const uint16_t* Ab = A + bm.aoff[b] + int64_t(live ? r0 + li : 0) * nbp + kq * 8;
  // S' (hi and lo) is shared by the four waves: stage 128-wide K chunks of
  // it in LDS (rows padded by 8 elements against bank conflicts); each wave
  // uses every S' fragment it reads for its two 16-row MFMA blocks
  constexpr int KC = 128, KP = KC + 8;
  __shared__ uint16_t sst[2 * LP * KP];
  const uint16_t* STb = ST + bm.yoff[b];
  floatx4 acc[2][NT];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[h][n] = floatx4{0.f, 0.f, 0.f, 0.f};
  // software pipeline over 128-wide K chunks, two deep: while a chunk's
  // MFMAs run, the A fragments and S' segments of the next two chunks are
  // in flight in registers (compile-time counts: 2 LP KC/8 segments over the
  // workgroup's threads, segments past the chunk's width skipped)
  constexpr int SEGS = KC / 8, NQ = 2 * LP * SEGS / kGemmT;
  static_assert(2 * LP * SEGS % kGemmT == 0, "copy loop");
  bf16x8 a[2][2][KC / 32], v[2][NQ];
  // (no branches around the loads: past a chunk's width the column is
  // clamped into the row, and the values land in LDS or registers that the
  // MFMA steps do not read; branches would make the compiler wait for every
  // load in flight before each store)
  auto fetch = [&](int k0, auto bufc) {
    constexpr int buf = decltype(bufc)::value;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int ks = 0; ks < KC / 32; ++ks)
        a[buf][h][ks] = *reinterpret_cast<const bf16x8*>(Ab + int64_t(16 * h) * nbp + min(k0 + ks * 32, nbp - 32));
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
      const int q = threadIdx.x + u * kGemmT;
      const int half = q / (LP * SEGS), rem = q - half * (LP * SEGS);
      const int j = rem / SEGS, sg = rem - j * SEGS;
      v[buf][u] = *reinterpret_cast<const bf16x8*>(STb + half * lo_off + int64_t(j) * nbp + min(k0 + sg * 8, nbp - 8));
    }
  };
  auto step = [&](int k0, auto bufc) {
    constexpr int buf = decltype(bufc)::value;
    const int nsteps = min(KC, nbp - k0) / 32;   // <= 0 past the end
    __syncthreads();  // the previous chunk's MFMAs are done with sst
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
      const int q = threadIdx.x + u * kGemmT;
      const int half = q / (LP * SEGS), rem = q - half * (LP * SEGS);
      const int j = rem / SEGS, sg = rem - j * SEGS;
      *reinterpret_cast<bf16x8*>(&sst[(half * LP + j) * KP + sg * 8]) = v[buf][u];
    }
    bf16x8 ac[2][KC / 32];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int ks = 0; ks < KC / 32; ++ks) ac[h][ks] = a[buf][h][ks];
    __syncthreads();
    fetch(k0 + 2 * KC, bufc);   // past the end: clamped, unused
#pragma unroll
    for (int ks = 0; ks < KC / 32; ++ks) {
      if (live && ks < nsteps) {
#pragma unroll
        for (int n = 0; n < NT; ++n) {
          const uint16_t* sp = &sst[(n * 16 + li) * KP + ks * 32 + kq * 8];
          const bf16x8 bhi = *reinterpret_cast<const bf16x8*>(sp);
          const bf16x8 blo = *reinterpret_cast<const bf16x8*>(sp + LP * KP);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            acc[h][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ac[h][ks], bhi, acc[h][n], 0, 0, 0);
            acc[h][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ac[h][ks], blo, acc[h][n], 0, 0, 0);
          }
        }
      }
    }
  };
  using B0 = std::integral_constant<int, 0>;
  using B1 = std::integral_constant<int, 1>;
  // chunks in pairs, every load unconditional, so the compiler counts the
  // loads in flight exactly and waits only for the chunk it stores (a chunk
  // past the end does no MFMA step)
  fetch(0, B0{});
  fetch(KC, B1{});
  for (int k0 = 0; k0 < nbp; k0 += 2 * KC) {
    step(k0, B0{});
    step(k0 + KC, B1{});
  }
  if (!live) return;
  float* Yb = Y + bm.yoff[b];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int n = 0; n < NT; ++n)
#pragma unroll
      for (int i = 0; i < 4; ++i) Yb[int64_t(r0 + 16 * h + kq * 4 + i) * LP + n * 16 + li] = acc[h][n][i];
}

// FP64 reference-precision variant: Y_b = A_bb S_b, plain FMA, one thread per
// (row, 4 columns) of a 64-row tile.
__global__ __launch_bounds__(kBlock) void k_gemm_f64(BlockMeta bm, const double* __restrict__ A,
                                                     const double* __restrict__ ST, double* __restrict__ Y) {
  const int b = bm.item_b[bm.i0 + blockIdx.x], t = bm.item_t[bm.i0 + blockIdx.x];
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

// G_b = Y_b' Y_b over the first l columns (FP64 accumulation) in two steps:
// every 64-row tile of a block writes its partial upper triangle (pair
// p <-> (i, j), i <= j, row-major over the triangle), then the kernel that
// consumes G_b (Cholesky or Jacobi, one workgroup per block) sums its tiles'
// partials in tile order (deterministic).

// LDS[r][c] (row stride lds_ld) <- src[r][c] (row stride src_ld) for r < rows,
// c < cols, as one flat loop so that several global loads are in flight.
template <class TS>
__device__ __forceinline__ void stage_rows(double* lds, int lds_ld, const TS* __restrict__ src, int64_t src_ld,
                                           int rows, int cols) {
  const int total = rows * cols;
#pragma unroll 4
  for (int q = threadIdx.x; q < total; q += kBlock) {
    const int r = q / cols, c = q - r * cols;
    lds[r * lds_ld + c] = double(src[int64_t(r) * src_ld + c]);
  }
}

// t -> (i, m) with m <= i, row-major over a lower triangle.
__device__ __forceinline__ void tri_of(int t, int& i, int& m) {
  int r = int((sqrtf(8.0f * float(t) + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  i = r;
  m = t - r * (r + 1) / 2;
}

// dst[r * LD + c] = src[r * LP + c] for the rows x LP row-major block src
// (16-byte aligned, rows <= ROWS), as TD, columns >= lmax and rows >= rows
// as zero: every thread issues all its 16-byte loads before its first LDS
// store, so a tile costs one round trip to memory rather than one per
// element.  NT threads.
template <int ROWS, int LP, int LD, int NT, class TS, class TD>
__device__ __forceinline__ void stage_block(TD* __restrict__ dst, const TS* __restrict__ src, int lmax,
                                            int rows = ROWS) {
  constexpr int PER = 16 / sizeof(TS);            // elements per 16-byte load
  constexpr int NV = ROWS * LP / PER;
  constexpr int IT = (NV + NT - 1) / NT;
  static_assert(LP % PER == 0, "rows of whole 16-byte vectors");
  const int nv = rows * LP / PER;
  uint4 buf[IT];
#pragma unroll
  for (int u = 0; u < IT; ++u) {
    const int q = threadIdx.x + u * NT;
    if (q < nv) buf[u] = reinterpret_cast<const uint4*>(src)[q];
  }
#pragma unroll
  for (int u = 0; u < IT; ++u) {
    const int q = threadIdx.x + u * NT;
    if (q < NV) {
      const int e = q * PER, r = e / LP, c = e - r * LP;
      const TS* v = reinterpret_cast<const TS*>(&buf[u]);
#pragma unroll
      for (int x = 0; x < PER; ++x) dst[r * LD + c + x] = (q < nv && c + x < lmax) ? TD(v[x]) : TD(0);
    }
  }
}

typedef double doublex4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64 on one wave: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; its four outputs are C[l / 16 + 4 i][l % 16].
__device__ __forceinline__ doublex4 mfma_f64(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// One 128-row item of Y (two 64-row tiles, or a block's last one): the
// upper 16 x 16 blocks (I <= J) of its Gram matrix Y' Y on FP64 MFMA (the
// FP32 entries are exact in FP64), three blocks per wave at a time over 8
// waves, written as the item's packed upper-triangle partial.  Block (I, J)
// needs A[m][k] = Y[k][16I + m] and B[k][n] = Y[k][16J + n]: both are row k
// of the staged tile.
constexpr int kGramT = 512;
template <class TY, int LP>
__global__ __launch_bounds__(kGramT) void k_gram_tiles(BlockMeta bm, const TY* __restrict__ Y,
                                                       double* __restrict__ part) {
  constexpr int NT = LP / 16, NB = NT * (NT + 1) / 2, LDT = LP + 1, NW = kGramT / kWave;
  __shared__ TY tile[128 * LDT];
  const int b = bm.pair_b[bm.p0 + blockIdx.x], t = bm.pair_t[bm.p0 + blockIdx.x];
  const int l = bm.l;
  const int npairs = l * (l + 1) / 2;
  const int rows = min(128, bm.nbp[b] - t * 64);
  // columns past l read as zero; rows past the block are zero in Y (zero
  // rows of the padded A_bb)
  stage_block<128, LP, LDT, kGramT>(tile, Y + bm.yoff[b] + int64_t(t) * 64 * LP, l, rows);
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int lm = lane % 16, lk = lane / 16;
  double* out = part + int64_t(bm.p0 + blockIdx.x) * npairs;
  for (int q0 = wave; q0 < NB; q0 += 3 * NW) {
    int bi[3], bj[3];
    doublex4 acc[3];
    const int nu = min(3, (NB - 1 - q0) / NW + 1);   // this wave's blocks in the round (uniform)
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int q = min(q0 + NW * u, NB - 1);
      tri_of(q, bj[u], bi[u]);   // bi <= bj
      acc[u] = doublex4{0.0, 0.0, 0.0, 0.0};
    }
    for (int k0 = 0; k0 < rows; k0 += 4) {
      const TY* row = tile + (k0 + lk) * LDT + lm;
#pragma unroll
      for (int u = 0; u < 3; ++u)
        if (u < nu) acc[u] = mfma_f64(double(row[16 * bi[u]]), double(row[16 * bj[u]]), acc[u]);
    }
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      if (q0 + NW * u >= NB) break;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * bi[u] + lk + 4 * v, j = 16 * bj[u] + lm;
        if (i <= j && j < l) out[i * l - i * (i - 1) / 2 + (j - i)] = acc[u][v];
      }
    }
  }
}

// Threads of the dense per-block kernels (Jacobi, eigensolver): one
// workgroup per diagonal block, 16 waves.
constexpr int kDense = 1024;

// Pair index p of the packed upper triangle (row-major, row m holds
// columns m .. l-1) -> (m, j): m is the largest row with
// m l - m(m-1)/2 <= p, from the quadratic's root, then corrected.
__device__ __forceinline__ void pair_rc(int p, int l, int& m, int& j) {
  const float bq = float(2 * l + 1);
  int r = int((bq - sqrtf(bq * bq - 8.0f * float(p))) * 0.5f);
  r = max(0, min(r, l - 1));
  while (r > 0 && r * l - r * (r - 1) / 2 > p) --r;
  while (r + 1 < l && (r + 1) * l - (r + 1) * r / 2 <= p) ++r;
  m = r;
  j = r + (p - (r * l - r * (r - 1) / 2));
}

// G_b = the sum of the block's tile partials in tile order (deterministic),
// written over the block's first partial; one thread per (pair, block)
// across the chip, so the dense per-block kernels read one packed triangle.
__global__ __launch_bounds__(256) void k_gram_reduce(BlockMeta bm, const int32_t* __restrict__ item0,
                                                     double* __restrict__ part) {
  const int l = bm.l, npairs = l * (l + 1) / 2;
  const int p = blockIdx.x * 256 + threadIdx.x, b = bm.b0 + blockIdx.y;
  if (p >= npairs) return;
  const int i0 = item0[b], i1 = item0[b + 1];
  double sacc = 0.0;
#pragma unroll 8
  for (int it = i0; it < i1; ++it) sacc += part[int64_t(it) * npairs + p];
  part[int64_t(i0) * npairs + p] = sacc;
}

// A (l x l in LDS, row-major, leading dimension ld) <- G_b, reduced by
// k_gram_reduce, mirrored.  NT threads.  fill() runs while the loads are in
// flight (it must not write the l x l corner of A).
struct NoFill {
  __device__ void operator()() const {}
};
template <int NT, class TA, class Fill = NoFill>
__device__ __forceinline__ void stage_gram(const BlockMeta& bm, const int32_t* __restrict__ item0,
                                           const double* __restrict__ part, int b, TA* A, int ld = -1,
                                           Fill fill = {}) {
  const int l = bm.l, npairs = l * (l + 1) / 2;
  if (ld < 0) ld = l;
  const double* Gb = part + int64_t(item0[b]) * npairs;
  // every round's load issued before the first store: one memory round trip
  constexpr int R = (kMaxLP * (kMaxLP + 1) / 2 + NT - 1) / NT;
  double g[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int p = threadIdx.x + u * NT;
    g[u] = p < npairs ? Gb[p] : 0.0;
  }
  fill();
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int p = threadIdx.x + u * NT;
    if (p < npairs) {
      int m, j;
      pair_rc(p, l, m, j);
      A[m * ld + j] = TA(g[u]);
      A[j * ld + m] = TA(g[u]);
    }
  }
}

// 16 x 16 block products on LDS by one wave: lane (r, c4) = (lane / 4,
// lane % 4) accumulates C[r][4 c4 + t], t < 4, of
// sum_k A[r][k] * (TB ? B[4 c4 + t][k] : B[k][4 c4 + t]).
template <bool TB>
__device__ __forceinline__ void blk_mm(double (&acc)[4], const double* __restrict__ Ab,
                                       const double* __restrict__ Bb, int ld, int r, int c0) {
#pragma unroll
  for (int kc = 0; kc < 16; kc += 4) {
    double av[4], bv[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) av[u] = Ab[r * ld + kc + u];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u) bv[t][u] = TB ? Bb[(c0 + t) * ld + kc + u] : Bb[(kc + u) * ld + c0 + t];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[t] += av[u] * bv[t][u];
  }
}

// L^-1 of the Cholesky factor of G_b = Y_b' Y_b (summed from the Gram tile
// partials), written to Li (LP x LP, lower, zero padded).  G_b is padded to
// N = 16 NX = LP with the identity and factored by 16 x 16 blocks
// (right-looking, Golub & Van Loan, alg. 4.2.2 by blocks), 512 threads:
//   for each block column k: one wave factors A_kk = L_kk L_kk' and forms
//   X_kk = L_kk^-1 in registers (an elimination on [A_kk | I] with unscaled
//   pivots, one row per lane, then L[r][c] = A[r][c] / sqrt(piv_c),
//   L^-1[r][c] = B[r][c] / sqrt(piv_r));
//   one wave per block row below forms L_ik = A_ik L_kk^-T, and one wave
//   per block left of the diagonal finishes X_kj = -X_kk W_kj; then the
//   lower block pairs are updated, A_ij -= L_ik L_jk', and the blocks X_ij
//   (i > k >= j) accumulate W_ij += L_ik X_kj, so that
//   X_ij = -L_ii^-1 sum_{k=j}^{i-1} L_ik X_kj (the blocks of L^-1) are done
//   with the factorisation.  One block of lookahead: wave 0 updates
//   A_{k+1,k+1} first and factors it (the next diagonal step) while the
//   other waves do the remaining updates.  Two barriers per block column.
// A non-positive or non-finite pivot triggers one retry with the shift
// 11 (n l + l (l+1)) u trace(G) (shifted CholQR, Fukaya et al. 2020); a
// second failure sets fail[b].
constexpr int kCholT = 512;   // 8 waves: 256 VGPRs each, so the diagonal step never spills
template <int NX>
__global__ __launch_bounds__(kCholT) void k_chol_inv(BlockMeta bm, const int32_t* __restrict__ item0,
                                                     const double* __restrict__ part, double* __restrict__ Li,
                                                     int32_t* __restrict__ fail) {
  constexpr int N = 16 * NX;
  constexpr int LD = N + 1;        // odd row stride: the 16 rows of a block fall in distinct banks
  extern __shared__ double sm[];
  double* const A = sm;            // N x N (stride LD): G, then L in the lower blocks
  double* const X = sm + N * LD;   // N x N (stride LD): L^-1 in the lower blocks
  __shared__ double s_tr, s_rs[16];
  __shared__ int s_bad;
  const int b = bm.b0 + blockIdx.x, tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const int r = lane >> 2, c0 = (lane & 3) * 4;
  const int l = bm.l, LP = bm.LP;
  const int n = bm.off[b + 1] - bm.off[b];
  // the diagonal step of block column kb, by wave 0: one row per lane (rows
  // r = lane % 16; the four copies of a row, one per row of 16 lanes,
  // compute alike); the trailing block stays symmetric, so column j is row
  // j, read from lane j of the lane's own row of 16; likewise row j of B.  No early exit, so the steps unroll and the rows stay in
  // registers; a failed pivot makes the result unused.  Column j of L
  // leaves unscaled: L[r][j] = a_j / sqrt(piv_j) once all pivots are known.
  auto diag = [&](int kb) {
    double* const Akk = A + kb * 16 * LD + kb * 16;
    const int rr = lane & 15;
    double a[16], x[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      a[c] = Akk[rr * LD + c];
      x[c] = rr == c ? 1.0 : 0.0;
    }
    double pr = 1.0;   // the lane's own row's pivot
    bool ok = true;
    static_for<0, 16>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      const double piv = row_bcast_d<j>(a[j]);
      ok = ok && piv > 0.0 && isfinite(piv);
      if (rr == j) pr = piv;
      // 1/piv: hardware reciprocal and two Newton steps
      double inv = __builtin_amdgcn_rcp(piv);
      inv = fma(inv, fma(-piv, inv, 1.0), inv);
      inv = fma(inv, fma(-piv, inv, 1.0), inv);
      if (lane < 16 && j <= rr) Akk[rr * LD + j] = a[j];
      const double cr = rr > j ? a[j] * inv : 0.0;
#pragma unroll
      for (int c = j + 1; c < 16; ++c) a[c] = fma(-cr, row_bcast_d<j>(a[c]), a[c]);
#pragma unroll
      for (int c = 0; c <= j; ++c) x[c] = fma(-cr, row_bcast_d<j>(x[c]), x[c]);
    });
    const double rs_r = 1.0 / sqrt(pr);
    if (!ok) {
      if (lane == 0) s_bad = 1;
    } else if (lane < 16) {
      double* const Xkk = X + kb * 16 * LD + kb * 16;
      s_rs[rr] = rs_r;
#pragma unroll
      for (int c = 0; c < 16; ++c) Xkk[rr * LD + c] = x[c] * rs_r;
      wave_sync();
#pragma unroll
      for (int c = 0; c < 16; ++c) Akk[rr * LD + c] = c <= rr ? Akk[rr * LD + c] * s_rs[c] : 0.0;
    }
  };
  for (int attempt = 0;; ++attempt) {
    // G, the identity on the padding; X (the W sums) zero
    stage_gram<kCholT>(bm, item0, part, b, A, LD, [&]() {
      for (int q = tid; q < N * N; q += kCholT) {
        const int i = q / N, j = q % N;
        if (i >= l || j >= l) A[i * LD + j] = i == j ? 1.0 : 0.0;
        X[i * LD + j] = 0.0;
      }
    });
    if (tid == 0) s_bad = 0;
    __syncthreads();
    if (attempt > 0) {
      // the retry's shift on the diagonal of G
      if (tid < kWave) {
        double t = 0.0;
        for (int i = tid; i < l; i += kWave) t += A[i * LD + i];
        for (int o2 = 32; o2 >= 1; o2 >>= 1) t += __shfl_xor(t, o2, kWave);
        if (tid == 0) s_tr = t;
      }
      __syncthreads();
      const double shift = 11.0 * (double(n) * l + double(l) * (l + 1)) * 1.1102230246251565e-16 * s_tr;
      if (tid < l) A[tid * LD + tid] += shift;
      __syncthreads();
    }
    // kb = -1 only runs the first diagonal step (one call site of diag)
    for (int kb = -1; kb < NX; ++kb) {
      const int nr = NX - kb - 1;
      if (kb < 0) {
        if (wave == 0) diag(0);
        __syncthreads();
        continue;
      }
      if (s_bad) break;   // uniform: the diagonal step of kb ran before the last barrier
      const double* const Xkk = X + kb * 16 * LD + kb * 16;
      if (wave < nr) {
        // panel: L_ik = A_ik L_kk^-T, one wave per block row below
        const int ib = kb + 1 + wave;
        double* const Aik = A + ib * 16 * LD + kb * 16;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        blk_mm<true>(acc, Aik, Xkk, LD, r, c0);
#pragma unroll
        for (int t = 0; t < 4; ++t) Aik[r * LD + c0 + t] = acc[t];
      } else if (wave < nr + kb) {
        // X_kj = -X_kk W_kj, one wave per block left of the diagonal
        double* const Xkj = X + kb * 16 * LD + (wave - nr) * 16;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        blk_mm<false>(acc, Xkk, Xkj, LD, r, c0);
#pragma unroll
        for (int t = 0; t < 4; ++t) Xkj[r * LD + c0 + t] = -acc[t];
      }
      __syncthreads();
      // trailing update of the lower blocks (one wave per block pair), and
      // W_ij += L_ik X_kj for the blocks of L^-1 below row k.  Wave 0 takes
      // the next diagonal block (pair 0) and goes straight on to its
      // diagonal step while the other waves finish the rest: no other
      // update reads or writes that block or X_{k+1,k+1}.
      const int npair = nr * (nr + 1) / 2, nw = nr * (kb + 1);
      auto update = [&](int pw) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (pw < npair) {
          int ii, jj;
          tri_of(pw, ii, jj);
          const int ib = kb + 1 + ii, jb = kb + 1 + jj;
          double* const Aij = A + ib * 16 * LD + jb * 16;
          blk_mm<true>(acc, A + ib * 16 * LD + kb * 16, A + jb * 16 * LD + kb * 16, LD, r, c0);
#pragma unroll
          for (int t = 0; t < 4; ++t) Aij[r * LD + c0 + t] -= acc[t];
        } else {
          const int q = pw - npair, ib = kb + 1 + q / (kb + 1), jb = q % (kb + 1);
          double* const Wij = X + ib * 16 * LD + jb * 16;
          blk_mm<false>(acc, A + ib * 16 * LD + kb * 16, X + kb * 16 * LD + jb * 16, LD, r, c0);
#pragma unroll
          for (int t = 0; t < 4; ++t) Wij[r * LD + c0 + t] += acc[t];
        }
      };
      if (nr > 0) {
        if (wave == 0) {
          update(0);
          wave_sync();
          diag(kb + 1);
        } else {
          for (int pw = wave; pw < npair + nw; pw += kCholT / kWave - 1) update(pw);
        }
      }
      __syncthreads();
    }
    if (!s_bad) break;
    if (attempt == 1) {
      if (tid == 0) fail[b] = 1;
      return;
    }
    __syncthreads();
  }
  double* Lb = Li + int64_t(b) * LP * LP;
  for (int q = tid; q < LP * LP; q += kCholT) {
    const int i = q / LP, c = q % LP;
    Lb[q] = (i < l && c <= i) ? X[i * LD + c] : 0.0;
  }
}

// Li <- identity on each block's l x l corner (zero elsewhere in LP x LP):
// k_apply_rinv with it lays Y out as the next product's operand unchanged
// (the power scheme of eq. 10, which has no orthonormalisation between
// products).
__global__ __launch_bounds__(256) void k_identity_factor(int64_t n, int LP, int l, double* __restrict__ Li) {
  for (int64_t q = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; q < n; q += int64_t(gridDim.x) * blockDim.x) {
    const int r = int(q % (int64_t(LP) * LP));
    const int i = r / LP, j = r - i * LP;
    Li[q] = (i == j && i < l) ? 1.0 : 0.0;
  }
}

// S = Y L^-T on a 128-row item: S[r][j] = sum_{i<=j} Y[r][i] Linv[j][i]
// (j < l), zero for j >= l and rows >= n_b (zero rows of Y, zero rows of
// Linv), on FP64 MFMA: wave w computes the 16 rows 16w.. for all column
// blocks J, skipping the k-steps above Linv's triangle; A[m][k] =
// Y[16w + m][k], B[k][n] = Linv[16J + n][k], Linv kept as its packed lower
// triangle.  Writes S (row-major) and, through LDS, ST (transposed, the next
// GEMM operand: BF16 hi/lo pair in the BF16 mode).
constexpr int kApplyT = 512;
template <class TY, class TST, int LP>
__global__ __launch_bounds__(kApplyT) void k_apply_rinv(BlockMeta bm, const TY* __restrict__ Y,
                                                        const double* __restrict__ Li, TY* __restrict__ S,
                                                        TST* __restrict__ ST, int64_t lo_off) {
  constexpr int NT = LP / 16, LD = LP + 1, NPK = LP * (LP + 1) / 2;
  __shared__ double Lp[NPK];       // Linv[r][c], c <= r, at r(r+1)/2 + c
  __shared__ TY Yt[128 * LD];      // the Y item, then the S item
  const int b = bm.pair_b[bm.p0 + blockIdx.x], t = bm.pair_t[bm.p0 + blockIdx.x];
  const int nbp = bm.nbp[b];
  const int rows = min(128, nbp - t * 64);
  {
    const double* Lb = Li + int64_t(b) * LP * LP;
    constexpr int IT = (NPK + kApplyT - 1) / kApplyT;
    double v[IT];
#pragma unroll
    for (int u = 0; u < IT; ++u) {
      const int q = threadIdx.x + u * kApplyT;
      int r = 0, c = 0;
      if (q < NPK) tri_of(q, r, c);
      v[u] = q < NPK ? Lb[r * LP + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < IT; ++u) {
      const int q = threadIdx.x + u * kApplyT;
      if (q < NPK) Lp[q] = v[u];
    }
  }
  stage_block<128, LP, LD, kApplyT>(Yt, Y + bm.yoff[b] + int64_t(t) * 64 * LP, LP, rows);
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int lm = lane % 16, lk = lane / 16;
  const bool live = 16 * wave < rows;
  doublex4 acc[NT];
#pragma unroll
  for (int J = 0; J < NT; ++J) acc[J] = doublex4{0.0, 0.0, 0.0, 0.0};
  if (live) {
#pragma unroll 4
    for (int k0 = 0; k0 < LP; k0 += 4) {
      const double a = double(Yt[(16 * wave + lm) * LD + k0 + lk]);
      const int c = k0 + lk;
#pragma unroll
      for (int J = 0; J < NT; ++J) {
        if (k0 <= 16 * J + 15) {
          const int r = 16 * J + lm;
          acc[J] = mfma_f64(a, c <= r ? Lp[r * (r + 1) / 2 + c] : 0.0, acc[J]);
        }
      }
    }
  }
  TY* Sb = S + bm.yoff[b] + int64_t(t) * 64 * LP;
  __syncthreads();   // every wave is done with the Y item
  if (live) {
#pragma unroll
    for (int J = 0; J < NT; ++J)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * wave + lk + 4 * v, j = 16 * J + lm;
        const TY sv = TY(acc[J][v]);
        Sb[int64_t(r) * LP + j] = sv;
        Yt[r * LD + j] = sv;
      }
  }
  __syncthreads();
  TST* STb = ST + bm.yoff[b];
  for (int q = threadIdx.x; q < LP * 128; q += kApplyT) {
    const int j = q / 128, r = q % 128;
    if (r >= rows) continue;
    const int64_t at = int64_t(j) * nbp + t * 64 + r;
    if constexpr (sizeof(TST) == 2) {
      // hi + lo BF16 pair (the lo half lives lo_off elements further on)
      const float f = float(Yt[r * LD + j]);
      const uint16_t hi = f32_to_bf16_rne(f);
      STb[at] = hi;
      STb[lo_off + at] = f32_to_bf16_rne(f - bf16_to_f32(hi));
    } else {
      STb[at] = Yt[r * LD + j];
    }
  }
}

// --------------------------------------------------------------- Jacobi --

// Eigen-decomposition of the symmetric l x l matrix G_b (= B B', summed from
// the Gram tile partials) by parallel cyclic Jacobi: round-robin pairing
// (circle method) gives l/2 disjoint index pairs per round, l-1 rounds per
// sweep; each pair's rotation is the one of Golub & Van Loan, sym.schur2.
// With J the product of a round's disjoint rotations, J'AJ restricted to the
// pair blocks (a, b) is J_a' A_ab J_b, so a round is one pass over independent
// 2 x 2 blocks (upper blocks a <= b, mirrored), plus V <- V J on the same
// blocks of V.  Every wave computes the round's rotations itself (lane a
// for pair a) and hands them to its threads' blocks by lane shuffles, so a
// round is a single barrier when A is double-buffered.  Writes the k largest
// eigenvalues' square roots (singular values of B, decreasing) and the
// matching eigenvectors (columns of Ut, l x k).
// NT threads; kJT = 2 x 2 blocks per thread and round (at 512 threads, 5
// covers l <= 80 and 7 covers l <= 96).
// TJ = arithmetic of the sweeps: FP64, or FP32 where the matrix comes from a
// BF16 sketch (its entries carry errors far above FP32 rounding); the sweeps
// stop when the off-diagonal Frobenius norm is below 1e-13 (FP64) or 1e-4
// (FP32: eigenvalue errors of order 1e-8 relative, eigenvector errors of
// order 1e-4 over the relative gap, both below the BF16 sketch's 4e-3) of
// the diagonal's.
template <class TJ>
struct JacPair {
  TJ c, s;     // the pair's rotation this round
  int p, q;    // p | (p l) << 8 and q | (q l) << 8: index and row offset
};
template <int NT, int kJT, class TJ, bool DB>
__global__ __launch_bounds__(NT) void k_jacobi(BlockMeta bm, const int32_t* __restrict__ item0,
                                               const double* __restrict__ part, double* __restrict__ sig,
                                               double* __restrict__ Ut, int max_sweeps) {
  extern __shared__ double sm[];
  const int b = bm.b0 + blockIdx.x, tid = threadIdx.x;
  const int l = bm.l, LP = bm.LP, kk = bm.kk;
  const int ne = l + (l & 1);  // even count (a dummy index l pairs with the odd one out)
  const int half = ne / 2;
  constexpr double kStop = sizeof(TJ) == 8 ? 1e-26 : 1e-8;   // squared relative off-diagonal norm
  constexpr TJ kTiny = sizeof(TJ) == 8 ? TJ(1e-300) : TJ(1e-30);
  constexpr int NW = NT / kWave;
  // LDS: A (twice when double-buffered, DB: a round reads one copy and
  // writes the other, so one barrier per round; otherwise in place with a
  // barrier between reading the rotations' entries and writing the blocks),
  // V, the ranks, and one pair table per wave.  Offsets from one base keep
  // every access an LDS instruction.
  TJ* const M = reinterpret_cast<TJ*>(sm);
  const int ll = l * l;
  const int oV = (DB ? 2 : 1) * ll;
  int* rank = reinterpret_cast<int*>(M + oV + ll);                       // [l]
  JacPair<TJ>* tab = reinterpret_cast<JacPair<TJ>*>(sm + (((DB ? 3 : 2) * ll * sizeof(TJ) + 4 * l + 15) / 16) * 2);
  __shared__ double s_off[NW], s_dg[NW];
  stage_gram<NT>(bm, item0, part, b, M);
  for (int q = tid; q < ll; q += NT) M[oV + q] = (q / l == q % l) ? TJ(1) : TJ(0);
  __syncthreads();
  // this thread's tasks t = tid + u * NT, in wave-uniform ranges: the
  // diagonal A blocks (pair a), the blocks above them (pairs a < b, stored
  // and mirrored), and V <- V J on row pair (2r, 2r+1) and column pair b
  const int nOff = half * (half - 1) / 2, nVr = (l + 1) / 2;
  const int n1 = half, n2 = n1 + nOff, n3 = n2 + nVr * half;
  int tk_k[kJT], tk_a[kJT], tk_b[kJT];   // kind 0 none, 1 diagonal, 2 above, 3 V
#pragma unroll
  for (int u = 0; u < kJT; ++u) {
    const int t = tid + u * NT;
    tk_k[u] = 0;
    tk_a[u] = tk_b[u] = 0;
    if (t < n1) {
      tk_k[u] = 1;
      tk_a[u] = tk_b[u] = t;
    } else if (t < n2) {
      int bb, aa;
      tri_of(t - n1, bb, aa);
      tk_k[u] = 2;
      tk_a[u] = aa;
      tk_b[u] = bb + 1;
    } else if (t < n3) {
      tk_k[u] = 3;
      tk_a[u] = (t - n2) / half;   // row pair
      tk_b[u] = (t - n2) - tk_a[u] * half;
    }
  }
  const int lane = tid % kWave;
  JacPair<TJ>* wtab = tab + (tid / kWave) * half;
  int oc = 0;   // offset of the current A
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // convergence: off-diagonal mass against the diagonal (fixed-order sums)
    double off = 0.0, dg = 0.0;
    for (int q = tid; q < ll; q += NT) {
      const double v = double(M[oc + q]) * double(M[oc + q]);
      if (q / l != q % l) off += v; else dg += v;
    }
    for (int o2 = 32; o2 >= 1; o2 >>= 1) {
      off += __shfl_xor(off, o2, kWave);
      dg += __shfl_xor(dg, o2, kWave);
    }
    if (lane == 0) {
      s_off[tid / kWave] = off;
      s_dg[tid / kWave] = dg;
    }
    __syncthreads();
    double off_t = 0.0, dg_t = 0.0;
    for (int w = 0; w < NW; ++w) {
      off_t += s_off[w];
      dg_t += s_dg[w];
    }
    __syncthreads();
    // eigenvalue errors are then of order off^2/gap: far below the FP64
    // CholQR noise, or the BF16 sketch's
    if (off_t <= kStop * dg_t) break;
    for (int round = 0; round < ne - 1; ++round) {
      const int on = DB ? ll - oc : oc;   // offset the round writes A to
      // lane a of every wave computes pair a (circle method: slot 0 fixed,
      // the others rotate; pair a is the slots (a, ne-1-a), ordered p < q)
      // and its rotation into the wave's own table (the same values in
      // every wave; a wave's LDS accesses complete in order)
      if (lane < half) {
        auto at = [&](int slot) {
          if (slot == 0) return 0;
          int v = slot - 1 + round;
          if (v >= ne - 1) v -= ne - 1;
          return 1 + v;
        };
        const int x0 = at(lane), y0 = at(ne - 1 - lane);
        const int p = min(x0, y0), q = max(x0, y0);
        TJ rc = TJ(1), rs = TJ(0);
        if (q < l) {
          const TJ apq = M[oc + p * l + q];
          if (fabs(apq) > kTiny) {
            const TJ tau = (M[oc + q * l + q] - M[oc + p * l + p]) / (TJ(2) * apq);
            const TJ tt = (tau >= TJ(0) ? TJ(1) : TJ(-1)) / (fabs(tau) + sqrt(TJ(1) + tau * tau));
            rc = TJ(1) / sqrt(TJ(1) + tt * tt);
            rs = tt * rc;
          }
        }
        wtab[lane] = JacPair<TJ>{rc, rs, p | (p * l) << 8, q | (q * l) << 8};
      }
      if constexpr (DB) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      } else {
        __syncthreads();   // every rotation read before any block is written
      }
      // this thread's tasks, all loads before any store (the tasks are
      // disjoint; the compiler cannot see that)
      JacPair<TJ> ea[kJT], eb[kJT];
      TJ x[kJT][4];
#pragma unroll
      for (int u = 0; u < kJT; ++u) {
        const int k = tk_k[u];
        if (k == 0) continue;
        eb[u] = wtab[tk_b[u]];
        if (k == 1) {
          const int p = eb[u].p & 255, pl = eb[u].p >> 8, q = eb[u].q & 255, ql = eb[u].q >> 8;
          x[u][0] = M[oc + pl + p];
          if (q < l) {
            x[u][1] = M[oc + pl + q];
            x[u][3] = M[oc + ql + q];
          }
        } else if (k == 2) {
          ea[u] = wtab[tk_a[u]];
          const int pa = ea[u].p & 255, pal = ea[u].p >> 8, qa = ea[u].q & 255, qal = ea[u].q >> 8;
          const int pb = eb[u].p & 255, qb = eb[u].q & 255;
          x[u][0] = M[oc + pal + pb];
          x[u][1] = qb < l ? M[oc + pal + qb] : TJ(0);
          x[u][2] = qa < l ? M[oc + qal + pb] : TJ(0);
          x[u][3] = (qa < l && qb < l) ? M[oc + qal + qb] : TJ(0);
        } else {
          const int r0 = 2 * tk_a[u], pb = eb[u].p & 255, qb = eb[u].q & 255;
          const bool r1 = r0 + 1 < l, q1 = qb < l;
          x[u][0] = M[oV + r0 * l + pb];
          x[u][1] = q1 ? M[oV + r0 * l + qb] : TJ(0);
          x[u][2] = r1 ? M[oV + (r0 + 1) * l + pb] : TJ(0);
          x[u][3] = (r1 && q1) ? M[oV + (r0 + 1) * l + qb] : TJ(0);
        }
      }
#pragma unroll
      for (int u = 0; u < kJT; ++u) {
        const int k = tk_k[u];
        if (k == 0) continue;
        const TJ cb = eb[u].c, sb = eb[u].s;
        if (k == 1) {
          // the pair's own 2 x 2 block J' X J: diagonalised, kept exactly
          // symmetric
          const int p = eb[u].p & 255, pl = eb[u].p >> 8, q = eb[u].q & 255, ql = eb[u].q >> 8;
          if (q < l) {
            const TJ x00 = x[u][0], x01 = x[u][1], x11 = x[u][3];
            const TJ r00 = cb * x00 - sb * x01, r01 = cb * x01 - sb * x11;
            const TJ r10 = sb * x00 + cb * x01, r11 = sb * x01 + cb * x11;
            const TJ y00 = cb * r00 - sb * r01, y01 = sb * r00 + cb * r01;
            const TJ y11 = sb * r10 + cb * r11;
            M[on + pl + p] = y00;
            M[on + ql + q] = y11;
            M[on + pl + q] = y01;
            M[on + ql + p] = y01;
          } else {
            M[on + pl + p] = x[u][0];
          }
        } else if (k == 2) {
          // rows by J_a' (p' = c p - s q, q' = s p + c q), then columns by J_b
          const TJ ca = ea[u].c, sa = ea[u].s;
          const TJ r00 = ca * x[u][0] - sa * x[u][2], r01 = ca * x[u][1] - sa * x[u][3];
          const TJ r10 = sa * x[u][0] + ca * x[u][2], r11 = sa * x[u][1] + ca * x[u][3];
          const TJ y00 = cb * r00 - sb * r01, y01 = sb * r00 + cb * r01;
          const TJ y10 = cb * r10 - sb * r11, y11 = sb * r10 + cb * r11;
          const int pa = ea[u].p & 255, pal = ea[u].p >> 8, qa = ea[u].q & 255, qal = ea[u].q >> 8;
          const int pb = eb[u].p & 255, pbl = eb[u].p >> 8, qb = eb[u].q & 255, qbl = eb[u].q >> 8;
          const bool q0 = qa < l, q1 = qb < l;
          M[on + pal + pb] = y00;
          M[on + pbl + pa] = y00;
          if (q1) {
            M[on + pal + qb] = y01;
            M[on + qbl + pa] = y01;
          }
          if (q0) {
            M[on + qal + pb] = y10;
            M[on + pbl + qa] = y10;
          }
          if (q0 && q1) {
            M[on + qal + qb] = y11;
            M[on + qbl + qa] = y11;
          }
        } else {
          // V <- V J_b on two rows
          const int r0 = 2 * tk_a[u], pb = eb[u].p & 255, qb = eb[u].q & 255;
          const bool r1 = r0 + 1 < l, q1 = qb < l;
          M[oV + r0 * l + pb] = cb * x[u][0] - sb * x[u][1];
          if (q1) M[oV + r0 * l + qb] = sb * x[u][0] + cb * x[u][1];
          if (r1) {
            M[oV + (r0 + 1) * l + pb] = cb * x[u][2] - sb * x[u][3];
            if (q1) M[oV + (r0 + 1) * l + qb] = sb * x[u][2] + cb * x[u][3];
          }
        }
      }
      __syncthreads();
      oc = on;
    }
  }
  const TJ* A = M + oc;
  const TJ* V = M + oV;
  // rank by decreasing eigenvalue (ties by index): output the leading kk
  for (int i = tid; i < l; i += NT) {
    const double li = A[i * l + i];
    int r = 0;
    for (int j = 0; j < l; ++j) {
      const double lj = A[j * l + j];
      r += (lj > li) || (lj == li && j < i);
    }
    rank[i] = r;
    if (r < kk) sig[int64_t(b) * kk + r] = sqrt(fmax(li, 0.0));
  }
  __syncthreads();
  for (int q = tid; q < l * l; q += NT) {
    const int r = q / l, i = q - r * l;
    if (rank[i] < kk) Ut[int64_t(b) * LP * kk + int64_t(r) * kk + rank[i]] = double(V[q]);
  }
}

// ------------------------------------------- tridiagonal eigensolver --

// Top-kk eigenpairs of the symmetric l x l matrix G_b (= B B', summed from
// the Gram tile partials) in FP32, for a BF16 sketch, as four phases in one
// workgroup per block (1024 threads):
//  1. Householder tridiagonalisation Q' G Q = T (Golub & Van Loan, alg.
//     8.3.1): step k has p = tau A22 v (16 lanes per row), then
//     A22 -= v w' + w v' with w = p - (tau/2)(p'v) v.  Wave 0 updates the
//     first column of A22 alone and forms the next reflector from it while
//     the other waves update the rest, so a step is two barriers; v_k is
//     kept in column k of A.
//  2. The kk largest eigenvalues of T by multisection on Sturm counts
//     (Golub & Van Loan, sec. 8.4.1): a coarse pass counts at 1024 points
//     of the Gershgorin bracket, then 16 lanes per eigenvalue (8 when kk >
//     64) split its bracket into 17 (9) parts per pass, 5 (6) passes.
//  3. Eigenvectors of T by inverse iteration, one lane per eigenvalue
//     (Golub & Van Loan, sec. 8.2.2): Gaussian elimination with partial
//     pivoting of T - lam I once, two solves from a fixed start vector, then
//     Gram-Schmidt (classical, twice) against the earlier vectors of the
//     same cluster (eigenvalues closer than 1e-3 |T|, the threshold of
//     LAPACK's stein), one wave per vector.
//  4. Back-transformation U = Q Z: each eigenvector's column held by 16
//     lanes in registers through the l-2 reflectors (no barriers).
// Writes sqrt of the eigenvalues (singular values of B, decreasing) to sig
// and the eigenvectors to Ut (l x kk), as the Jacobi kernel does.
// cw = eigenvectors per inverse-iteration pass (64, or 32 where the
// factors of 64 would not fit in LDS).
constexpr int kEigT = 1024;
constexpr int kEigSolves = 2;
constexpr int kZ = kMaxLP / 16;   // entries of a column per lane of a 16-lane group

__device__ __forceinline__ float wave_sum_f(float x) { return wave_sum_dpp(x); }

// Reflector of x (two entries per lane of wave 0: x_lane, x_{lane+64};
// n entries): H x = beta e_1, H = I - t v v', v_0 = 1.  Writes v to vbuf
// and to column col of A from row r0, and tau, e at index k.
__device__ __forceinline__ void eig_reflector(float x0, float x1, int n, int k, int r0, int col, int l,
                                              float* __restrict__ A, float* __restrict__ vbuf,
                                              float* __restrict__ tau, float* __restrict__ ee) {
  const int lane = threadIdx.x % kWave;
  const float alpha = readlane_f(x0, 0);
  const float s2 = wave_sum_f((lane >= 1 && lane < n ? x0 * x0 : 0.f) + (lane + 64 < n ? x1 * x1 : 0.f));
  float t = 0.f, beta = alpha, scale = 0.f;
  if (s2 > 0.f) {
    const float nrm = sqrtf(alpha * alpha + s2);
    beta = alpha >= 0.f ? -nrm : nrm;
    t = (beta - alpha) / beta;
    scale = 1.f / (alpha - beta);
  }
  if (lane < n) {
    const float v = lane == 0 ? 1.f : x0 * scale;
    vbuf[lane] = v;
    A[(r0 + lane) * l + col] = v;
  }
  if (lane + 64 < n) {
    const float v = x1 * scale;
    vbuf[lane + 64] = v;
    A[(r0 + lane + 64) * l + col] = v;
  }
  if (lane == 0) {
    tau[k] = t;
    ee[k] = beta;
  }
}

__global__ __launch_bounds__(kEigT) void k_eig_tridiag(BlockMeta bm, const int32_t* __restrict__ item0,
                                                       const double* __restrict__ part, double* __restrict__ sig,
                                                       double* __restrict__ Ut, int cw) {
  extern __shared__ double sm[];
  const int b = bm.b0 + blockIdx.x, tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
  const int l = bm.l, LP = bm.LP, kk = bm.kk;
  float* const A = reinterpret_cast<float*>(sm);     // l x l, row-major
  float* const Z = A + l * l;                        // l x kk, Z[i * kk + j]
  float* const FA = Z + l * kk;                      // l x cw each: the factors of T - lam I:
  float* const FB = FA + l * cw;                     //   1 / pivot, first and second superdiagonal,
  float* const FC = FB + l * cw;                     //   multiplier, row swap (1) or not (0)
  float* const FM = FC + l * cw;
  float* const FS = FM + l * cw;
  __shared__ float vb[2][kMaxLP], pb[kMaxLP], ee[kMaxLP + 8], tau[kMaxLP], lam[kMaxLP];
  __shared__ __align__(16) float dd[kMaxLP + 8], e2s[kMaxLP + 8];
  __shared__ int s_cnt[kEigT];
  __shared__ int cst[kMaxLP];
  __shared__ float s_lo, s_hi, s_piv, s_nrm;
  stage_gram<kEigT>(bm, item0, part, b, A);
  __syncthreads();
  // 1. tridiagonalisation
  if (l >= 3) {
    if (wave == 0) {
      if (lane == 0) dd[0] = A[0];
      const float x0 = lane < l - 1 ? A[(1 + lane) * l] : 0.f;
      const float x1 = lane + 64 < l - 1 ? A[(65 + lane) * l] : 0.f;
      eig_reflector(x0, x1, l - 1, 0, 1, 0, l, A, vb[0], tau, ee);
    }
    __syncthreads();
  }
  for (int k = 0; k + 2 < l; ++k) {
    const int m = l - k - 1;   // order of A22 = A[k+1:, k+1:]
    const float* v = vb[k & 1];
    const float t = tau[k];
    float* const A22 = A + (k + 1) * l + (k + 1);
    if (t != 0.f) {   // uniform
      // p = t A22 v, 16 lanes per row
      const int g = tid >> 4, c16 = tid & 15;
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int i = g + 64 * r;
        if (i < m) {
          const float* row = A22 + i * l;
          float acc = 0.f;
#pragma unroll
          for (int u = 0; u < kZ; ++u) {
            const int j = c16 + 16 * u;
            if (j < m) acc += row[j] * v[j];
          }
          acc = row16_sum(acc);
          if (c16 == 0) pb[i] = t * acc;
        }
      }
    }
    __syncthreads();
    // K = t/2 p'v (every wave forms the same sum)
    float K = 0.f;
    if (t != 0.f) {
      float kp = 0.f;
      if (lane < m) kp += pb[lane] * v[lane];
      if (lane + 64 < m) kp += pb[lane + 64] * v[lane + 64];
      K = 0.5f * t * wave_sum_f(kp);
    }
    if (wave == 0) {
      // first column of A22 (rows 1..m-1 in the lanes, row 0 uniform), then
      // the next reflector from it, or the last entries of T
      const float w0 = t != 0.f ? pb[0] - K : 0.f;
      float x0 = 0.f, x1 = 0.f;
      if (lane + 1 < m) {
        const int i = lane + 1;
        const float vi = v[i], wi = t != 0.f ? pb[i] - K * vi : 0.f;
        x0 = A22[i * l] - (vi * w0 + wi);
      }
      if (lane + 65 < m) {
        const int i = lane + 65;
        const float vi = v[i], wi = t != 0.f ? pb[i] - K * vi : 0.f;
        x1 = A22[i * l] - (vi * w0 + wi);
      }
      if (lane == 0) dd[k + 1] = A22[0] - (w0 + w0);
      if (m >= 3) {
        eig_reflector(x0, x1, m - 1, k + 1, k + 2, k + 1, l, A, vb[(k + 1) & 1], tau, ee);
      } else if (lane == 0) {
        ee[k + 1] = x0;
      }
    } else if (t != 0.f) {
      // the rest of A22 (rows and columns >= 1; row 0 is not read again)
      const int u0 = tid - kWave, g = u0 >> 4, c16 = u0 & 15;
      constexpr int NG = (kEigT - kWave) / 16;
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int i = 1 + g + NG * r;
        if (i < m) {
          const float vi = v[i], wi = pb[i] - K * vi;
          float* row = A22 + i * l;
#pragma unroll
          for (int u = 0; u < kZ; ++u) {
            const int j = 1 + c16 + 16 * u;
            if (j < m) {
              const float vj = v[j], wj = pb[j] - K * vj;
              row[j] -= vi * wj + wi * vj;
            }
          }
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (l <= 2) {
      dd[0] = A[0];
      if (l == 2) ee[0] = A[l];
    }
    dd[l - 1] = A[(l - 1) * l + (l - 1)];
  }
  __syncthreads();
  // Gershgorin bracket, the Sturm pivot floor and |T| (one wave); e2s[i] =
  // e_{i-1}^2 lines up with dd[i]
  if (wave == 0) {
    float lo = 3.4e38f, hi = -3.4e38f, emax = 0.f, tn = 0.f;
    for (int i = lane; i < l; i += kWave) {
      const float r = (i > 0 ? fabsf(ee[i - 1]) : 0.f) + (i + 1 < l ? fabsf(ee[i]) : 0.f);
      lo = fminf(lo, dd[i] - r);
      hi = fmaxf(hi, dd[i] + r);
      tn = fmaxf(tn, fabsf(dd[i]) + r);
      const float e2 = i > 0 ? ee[i - 1] * ee[i - 1] : 0.f;
      e2s[i] = e2;
      emax = fmaxf(emax, e2);
    }
    lo = wave_reduce(lo, OpMin{});
    hi = wave_reduce(hi, OpMax{});
    emax = wave_reduce(emax, OpMax{});
    tn = wave_reduce(tn, OpMax{});
    if (lane == 0) {
      const float span = fmaxf(hi - lo, 1e-30f);
      s_lo = lo - 1e-6f * span;
      s_hi = hi + 1e-6f * span;
      s_piv = 1.1754944e-38f * fmaxf(1.f, emax);
      s_nrm = fmaxf(tn, 1e-30f);
    }
  }
  __syncthreads();
  // 2. multisection: the r-th largest eigenvalue lies where the count of
  // eigenvalues below x passes l - 1 - r.  A coarse pass counts at kEigT
  // points across the Gershgorin bracket (one per thread) and gives every
  // eigenvalue a bracket of one step; groups of g lanes then split it into
  // g + 1 parts per pass.
  const float piv = s_piv;
  // count of eigenvalues of T below x (Sturm sequence of the LDL' pivots
  // of T - x I); the next four entries are loaded while four are processed
  auto sturm = [&](float x) {
    float q = dd[0] - x;
    int c = q < 0.f;
    float4 D = *reinterpret_cast<const float4*>(dd), E = *reinterpret_cast<const float4*>(e2s);
    for (int i0 = 0; i0 < l; i0 += 4) {
      const float4 Dn = *reinterpret_cast<const float4*>(dd + i0 + 4);
      const float4 En = *reinterpret_cast<const float4*>(e2s + i0 + 4);
      const float dv[4] = {D.x, D.y, D.z, D.w}, ev[4] = {E.x, E.y, E.z, E.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u;
        if (i >= 1 && i < l) {
          if (fabsf(q) < piv) q = -piv;
          q = (dv[u] - x) - ev[u] * __builtin_amdgcn_rcpf(q);
          c += q < 0.f;
        }
      }
      D = Dn;
      E = En;
    }
    return c;
  };
  {
    const float lo0 = s_lo, span = s_hi - s_lo;
    s_cnt[tid] = sturm(lo0 + span * float(tid + 1) / float(kEigT + 1));
    __syncthreads();
    const int G = kk <= kEigT / 16 ? 16 : 8;
    const int g = tid / G, gl = tid % G;
    const int npass = G == 16 ? 5 : 6;   // 17^5, 9^6 > 2^17: with the coarse 2^10, past FP32 resolution
    for (int r = g; r < kk; r += kEigT / G) {
      const int target = l - 1 - r;
      // the last coarse point whose count is <= target (counts rise with x)
      int lo_i = -1, hi_i = kEigT;
      while (hi_i - lo_i > 1) {
        const int mid = (lo_i + hi_i) >> 1;
        if (s_cnt[mid] <= target) lo_i = mid;
        else hi_i = mid;
      }
      float lo = lo_i < 0 ? lo0 : lo0 + span * float(lo_i + 1) / float(kEigT + 1);
      float hi = hi_i >= kEigT ? s_hi : lo0 + span * float(hi_i + 1) / float(kEigT + 1);
      for (int it = 0; it < npass; ++it) {
        const float x = lo + (hi - lo) * float(gl + 1) / float(G + 1);
        const int c = sturm(x);
        // the group's flags (count <= target) are a prefix; its length picks
        // the sub-bracket, and every lane recomputes its ends the way the
        // lanes computed their points
        const uint64_t bal = __ballot(c <= target);
        const uint32_t mine = uint32_t(bal >> ((lane / G) * G)) & ((1u << G) - 1);
        const int qn = __builtin_ctz(~mine);
        const float xl = lo + (hi - lo) * float(qn) / float(G + 1);
        const float xh = lo + (hi - lo) * float(qn + 1) / float(G + 1);
        lo = qn > 0 ? xl : lo;
        hi = qn < G ? xh : hi;
      }
      if (gl == 0) lam[r] = 0.5f * (lo + hi);
    }
  }
  __syncthreads();
  // clusters: j continues the cluster of j-1 when their gap is below
  // 1e-3 |T|
  if (tid == 0) {
    const float ortol = 1e-3f * s_nrm;
    cst[0] = 0;
    for (int j = 1; j < kk; ++j) cst[j] = (lam[j - 1] - lam[j] < ortol) ? cst[j - 1] : j;
  }
  __syncthreads();
  int cmax = 1;
  for (int jj = 1; jj < kk; ++jj) cmax = max(cmax, jj - cst[jj] + 1);
  // 3. inverse iteration, cw eigenvalues per pass.  The per-lane loops run
  // along T, each step's LDS operands loaded one step ahead.
  const float eps3 = 1.1920929e-7f * s_nrm;   // pivot floor and separation of equal eigenvalues
  for (int j0 = 0; j0 < kk; j0 += cw) {
    const int jc = tid, j = j0 + jc;
    const bool mine = jc < cw && j < kk;
    if (mine) {
      float lj = lam[j];
      // equal eigenvalues get distinct shifts (LAPACK's stein does the same)
      if (j > cst[j]) lj = fminf(lj, lam[j - 1] - 10.f * eps3 * float(j - cst[j]));
      // Gaussian elimination with partial pivoting of T - lj I; the rows
      // kept in registers are the current pivot row (ca, cb)
      float ca = dd[0] - lj, cb = l > 1 ? ee[0] : 0.f;
      float cl = ee[0], dn = l > 1 ? dd[1] : 0.f, en = l > 2 ? ee[1] : 0.f;
      for (int i = 0; i + 1 < l; ++i) {
        const float na = dn - lj, nb = i + 2 < l ? en : 0.f, cli = cl;
        // next step's operands
        cl = ee[i + 1];
        dn = dd[i + 2];
        en = ee[i + 2];
        const bool sw = fabsf(ca) < fabsf(cli);
        const float pv = sw ? cli : (fabsf(ca) >= eps3 ? ca : (ca >= 0.f ? eps3 : -eps3));
        const float rp = __builtin_amdgcn_rcpf(pv);
        const float mlt = (sw ? ca : cli) * rp;
        FA[i * cw + jc] = rp;
        FB[i * cw + jc] = sw ? na : cb;
        FC[i * cw + jc] = sw ? nb : 0.f;
        FM[i * cw + jc] = mlt;
        FS[i * cw + jc] = sw ? 1.f : 0.f;
        const float nca = sw ? cb - mlt * na : na - mlt * cb;
        cb = sw ? -mlt * nb : nb;
        ca = nca;
      }
      if (fabsf(ca) < eps3) ca = ca >= 0.f ? eps3 : -eps3;
      FA[(l - 1) * cw + jc] = __builtin_amdgcn_rcpf(ca);
      // start vector: a fixed pseudo-random vector
      for (int i = 0; i < l; ++i) {
        uint32_t hsh = uint32_t(i) * 2654435761u ^ uint32_t(j + 1) * 2246822519u;
        hsh ^= hsh >> 15;
        hsh *= 2654435761u;
        hsh ^= hsh >> 13;
        Z[i * kk + j] = 1.f + 0.5f * (float(hsh & 0xffffu) / 65535.f - 0.5f);
      }
    }
    for (int it = 0; it < kEigSolves; ++it) {
      if (mine) {
        // row operations of the elimination on the right side, then back
        // substitution and the 2-norm
        float cur = Z[j];
        float nx = l > 1 ? Z[kk + j] : 0.f, mlt = FM[jc], swf = FS[jc];
        for (int i = 0; i + 1 < l; ++i) {
          const float nxi = nx, mi = mlt;
          const bool sw = swf != 0.f;
          if (i + 2 < l) {
            nx = Z[(i + 2) * kk + j];
            mlt = FM[(i + 1) * cw + jc];
            swf = FS[(i + 1) * cw + jc];
          }
          Z[i * kk + j] = sw ? nxi : cur;
          cur = sw ? cur - mi * nxi : nxi - mi * cur;
        }
        float z2 = cur * FA[(l - 1) * cw + jc], z1 = 0.f;
        Z[(l - 1) * kk + j] = z2;
        float nrm2 = z2 * z2;
        int i = l - 2;
        float zb = i >= 0 ? Z[i * kk + j] : 0.f, fb = i >= 0 ? FB[i * cw + jc] : 0.f;
        float fc = i >= 0 ? FC[i * cw + jc] : 0.f, fa = i >= 0 ? FA[i * cw + jc] : 0.f;
        for (; i >= 0; --i) {
          const float zbi = zb, fbi = fb, fci = fc, fai = fa;
          if (i >= 1) {
            zb = Z[(i - 1) * kk + j];
            fb = FB[(i - 1) * cw + jc];
            fc = FC[(i - 1) * cw + jc];
            fa = FA[(i - 1) * cw + jc];
          }
          const float zi = (zbi - fbi * z2 - fci * z1) * fai;
          Z[i * kk + j] = zi;
          nrm2 += zi * zi;
          z1 = z2;
          z2 = zi;
        }
        const float inv = 1.f / sqrtf(nrm2);
        for (int q = 0; q < l; ++q) Z[q * kk + j] *= inv;
      }
      // after the last solve: Gram-Schmidt in clusters, by position in the
      // cluster; one wave per vector (entries lane, lane + 64 in
      // registers), classical twice (the earlier members' projections from
      // one set of inner products, then once more), four inner products
      // reduced at a time.  The solves of nearly equal eigenvalues already
      // use separated shifts.
      for (int pos = 1; it + 1 == kEigSolves && pos < cmax; ++pos) {
        __syncthreads();
        for (int jv = j0 + wave; jv < min(kk, j0 + cw); jv += kEigT / kWave) {
          if (jv - cst[jv] != pos) continue;   // uniform in the wave
          float z0 = lane < l ? Z[lane * kk + jv] : 0.f;
          float z1 = lane + 64 < l ? Z[(lane + 64) * kk + jv] : 0.f;
          for (int rep = 0; rep < 2; ++rep) {
            float y0 = 0.f, y1 = 0.f;   // sum of the projections
            for (int c0 = cst[jv]; c0 < jv; c0 += 4) {
              float q0[4], q1[4], d[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const int c = c0 + u;
                q0[u] = (c < jv && lane < l) ? Z[lane * kk + c] : 0.f;
                q1[u] = (c < jv && lane + 64 < l) ? Z[(lane + 64) * kk + c] : 0.f;
                d[u] = z0 * q0[u] + z1 * q1[u];
              }
#pragma unroll
              for (int u = 0; u < 4; ++u) d[u] = wave_sum_dpp(d[u]);
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                y0 += d[u] * q0[u];
                y1 += d[u] * q1[u];
              }
            }
            z0 -= y0;
            z1 -= y1;
          }
          const float inv = 1.f / sqrtf(wave_sum_f(z0 * z0 + z1 * z1));
          if (lane < l) Z[lane * kk + jv] = z0 * inv;
          if (lane + 64 < l) Z[(lane + 64) * kk + jv] = z1 * inv;
        }
      }
      __syncthreads();
    }
  }
  // 4. back-transformation: column c of Z by the 16 lanes of group c,
  // rows sl + 16u in registers; the next reflector's entries are loaded
  // while the current one is applied
  {
    const int sl = tid & 15;
    for (int c = tid >> 4; c < kk; c += kEigT / 16) {
      float z[kZ], vn[kZ];
#pragma unroll
      for (int u = 0; u < kZ; ++u) {
        const int i = sl + 16 * u;
        z[u] = i < l ? Z[i * kk + c] : 0.f;
      }
      float tn = 0.f;
      if (l >= 3) {
        const int k = l - 3;
        tn = tau[k];
#pragma unroll
        for (int u = 0; u < kZ; ++u) {
          const int i = sl + 16 * u;
          vn[u] = (i > k && i < l) ? A[i * l + k] : 0.f;
        }
      }
      for (int k = l - 3; k >= 0; --k) {
        float v[kZ];
#pragma unroll
        for (int u = 0; u < kZ; ++u) v[u] = vn[u];
        const float t = tn;
        if (k > 0) {
          tn = tau[k - 1];
#pragma unroll
          for (int u = 0; u < kZ; ++u) {
            const int i = sl + 16 * u;
            vn[u] = (i > k - 1 && i < l) ? A[i * l + (k - 1)] : 0.f;
          }
        }
        float sdot = 0.f;
#pragma unroll
        for (int u = 0; u < kZ; ++u) sdot += v[u] * z[u];
        const float f = t * row16_sum(sdot);
#pragma unroll
        for (int u = 0; u < kZ; ++u) z[u] -= f * v[u];
      }
      double* Ub = Ut + int64_t(b) * LP * kk;
#pragma unroll
      for (int u = 0; u < kZ; ++u) {
        const int i = sl + 16 * u;
        if (i < l) Ub[int64_t(i) * kk + c] = double(z[u]);
      }
      if (sl == 0) sig[int64_t(b) * kk + c] = sqrt(fmax(double(lam[c]), 0.0));
    }
  }
}

// U[o_b + r][c] = sum_{i<l} S_b[r][i] Ut_b[i][c], c < kk (global N x kk, FP32)
// on a 128-row item, FP64 MFMA: wave w computes the 16 rows 16w.. for all
// column blocks; A[m][k] = S[16w + m][k], B[k][n] = Ut[k][16J + n] (Ut
// staged in FP32, the precision U is stored in).
constexpr int kBasisT = 512;
template <class TY, int LP>
__global__ __launch_bounds__(kBasisT) void k_basis(BlockMeta bm, const TY* __restrict__ S,
                                                   const double* __restrict__ Ut, float* __restrict__ U) {
  constexpr int LD = LP + 1, KS = kMaxLP + 1, NCM = kMaxLP / 16;
  __shared__ float Ub[LP * KS];    // Ut_b, rows < l (zero beyond), odd row stride
  __shared__ TY St[128 * LD];
  const int b = bm.pair_b[bm.p0 + blockIdx.x], t = bm.pair_t[bm.p0 + blockIdx.x];
  const int o = bm.off[b], n = bm.off[b + 1] - o, nbp = bm.nbp[b];
  const int l = bm.l, kk = bm.kk;
  const int rows = min(128, nbp - t * 64);
  const double* Utb = Ut + int64_t(b) * LP * kk;
  for (int q = threadIdx.x; q < LP * kk; q += kBasisT) {
    const int i = q / kk, c = q - i * kk;
    Ub[i * KS + c] = i < l ? float(Utb[q]) : 0.f;
  }
  stage_block<128, LP, LD, kBasisT>(St, S + bm.yoff[b] + int64_t(t) * 64 * LP, l, rows);
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int lm = lane % 16, lk = lane / 16;
  const int vrows = min(rows, n - t * 64);   // rows of the block (the padding has no U)
  if (16 * wave >= vrows) return;
  const int nc = (kk + 15) / 16;
  doublex4 acc[NCM];
#pragma unroll
  for (int J = 0; J < NCM; ++J) acc[J] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k0 = 0; k0 < LP; k0 += 4) {
    const double a = double(St[(16 * wave + lm) * LD + k0 + lk]);
#pragma unroll
    for (int J = 0; J < NCM; ++J)
      if (J < nc) acc[J] = mfma_f64(a, double(Ub[(k0 + lk) * KS + 16 * J + lm]), acc[J]);
  }
  // columns past kk of Ub are not staged: their outputs are not written
#pragma unroll
  for (int J = 0; J < NCM; ++J)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * wave + lk + 4 * v, c = 16 * J + lm;
      if (J < nc && r < vrows && c < kk) U[int64_t(o + t * 64 + r) * kk + c] = float(acc[J][v]);
    }
}

// ------------------------------------------------ block preconditioner --

// dT_b = diag(d_b) U_b' R_b, d_i = sigma_i / (1 + lambda - sigma_i), in two
// steps: every (64-row tile, 64-column slab) writes its partial product
// (kk x 64, FP64), then the tiles of a block are summed in tile order.
constexpr int kPrecT = 24;  // outputs per thread: kk * 64 <= 256 * kPrecT
template <class T>
__global__ __launch_bounds__(kBlock) void k_prec_t_tiles(BlockMeta bm, const float* __restrict__ U,
                                                         const T* __restrict__ R, int64_t ldr, int nrhs,
                                                         double* __restrict__ part) {
  __shared__ double su[64 * kMaxLP];
  __shared__ double sr[64 * 64];
  const int b = bm.item_b[blockIdx.x], t = bm.item_t[blockIdx.x];
  const int c0 = blockIdx.y * 64;
  const int o = bm.off[b], n = bm.off[b + 1] - o, kk = bm.kk;
  const int nc = min(64, nrhs - c0);
  const int r0 = t * 64;
  const int rows = max(0, min(64, n - r0));
  stage_rows(su, kk, U + int64_t(o + r0) * kk, kk, rows, kk);
  stage_rows(sr, 64, R + int64_t(o + r0) * ldr + c0, ldr, rows, nc);
  __syncthreads();
  double* out = part + (int64_t(blockIdx.x) * gridDim.y + blockIdx.y) * kk * 64;
#pragma unroll
  for (int a = 0; a < kPrecT; ++a) {
    const int w = threadIdx.x + a * kBlock;
    if (w < kk * 64) {
      const int i = w >> 6, cc = w & 63;
      double sacc = 0.0;
      if (cc < nc)
        for (int rr = 0; rr < rows; ++rr) sacc += su[rr * kk + i] * sr[rr * 64 + cc];
      out[w] = sacc;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_prec_t_reduce(BlockMeta bm, const int32_t* __restrict__ item0,
                                                          const double* __restrict__ part, const double* __restrict__ sig,
                                                          double lam, int nrhs, int slabs, double* __restrict__ dT) {
  const int b = blockIdx.x;
  const int kk = bm.kk;
  const int w = blockIdx.y * kBlock + threadIdx.x;  // over kk * nrhs outputs
  if (w >= kk * nrhs) return;
  const int i = w / nrhs, c = w - i * nrhs;
  const int slab = c >> 6, cc = c & 63;
  double sacc = 0.0;
#pragma unroll 8
  for (int it = item0[b]; it < item0[b + 1]; ++it)
    sacc += part[(int64_t(it) * slabs + slab) * kk * 64 + i * 64 + cc];
  const double si = sig[int64_t(b) * kk + i];
  dT[(int64_t(b) * kk + i) * nrhs + c] = sacc * si / (1.0 + lam - si);
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
    if (threadIdx.x < W && c < nrhs) part[int64_t(t) * nrhs + c] = s;
    if (blockIdx.y == 0) {
      const int64_t total = int64_t(n_long) * nrhs;
      for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
           i += int64_t(gridDim.x) * blockDim.x)
        part[int64_t(n_tiles) * nrhs + i] = 0.0;
    }
  }
}

// -------------------------------------------------------------- driver --

// Workspace of the block rSVD; kept by the handle between calls (buffers
// only grow), so repeated calls allocate nothing.
struct Rsvd {
  int nb = 0, l = 0, LP = 0, kk = 0;
  bool f64 = false;
  std::vector<int32_t> off, nbp, item_b, item_t, item0, pair_b, pair_t, pair0, gemm_b, gemm_t;
  std::vector<int64_t> aoff, yoff;
  int64_t a_elems = 0, y_elems = 0;
  int max_nbp = 0;
  // device
  DevBuf meta, A, Y, S, ST, Gpart, Li, Ut, sig, fail, omega, U, dT, Tpart;
  const int32_t* item0_d = nullptr;
  const int32_t* pair0_d = nullptr;   // [nb+1] first 128-row item of each block
  BlockMeta bm{};
  // the block layout the metadata was built for, and its generation
  std::vector<int32_t> layout_key;
  uint64_t layout_gen = 0;
  // groups of consecutive blocks: first blocks [ngroups+1], and the start
  // and length of each group's GEMM list ([0]: all blocks as one group)
  std::vector<int> grp_b0, grp_g0, grp_ng;
  // the rSVD's launches recorded as a HIP graph, replayed while the values
  // they bake in are unchanged; a capture stream and an event per group
  hipGraphExec_t graph = nullptr;
  std::vector<uint64_t> graph_key;
  hipStream_t cap[kGroups] = {};
  hipEvent_t ev[kGroups] = {};
};

static void rsvd_delete(void* p) {
  Rsvd* R = static_cast<Rsvd*>(p);
  DevBuf* bufs[] = {&R->meta, &R->A, &R->Y, &R->S, &R->ST, &R->Gpart, &R->Li,
                    &R->Ut, &R->sig, &R->fail, &R->omega, &R->U, &R->dT, &R->Tpart};
  for (DevBuf* b : bufs) b->release();
  if (R->graph) (void)hipGraphExecDestroy(R->graph);
  for (hipStream_t c : R->cap)
    if (c) (void)hipStreamDestroy(c);
  for (hipEvent_t e : R->ev)
    if (e) (void)hipEventDestroy(e);
  delete R;
}

static Rsvd& rsvd_of(hgl_handle* h) {
  if (!h->rsvd_ws) {
    Rsvd* R = new Rsvd();
    attach(h, R->meta, R->A, R->Y, R->S, R->ST, R->Gpart, R->Li, R->Ut, R->sig, R->fail, R->omega, R->U, R->dT,
           R->Tpart);
    h->rsvd_ws = R;
    h->rsvd_free = &rsvd_delete;
  }
  return *static_cast<Rsvd*>(h->rsvd_ws);
}

static int rsvd_setup(hgl_handle* h, Rsvd& R, int n_blocks, const int32_t* offs, const hgl_rsvd_opts* o,
                      hipStream_t s) {
  // unchanged layout: the metadata and buffers of the last call stand
  std::vector<int32_t> key = {n_blocks, o->k, o->p, o->sketch};
  key.insert(key.end(), offs, offs + n_blocks + 1);
  if (R.meta.p && key == R.layout_key) return HGL_OK;
  R.nb = n_blocks;
  R.l = o->k + o->p;
  R.kk = o->k;
  R.LP = (R.l + 15) / 16 * 16;
  R.f64 = o->sketch == HGL_SKETCH_F64;
  R.off.assign(offs, offs + n_blocks + 1);
  R.nbp.assign(n_blocks, 0);
  R.aoff.assign(n_blocks, 0);
  R.yoff.assign(n_blocks, 0);
  R.item_b.clear();
  R.item_t.clear();
  R.item0.assign(n_blocks + 1, 0);
  R.pair_b.clear();
  R.pair_t.clear();
  R.pair0.assign(n_blocks + 1, 0);
  R.max_nbp = 0;
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
    R.item0[b] = int32_t(R.item_b.size());
    for (int t = 0; t < p / 64; ++t) {
      R.item_b.push_back(b);
      R.item_t.push_back(t);
    }
    R.pair0[b] = int32_t(R.pair_b.size());
    for (int t = 0; t < p / 64; t += 2) {
      R.pair_b.push_back(b);
      R.pair_t.push_back(t);
    }
  }
  R.item0[n_blocks] = int32_t(R.item_b.size());
  R.pair0[n_blocks] = int32_t(R.pair_b.size());
  // GEMM items in XCD order: the dispatcher deals workgroup w to XCD w % 8,
  // so the blocks are dealt to the XCDs (largest first, each to the least
  // loaded, load = items x rows) and the launch interleaves the XCDs'
  // lists: every item of a block then runs on one XCD, whose L2 keeps the
  // block's S' for all of them.
  // One list for all blocks, then one per group (each a multiple of kXcd
  // long, so a group's launch keeps the dealing).
  R.gemm_b.clear();
  R.gemm_t.clear();
  R.grp_g0.clear();
  R.grp_ng.clear();
  auto deal = [&](int b_lo, int b_hi) {
    std::vector<int> order;
    for (int b = b_lo; b < b_hi; ++b) order.push_back(b);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return R.nbp[x] > R.nbp[y]; });
    std::vector<std::vector<int>> lists(kXcd);
    std::vector<int64_t> load(kXcd, 0);
    for (int b : order) {
      const int x = int(std::min_element(load.begin(), load.end()) - load.begin());
      for (int q = R.pair0[b]; q < R.pair0[b + 1]; ++q) lists[x].push_back(q);
      load[x] += int64_t(R.pair0[b + 1] - R.pair0[b]) * R.nbp[b];
    }
    size_t len = 0;
    for (const auto& v : lists) len = std::max(len, v.size());
    const size_t g0 = R.gemm_b.size();
    R.gemm_b.resize(g0 + len * kXcd, -1);
    R.gemm_t.resize(g0 + len * kXcd, 0);
    for (int x = 0; x < kXcd; ++x)
      for (size_t j = 0; j < lists[x].size(); ++j) {
        R.gemm_b[g0 + j * kXcd + x] = R.pair_b[lists[x][j]];
        R.gemm_t[g0 + j * kXcd + x] = R.pair_t[lists[x][j]];
      }
    R.grp_g0.push_back(int(g0));
    R.grp_ng.push_back(int(len * kXcd));
  };
  deal(0, n_blocks);
  const int ngrp = std::min(kGroups, n_blocks);
  R.grp_b0.assign(1, 0);
  for (int g = 0; g < ngrp; ++g) {
    R.grp_b0.push_back(int(int64_t(n_blocks) * (g + 1) / ngrp));
    deal(R.grp_b0[g], R.grp_b0[g + 1]);
  }
  R.a_elems = a;
  R.y_elems = y;
  const size_t nI = R.item_b.size(), nP = R.pair_b.size(), nG = R.gemm_b.size();
  const size_t meta_bytes = 4 * (n_blocks + 1) + 4 * n_blocks + 8 * 2 * n_blocks + 4 * 2 * nI + 4 * (n_blocks + 1) +
                            4 * 2 * nP + 4 * (n_blocks + 1) + 4 * 2 * nG + 64;
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
  const size_t p_i0 = put(R.item0.data(), 4 * (n_blocks + 1), 4);
  const size_t p_pb = put(R.pair_b.data(), 4 * nP, 4);
  const size_t p_pt = put(R.pair_t.data(), 4 * nP, 4);
  const size_t p_p0 = put(R.pair0.data(), 4 * (n_blocks + 1), 4);
  const size_t p_gb = put(R.gemm_b.data(), 4 * nG, 4);
  const size_t p_gt = put(R.gemm_t.data(), 4 * nG, 4);
  HGL_TRY(ensure_pinned(h, (pos + 7) / 8 + 8));
  std::memcpy(h->pinned_d, host.data(), pos);
  HGL_HIP(hipMemcpyAsync(R.meta.p, h->pinned_d, pos, hipMemcpyHostToDevice, s));
  HGL_HIP(hipStreamSynchronize(s));
  char* base = static_cast<char*>(R.meta.p);
  R.bm = BlockMeta{n_blocks, R.l, R.LP, R.kk,
                   reinterpret_cast<const int32_t*>(base + p_off), reinterpret_cast<const int32_t*>(base + p_nbp),
                   reinterpret_cast<const int64_t*>(base + p_aoff), reinterpret_cast<const int64_t*>(base + p_yoff),
                   reinterpret_cast<const int32_t*>(base + p_ib), reinterpret_cast<const int32_t*>(base + p_it),
                   reinterpret_cast<const int32_t*>(base + p_pb), reinterpret_cast<const int32_t*>(base + p_pt),
                   reinterpret_cast<const int32_t*>(base + p_gb), reinterpret_cast<const int32_t*>(base + p_gt)};
  R.item0_d = reinterpret_cast<const int32_t*>(base + p_i0);
  R.pair0_d = reinterpret_cast<const int32_t*>(base + p_p0);
  HGL_TRY(R.Gpart.reserve(8 * nP * size_t(R.l) * (R.l + 1) / 2));
  const size_t ea = R.f64 ? 8 : 2, ey = R.f64 ? 8 : 4;
  HGL_TRY(R.A.reserve(ea * R.a_elems));
  HGL_TRY(R.Y.reserve(ey * R.y_elems));
  HGL_TRY(R.S.reserve(ey * R.y_elems));
  HGL_TRY(R.ST.reserve(ea * R.y_elems * (R.f64 ? 1 : 2)));  // BF16: hi and lo halves
  HGL_TRY(R.Li.reserve(8 * size_t(n_blocks) * R.LP * R.LP));
  HGL_TRY(R.Ut.reserve(8 * size_t(n_blocks) * R.LP * R.kk));
  HGL_TRY(R.sig.reserve(8 * size_t(n_blocks) * R.kk));
  HGL_TRY(R.fail.reserve(4 * size_t(n_blocks)));
  R.layout_key = key;
  ++R.layout_gen;
  return HGL_OK;
}

__global__ void k_zero_i32(int32_t* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Bytes of LDS the kernel declares statically (0 if the query fails).
template <class K>
static size_t static_lds(K kernel) {
  hipFuncAttributes attr{};
  if (hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(kernel)) != hipSuccess) return 0;
  return attr.sharedSizeBytes;
}

// Kernels whose dynamic LDS exceeds the default 64 KiB must opt in (gfx950
// has 160 KiB of LDS per CU, static and dynamic together).
template <class K>
static int allow_lds(K kernel, size_t bytes) {
  if (bytes + static_lds(kernel) > 160 * 1024) {
    set_error("kernel needs %zu bytes of LDS", bytes + static_lds(kernel));
    return HGL_EUNSUPPORTED;
  }
  if (bytes > 64 * 1024)
    HGL_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
  return HGL_OK;
}

// Calls f(std::integral_constant<int, LP>{}) for the supported padded widths.
template <class F>
static int with_lp(int LP, F&& f) {
  switch (LP) {
    case 16: return f(std::integral_constant<int, 16>{});
    case 32: return f(std::integral_constant<int, 32>{});
    case 48: return f(std::integral_constant<int, 48>{});
    case 64: return f(std::integral_constant<int, 64>{});
    case 80: return f(std::integral_constant<int, 80>{});
    case 96: return f(std::integral_constant<int, 96>{});
    default: set_error("unsupported padded sketch width %d", LP); return HGL_EUNSUPPORTED;
  }
}

// Consecutive blocks whose chain of launches runs on one stream: the blocks
// are independent, so while one group's single-CU steps (Cholesky, the
// small eigenproblem) hold a few CUs, another group's products fill the rest.
struct Grp {
  BlockMeta bm;   // the handle's, with the group's first block and items
  hipStream_t s;
  int nb, npair, nitem, ngemm;
};

// All blocks as one group on s, or the layout's groups on st[0..].
static std::vector<Grp> groups_of(const Rsvd& R, bool split, hipStream_t s, const hipStream_t* st) {
  std::vector<Grp> G;
  if (!split || R.grp_b0.size() < 3) {
    G.push_back({R.bm, s, R.nb, int(R.pair_b.size()), int(R.item_b.size()), R.grp_ng[0]});
    return G;
  }
  for (size_t g = 0; g + 1 < R.grp_b0.size(); ++g) {
    const int b0 = R.grp_b0[g], b1 = R.grp_b0[g + 1];
    Grp x{R.bm, st[g], b1 - b0, R.pair0[b1] - R.pair0[b0], R.item0[b1] - R.item0[b0], R.grp_ng[g + 1]};
    x.bm.b0 = b0;
    x.bm.p0 = R.pair0[b0];
    x.bm.i0 = R.item0[b0];
    x.bm.g0 = R.grp_g0[g + 1];
    G.push_back(x);
  }
  return G;
}

static int launch_gemm(hgl_handle* h, Rsvd& R, const std::vector<Grp>& G) {
  for (const Grp& g : G) {
    if (R.f64) {
      launch(h, -1, k_gemm_f64, dim3(g.nitem), dim3(kBlock), 0, g.s, g.bm, R.A.as<double>(), R.ST.as<double>(),
             R.Y.as<double>());
    } else {
      HGL_TRY(with_lp(R.LP, [&](auto c) {
        constexpr int LP = decltype(c)::value;
        launch(h, -1, k_gemm_bf16<LP>, dim3(g.ngemm), dim3(kGemmT), 0, g.s, g.bm, R.A.as<uint16_t>(),
               R.ST.as<uint16_t>(), R.y_elems, R.Y.as<float>());
        return HGL_OK;
      }));
    }
  }
  HGL_HIP(hipGetLastError());
  return HGL_OK;
}

// Gram tile partials of Yb, then each block's sum over its first partial.
template <class TY>
static int launch_gram(hgl_handle* h, Rsvd& R, const DevBuf& Yb, const std::vector<Grp>& G) {
  const int npairs = R.l * (R.l + 1) / 2;
  for (const Grp& g : G) {
    HGL_TRY(with_lp(R.LP, [&](auto c) {
      constexpr int LP = decltype(c)::value;
      launch(h, -1, k_gram_tiles<TY, LP>, dim3(g.npair), dim3(kGramT), 0, g.s, g.bm, Yb.as<TY>(),
             R.Gpart.as<double>());
      return HGL_OK;
    }));
    launch(h, -1, k_gram_reduce, dim3((npairs + 255) / 256, g.nb), dim3(256), 0, g.s, g.bm, R.pair0_d,
           R.Gpart.as<double>());
  }
  HGL_HIP(hipGetLastError());
  return HGL_OK;
}

// S, ST <- orth(Y) by CholQR2 (Y is overwritten by the first pass).
template <class TY, class TST>
static int cholqr(hgl_handle* h, Rsvd& R, const std::vector<Grp>& G, int passes) {
  const size_t lds_chol = sizeof(double) * 2 * size_t(R.LP) * (R.LP + 1);
  prof_begin(h, kProfQr, G[0].s);
  for (int pass = 0; pass < passes; ++pass) {
    DevBuf& in = pass == 0 ? R.Y : R.S;
    DevBuf& out = pass == 0 ? R.S : R.Y;
    HGL_TRY(launch_gram<TY>(h, R, in, G));
    for (const Grp& g : G) {
      HGL_TRY(with_lp(R.LP, [&](auto c) -> int {
        constexpr int NX = decltype(c)::value / 16;
        HGL_TRY(allow_lds(k_chol_inv<NX>, lds_chol));
        launch(h, -1, k_chol_inv<NX>, dim3(g.nb), dim3(kCholT), lds_chol, g.s, g.bm, R.pair0_d,
               R.Gpart.as<double>(), R.Li.as<double>(), R.fail.as<int32_t>());
        return HGL_OK;
      }));
      HGL_TRY(with_lp(R.LP, [&](auto c) {
        constexpr int LP = decltype(c)::value;
        launch(h, -1, k_apply_rinv<TY, TST, LP>, dim3(g.npair), dim3(kApplyT), 0, g.s, g.bm, in.as<TY>(),
               R.Li.as<double>(), out.as<TY>(), R.ST.as<TST>(), R.y_elems);
        return HGL_OK;
      }));
    }
    HGL_HIP(hipGetLastError());
  }
  prof_end(h, G[0].s);
  // after two passes the basis is in R.Y; keep it in R.S
  if (passes == 2) std::swap(R.Y, R.S);
  return HGL_OK;
}

// The launches of Algorithm 1 before the basis product: the ones over all
// blocks on s0, then each group's chain on its stream (the groups' streams
// already wait for s0).
template <class TY, class TST>
static int run_rsvd(hgl_handle* h, Rsvd& R, const hgl_rsvd_opts* o, const uint16_t* omega, hipStream_t s0,
                    const std::vector<Grp>& G, const std::function<int()>& fork) {
  launch(h, -1, k_zero_i32, dim3((R.nb + 255) / 256), dim3(256), 0, s0, R.fail.as<int32_t>(), R.nb);
  const size_t lds_ex = (R.f64 ? sizeof(double) : sizeof(float)) * kExW * R.max_nbp;
  if (lds_ex > 160 * 1024) {
    set_error("diagonal block too large for LDS staging (%d rows)", R.max_nbp);
    return HGL_EUNSUPPORTED;
  }
  // the sketch Omega (caller's, or Philox from the seed: its buffer was
  // reserved by the caller)
  const uint16_t* om = omega;
  if (!om) {
    const int64_t pairs = (int64_t(h->N) * R.l + 1) / 2;
    launch(h, -1, k_philox_sketch, dim3(int((pairs + 255) / 256)), dim3(256), 0, s0, int64_t(h->N), R.l, o->seed,
           R.omega.as<uint16_t>());
    om = R.omega.as<uint16_t>();
  }
  const bool power = o->scheme == HGL_RSVD_POWER;
  if (power && o->q > 0) {
    // the power scheme lays each product out unchanged as the next operand:
    // identity factors (no orthonormalisation before the last product)
    const int64_t n = int64_t(R.nb) * R.LP * R.LP;
    launch(h, -1, k_identity_factor, dim3(int(std::min<int64_t>((n + 255) / 256, 4096))), dim3(256), 0, s0, n,
           R.LP, R.l, R.Li.as<double>());
  }
  HGL_HIP(hipGetLastError());
  HGL_TRY(fork());
  // 1. dense diagonal blocks A_bb, and Omega's rows of each block into ST
  prof_begin(h, kProfExtract, G[0].s);
  for (const Grp& g : G) {
    dim3 grid((R.max_nbp + kExW - 1) / kExW, g.nb);
    if (R.f64) {
      HGL_TRY(allow_lds(k_extract_blocks<double>, lds_ex));
      launch(h, -1, k_extract_blocks<double>, grid, dim3(kExW * kWave), lds_ex, g.s, g.bm, h->vtx_ptr, h->vtx_edge,
             h->edge_ptr, h->edge_vtx, h->s64, h->c64, R.A.as<double>(), R.max_nbp);
    } else {
      HGL_TRY(allow_lds(k_extract_blocks<uint16_t>, lds_ex));
      launch(h, -1, k_extract_blocks<uint16_t>, grid, dim3(kExW * kWave), lds_ex, g.s, g.bm, h->vtx_ptr,
             h->vtx_edge, h->edge_ptr, h->edge_vtx, h->s64, h->c64, R.A.as<uint16_t>(), R.max_nbp);
    }
  }
  HGL_HIP(hipGetLastError());
  prof_end(h, G[0].s);
  for (const Grp& g : G)
    launch(h, -1, k_sketch_to_st<TST>, dim3(64, g.nb), dim3(256), 0, g.s, g.bm, om, R.ST.as<TST>(), R.y_elems);
  HGL_HIP(hipGetLastError());
  // 2. Y = A Omega, S = orth(Y); q subspace iterations (or the power scheme)
  auto gemm = [&]() -> int {
    prof_begin(h, kProfGemm, G[0].s);
    const int st = launch_gemm(h, R, G);
    prof_end(h, G[0].s);
    return st;
  };
  // Orthonormalisation by CholQR2 (two passes) where the basis must be
  // orthonormal to working precision: the one the Rayleigh-Ritz step uses,
  // and every one of an FP64 sketch.  Between the products of a BF16 sketch
  // one pass suffices: it only has to keep the basis well conditioned, and
  // the next product and the final CholQR2 act on the subspace it spans.
  auto orth = [&](bool last) { return cholqr<TY, TST>(h, R, G, (last || R.f64) ? 2 : 1); };
  HGL_TRY(gemm());
  if (power) {
    // eq. 10: Y = (A A')^q A Omega (A_bb is symmetric: 2q + 1 products with
    // A), each product's result laid out unchanged as the next operand, and
    // one two-pass CholQR of the last Y
    for (int i = 0; i < 2 * o->q; ++i) {
      prof_begin(h, kProfQr, G[0].s);
      for (const Grp& g : G)
        HGL_TRY(with_lp(R.LP, [&](auto c) {
          constexpr int LP = decltype(c)::value;
          launch(h, -1, k_apply_rinv<TY, TST, LP>, dim3(g.npair), dim3(kApplyT), 0, g.s, g.bm, R.Y.as<TY>(),
                 R.Li.as<double>(), R.S.as<TY>(), R.ST.as<TST>(), R.y_elems);
          return HGL_OK;
        }));
      HGL_HIP(hipGetLastError());
      prof_end(h, G[0].s);
      HGL_TRY(gemm());
    }
    HGL_TRY(orth(true));
  } else {
    HGL_TRY(orth(o->q == 0));
    for (int i = 0; i < 2 * o->q; ++i) {
      HGL_TRY(gemm());
      HGL_TRY(orth(i == 2 * o->q - 1));
    }
  }
  // 3. W = A S; B B' = W'W; its top eigenpairs
  HGL_TRY(gemm());  // W in R.Y, basis S in R.S
  prof_begin(h, kProfEig, G[0].s);
  HGL_TRY(launch_gram<TY>(h, R, R.Y, G));
  const int half = (R.l + (R.l & 1)) / 2;
  if (!R.f64) {
    // BF16 sketch: FP32 tridiagonal eigensolver
    auto lds_eig = [&](int cw) {
      return sizeof(float) * (size_t(R.l) * R.l + size_t(R.l) * R.kk + 5 * size_t(R.l) * cw);
    };
    const int cw = lds_eig(64) + static_lds(k_eig_tridiag) <= 160 * 1024 ? 64 : 32;
    HGL_TRY(allow_lds(k_eig_tridiag, lds_eig(cw)));
    for (const Grp& g : G)
      launch(h, -1, k_eig_tridiag, dim3(g.nb), dim3(kEigT), lds_eig(cw), g.s, g.bm, R.pair0_d, R.Gpart.as<double>(),
             R.sig.as<double>(), R.Ut.as<double>(), cw);
  } else {
    // FP64 sketch: FP64 cyclic Jacobi, A double-buffered where it fits in
    // LDS; 1024 threads while three tasks per thread cover a round (l <= 90),
    // 512 beyond (more tasks per thread without register spills)
    const int ntask = half + half * (half - 1) / 2 + (R.l + 1) / 2 * half;
    const int nt = ntask <= 3 * 1024 ? 1024 : 512;
    auto lds_jac = [&](int copies) {
      const size_t mats = (sizeof(double) * copies * R.l * R.l + 4 * R.l + 15) / 16 * 16;
      return mats + (nt / kWave) * half * sizeof(JacPair<double>);
    };
    const bool db = lds_jac(3) <= 160 * 1024;
    const size_t lds_j = lds_jac(db ? 3 : 2);
    using JacFn = void (*)(BlockMeta, const int32_t*, const double*, double*, double*, int);
    JacFn jac = nt == 1024 ? (db ? &k_jacobi<1024, 3, double, true> : &k_jacobi<1024, 3, double, false>)
                           : (db ? &k_jacobi<512, 7, double, true> : &k_jacobi<512, 7, double, false>);
    HGL_TRY(allow_lds(jac, lds_j));
    for (const Grp& g : G)
      launch(h, -1, jac, dim3(g.nb), dim3(nt), lds_j, g.s, g.bm, R.pair0_d, R.Gpart.as<double>(),
             R.sig.as<double>(), R.Ut.as<double>(), 30);
  }
  HGL_HIP(hipGetLastError());
  prof_end(h, G[0].s);
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
  HGL_CHECK_ARG(o->scheme == HGL_RSVD_SUBSPACE || o->scheme == HGL_RSVD_POWER, "unknown rSVD scheme %d", o->scheme);
  for (int b = 0; b < n_blocks; ++b)
    HGL_CHECK_ARG(offs[b + 1] - offs[b] >= o->k + o->p,
                  "block %d has %d rows, fewer than k + p = %d", b, offs[b + 1] - offs[b], o->k + o->p);
  return HGL_OK;
}

static int finish_rsvd(hgl_handle* h, Rsvd& R, float* U_out, double* sigma_out, hipStream_t s) {
  const std::vector<Grp> G = groups_of(R, false, s, nullptr);
  HGL_TRY(with_lp(R.LP, [&](auto c) {
    constexpr int LP = decltype(c)::value;
    if (R.f64)
      launch(h, -1, k_basis<double, LP>, dim3(G[0].npair), dim3(kBasisT), 0, s, R.bm, R.S.as<double>(),
             R.Ut.as<double>(), U_out);
    else
      launch(h, -1, k_basis<float, LP>, dim3(G[0].npair), dim3(kBasisT), 0, s, R.bm, R.S.as<float>(),
             R.Ut.as<double>(), U_out);
    return HGL_OK;
  }));
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

// The rSVD's launches, recorded once as a HIP graph on a capture stream and
// replayed on s while every value they bake in (buffer addresses, the
// layout, the options, the sketch) is unchanged: the launches over all
// blocks, then a fork into the groups' chains (one capture stream each)
// and a join.  Direct launches, the first group on s and the others on
// spare streams, while kernel timing is on.  The graph holds kernels only.
static int rsvd_any(hgl_handle* h, Rsvd& R, const hgl_rsvd_opts* o, const uint16_t* omega, hipStream_t s) {
  if (!omega) HGL_TRY(R.omega.reserve(sizeof(uint16_t) * size_t(h->N) * R.l + 16));
  auto run = [&](hipStream_t s0, const std::vector<Grp>& G, const std::function<int()>& fork) {
    return R.f64 ? run_rsvd<double, double>(h, R, o, omega, s0, G, fork)
                 : run_rsvd<float, uint16_t>(h, R, o, omega, s0, G, fork);
  };
  for (int g = 1; g < kGroups; ++g)
    if (!R.cap[g]) HGL_HIP(hipStreamCreateWithFlags(&R.cap[g], hipStreamNonBlocking));
  if (!R.ev[0])
    for (auto& e : R.ev) HGL_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  // fork: the other groups' streams wait for what is queued on st[0] so far
  auto forker = [&](const std::vector<Grp>& G, const hipStream_t* st) {
    return [&G, st, &R]() -> int {
      if (G.size() > 1) {
        HGL_HIP(hipEventRecord(R.ev[0], st[0]));
        for (size_t g = 1; g < G.size(); ++g) HGL_HIP(hipStreamWaitEvent(st[g], R.ev[0], 0));
      }
      return HGL_OK;
    };
  };
  auto join = [&](const std::vector<Grp>& G, const hipStream_t* st) -> int {
    for (size_t g = 1; g < G.size(); ++g) {
      HGL_HIP(hipEventRecord(R.ev[g], st[g]));
      HGL_HIP(hipStreamWaitEvent(st[0], R.ev[g], 0));
    }
    return HGL_OK;
  };
  if (h->prof_on) {
    // direct launches: the groups on s and the spare streams
    hipStream_t st[kGroups];
    st[0] = s;
    for (int g = 1; g < kGroups; ++g) st[g] = R.cap[g];
    const std::vector<Grp> G = groups_of(R, true, s, st);
    HGL_TRY(run(s, G, forker(G, st)));
    return join(G, st);
  }
  auto u = [](const void* p) { return uint64_t(reinterpret_cast<uintptr_t>(p)); };
  // (the host swaps the roles of R.Y and R.S while it records; a replay
  // does not, so the key a replay must match is the one after recording)
  auto key_now = [&]() {
    return std::vector<uint64_t>{R.layout_gen, u(R.meta.p), u(R.A.p), u(R.Y.p), u(R.S.p), u(R.ST.p),
                                 u(R.Gpart.p), u(R.Li.p), u(R.Ut.p), u(R.sig.p), u(R.fail.p), u(R.omega.p),
                                 u(omega), u(h->vtx_ptr), u(h->vtx_edge), u(h->edge_ptr), u(h->edge_vtx),
                                 u(h->s64), u(h->c64), uint64_t(o->k), uint64_t(o->p), uint64_t(o->q),
                                 uint64_t(o->scheme), uint64_t(o->sketch), o->seed};
  };
  if (!R.graph || key_now() != R.graph_key) {
    if (R.graph) {
      HGL_HIP(hipGraphExecDestroy(R.graph));
      R.graph = nullptr;
    }
    if (!R.cap[0]) HGL_HIP(hipStreamCreateWithFlags(&R.cap[0], hipStreamNonBlocking));
    // the groups' streams join the capture after the launches over all
    // blocks, and the capture stream waits for them at the end
    const std::vector<Grp> G = groups_of(R, true, R.cap[0], R.cap);
    hipGraph_t gr = nullptr;
    HGL_HIP(hipStreamBeginCapture(R.cap[0], hipStreamCaptureModeThreadLocal));
    int rc = run(R.cap[0], G, forker(G, R.cap));
    if (rc == HGL_OK) rc = join(G, R.cap);
    const hipError_t e = hipStreamEndCapture(R.cap[0], &gr);
    if (rc != HGL_OK) {
      if (gr) (void)hipGraphDestroy(gr);
      return rc;
    }
    HGL_HIP(e);
    const hipError_t e2 = hipGraphInstantiate(&R.graph, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    HGL_HIP(e2);
    R.graph_key = key_now();
  }
  HGL_HIP(hipGraphLaunch(R.graph, s));
  return HGL_OK;
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
  const int slabs = (nrhs + 63) / 64;
  const int n_items = int(R.item_b.size());
  launch(h, -1, k_prec_t_tiles<T>, dim3(n_items, slabs), dim3(kBlock), 0, s, R.bm, P->U, Rm, ldr, nrhs,
                     R.Tpart.as<double>());
  launch(h, -1, k_prec_t_reduce, dim3(R.nb, (R.kk * nrhs + kBlock - 1) / kBlock), dim3(kBlock), 0, s, R.bm,
                     R.item0_d, R.Tpart.as<double>(), R.sig.as<double>(), P->lam, nrhs, slabs, P->dT->as<double>());
  HGL_HIP(hipGetLastError());
  const ColShape cs = pick_shape(nrhs, sizeof(T), {Rm, Z}, {ldr, ldz});
  const double g = P->lam / (1.0 + P->lam);
  return HGL_DISPATCH_SHAPE(cs, sizeof(T), {
    launch(h, -1, k_prec_z<T, GL, V>, dim3(h->n_tiles, cs.slabs), dim3(kBlock), 0, s, R.bm, h->n_tiles,
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
  enter(h, s);
  HGL_TRY(check_opts(h, n_blocks, block_offsets_host, o));
  HGL_CHECK_ARG(U_out != nullptr, "U_out must not be NULL");
  Rsvd& R = rsvd_of(h);
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
  enter(h, s);
  HGL_TRY(check_opts(h, n_blocks, block_offsets_host, o));
  HGL_CHECK_ARG(lambda > 0.0 && std::isfinite(lambda), "lambda must be > 0");
  HGL_CHECK_ARG(Y && F && nrhs >= 1 && ldy >= nrhs && ldf >= nrhs, "bad Y/F/nrhs/leading dimensions");
  HGL_CHECK_ARG(o->refine_tol > 0.0, "refine_tol must be > 0");
  Rsvd& R = rsvd_of(h);
  HGL_TRY(rsvd_setup(h, R, n_blocks, block_offsets_host, o, s));
  HGL_TRY(rsvd_any(h, R, o, omega_bf16, s));
  HGL_TRY(R.U.reserve(sizeof(float) * size_t(h->N) * R.kk));
  HGL_TRY(R.dT.reserve(sizeof(double) * size_t(n_blocks) * R.kk * nrhs));
  HGL_TRY(R.Tpart.reserve(sizeof(double) * R.item_b.size() * size_t((nrhs + 63) / 64) * R.kk * 64));
  int st = finish_rsvd(h, R, R.U.as<float>(), sigma_out, s);
  if (st < 0) return st;
  BlockPrec bp{h, &R, R.U.as<float>(), lambda, &R.dT};
  Precond pc;
  pc.ctx = &bp;
  pc.apply_f32 = &prec_apply<float>;
  pc.apply_f64 = &prec_apply<double>;
  uint64_t lam_bits;
  std::memcpy(&lam_bits, &lambda, sizeof(lam_bits));
  auto u = [](const void* p) { return uint64_t(reinterpret_cast<uintptr_t>(p)); };
  pc.key = {u(R.meta.p), u(R.U.p), u(R.dT.p), u(R.Tpart.p), u(R.sig.p), lam_bits, uint64_t(R.nb),
            uint64_t(R.kk) | uint64_t(R.item_b.size()) << 32};
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

extern "C" int hgl_philox4x32_10(int64_t n, const uint32_t* ctr, uint64_t key, uint32_t* out, hipStream_t s) {
  clear_error();
  HGL_CHECK_ARG(n >= 1 && ctr != nullptr && out != nullptr, "need n >= 1 and ctr, out");
  hipLaunchKernelGGL(k_philox_words, dim3(int((n + 255) / 256)), dim3(256), 0, s, n, ctr, key, out);
  HGL_HIP(hipGetLastError());
  return HGL_OK;
}
