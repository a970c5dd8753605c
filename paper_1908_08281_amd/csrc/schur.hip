// Block inverse through Schur complements (paper, section 3, eqs. 12-14)
// under nested tessellation of every diagonal block, and its use as the
// block-diagonal preconditioner of CG.
//
// A diagonal block M_bb = (I + L/lambda)[o_b, o_b+1) of n rows is split into
// 2x2 blocks with n1 = floor(n/2) while both halves keep at least min_block
// rows.  A split node computes, in FP32 on MFMA (v_mfma_f32_16x16x4f32):
//   W1 = X11^-1, W2 = X22^-1                 (child nodes)
//   T1 = X12 W2, T2 = X21 W1, T3 = W1 X12
//   Z1 = X11 - T1 X21 (eq. 13), Z2 = X22 - T2 X12 (eq. 14)
//   Z1^-1, Z2^-1                             (child nodes, into the output)
//   top right = -T3 Z2^-1, bottom left = -Z2^-1 T2 (eq. 12)
// The smallest submatrices (min_block .. 2 min_block - 1 rows) are inverted
// exactly: eq. 15 with all of a submatrix's singular values is its exact
// inverse, and any exact method gives the same matrix up to rounding.  A
// smallest submatrix of at most kLeafMax rows is inverted by Gauss-Jordan
// elimination in FP32 registers; a larger one (min_block above 64, e.g. the
// paper's 500) by the same 2x2 construction carried on below it down to
// such pieces.  No pivoting: every matrix inverted
// here is a diagonal block of a symmetric positive definite matrix or a
// Schur complement of one, so it is symmetric positive definite too, with
// its eigenvalues in [1, 1 + 1/lambda] like those of M.
//
// Nodes run in phases: a node's two first children run in one phase range,
// its first products after them, and so on; one phase's products and
// leaves are independent, so every phase is one launch over all blocks'
// tasks of that phase (one more for its leaves).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"

namespace hgl {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kLeafMax = 127;   // rows of the largest leaf: one thread column per leaf column
constexpr int kMinBlockLo = 16;
constexpr int kMaxBlock = 4096;  // rows of a diagonal block (the extraction stages 4 FP64 rows)
constexpr int kGT = 64;          // product tile: 64 x 64 outputs per workgroup
constexpr int kGK = 16;          // k-depth of one LDS stage
constexpr int kAPT = kGT * kGK / kBlock;  // elements of A (and of B) a thread stages
static_assert(kGK % kAPT == 0 && kGT % kAPT == 0 && kBlock == (kGK / kAPT) * kGT, "stage mapping");

// D = alpha A B + beta C over FP32 row-major views of the arena (element
// offsets).  In the preconditioner's products b and d are first rows of
// the right-hand side and result, whose leading dimensions are arguments.
struct GemmTask {
  int64_t a, b, c, d;
  int32_t lda, ldb, ldc, ldd;
  int32_t m, n, k;
  float alpha, beta;
};

struct LeafTask {
  int64_t in, out;
  int32_t ldi, ldo, n, pad;
};

// M_bb = a I - b A_bb (FP32, row-major, n_b x n_b at moff[b]) with
// A_bb[u][v] = s_u s_v sum of c_e over the hyperedges holding u and v.  One
// wave per row, accumulated in LDS in FP64: hyperedges of u in increasing id
// order, members of one hyperedge on distinct lanes.
__global__ __launch_bounds__(kBlock) void k_schur_extract(const int32_t* __restrict__ boff,
                                                          const int64_t* __restrict__ moff,
                                                          const int32_t* __restrict__ vtx_ptr,
                                                          const int32_t* __restrict__ vtx_edge,
                                                          const int32_t* __restrict__ edge_ptr,
                                                          const int32_t* __restrict__ edge_vtx,
                                                          const double* __restrict__ s,
                                                          const double* __restrict__ c, double a, double b,
                                                          float* __restrict__ arena, int max_n) {
  extern __shared__ double srow[];  // [4][max_n]
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int blk = blockIdx.y;
  const int o = boff[blk], n = boff[blk + 1] - o;
  if (blockIdx.x * 4 >= n) return;  // the same for the whole workgroup
  const int ur = blockIdx.x * 4 + wave;
  double* row = srow + int64_t(wave) * max_n;
  for (int j = lane; j < n; j += kWave) row[j] = 0.0;
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
  if (ur < n) {
    const double su = s[o + ur];
    float* dst = arena + moff[blk] + int64_t(ur) * n;
    for (int j = lane; j < n; j += kWave) dst[j] = float((j == ur ? a : 0.0) - b * su * row[j]);
  }
}

// One kGT x kGT output tile per workgroup; four waves of kGT/2 x kGT/2,
// each as kGT/32 x kGT/32 MFMA 16x16x4 tiles.  A is staged k-major and B
// row-major in LDS, 16 deep, in two buffers: the next stage's loads are
// issued before this stage's MFMAs and stored into the other buffer after
// them, so one barrier per stage suffices (a buffer is rewritten only after
// the barrier that follows its last read).
// MFMA 16x16x4 f32 lane layout: lane l holds A[l%16][l/16], B[l/16][l%16]
// and D[4(l/16)+v][l%16], v < 4.
template <bool PREC>
__global__ __launch_bounds__(kBlock) void k_schur_gemm(const GemmTask* __restrict__ tasks,
                                                       const int32_t* __restrict__ tile_task,
                                                       const int32_t* __restrict__ tile_mn,
                                                       const float* __restrict__ Abase,
                                                       const float* __restrict__ Bbase,
                                                       const float* __restrict__ Cbase, float* __restrict__ Dbase,
                                                       int64_t ldb_rows, int64_t ldd_rows, Gate gate) {
  if (gate.skip()) return;
  __shared__ float As[2][kGK][kGT + 4];
  __shared__ float Bs[2][kGK][kGT + 4];
  const int32_t task = tile_task[blockIdx.x];
  if (task < 0) return;   // padding of the XCD order
  const GemmTask t = tasks[task];
  const int mn = tile_mn[blockIdx.x];
  const int m0 = (mn >> 16) * kGT, n0 = (mn & 0xffff) * kGT;
  const float* A = Abase + t.a;
  const float* B;
  float* D;
  int64_t ldb, ldd;
  if constexpr (PREC) {
    B = Bbase + t.b * ldb_rows;
    ldb = ldb_rows;
    D = Dbase + t.d * ldd_rows;
    ldd = ldd_rows;
  } else {
    B = Bbase + t.b;
    ldb = t.ldb;
    D = Dbase + t.d;
    ldd = t.ldd;
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int kAT = kGK / kAPT, kBT = kGT / kAPT;  // threads per row of the A and B stages
  const int ar = tid / kAT, ak = (tid % kAT) * kAPT;  // A stage: row, first k
  const int bk = tid / kBT, bc = (tid % kBT) * kAPT;  // B stage: k, first column
  float ra[kAPT], rb[kAPT];
  // (no branches around the loads: an element outside the operand reads
  // the operand's first element, and the store replaces it by zero, so the
  // loads stay in flight through the MFMAs)
  uint32_t okA = 0, okB = 0;
  auto load = [&](int k0) {
    const int gr = m0 + ar;
    okA = okB = 0;
#pragma unroll
    for (int j = 0; j < kAPT; ++j) {
      const int gk = k0 + ak + j;
      const bool ok = gr < t.m && gk < t.k;
      ra[j] = A[ok ? int64_t(gr) * t.lda + gk : 0];
      okA |= uint32_t(ok) << j;
    }
    const int gk = k0 + bk;
#pragma unroll
    for (int j = 0; j < kAPT; ++j) {
      const int gc = n0 + bc + j;
      const bool ok = gk < t.k && gc < t.n;
      rb[j] = B[ok ? int64_t(gk) * ldb + gc : 0];
      okB |= uint32_t(ok) << j;
    }
  };
  constexpr int kWT = kGT / 2, kFT = kWT / 16;  // wave tile, MFMA fragments along each side
  floatx4 acc[kFT][kFT];
#pragma unroll
  for (int i = 0; i < kFT; ++i)
#pragma unroll
    for (int j = 0; j < kFT; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int wr = (wave >> 1) * kWT, wc = (wave & 1) * kWT;
  const int r = lane & 15, q = lane >> 4;
  auto store = [&](int buf) {
#pragma unroll
    for (int j = 0; j < kAPT; ++j) {
      As[buf][ak + j][ar] = (okA >> j) & 1u ? ra[j] : 0.f;
      Bs[buf][bk][bc + j] = (okB >> j) & 1u ? rb[j] : 0.f;
    }
  };
  load(0);
  store(0);
  __syncthreads();
  int cur = 0;
  for (int k0 = 0; k0 < t.k; k0 += kGK) {
    const bool more = k0 + kGK < t.k;
    if (more) load(k0 + kGK);
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 4) {
      float a[kFT], b[kFT];
#pragma unroll
      for (int i = 0; i < kFT; ++i) {
        a[i] = As[cur][kk + q][wr + 16 * i + r];
        b[i] = Bs[cur][kk + q][wc + 16 * i + r];
      }
#pragma unroll
      for (int i = 0; i < kFT; ++i)
#pragma unroll
        for (int j = 0; j < kFT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  // C's elements loaded all at once (an element outside the tile reads C's
  // first one, unused), then the outputs
  float cv[kFT][kFT][4] = {};
  if constexpr (!PREC) {
    if (t.beta != 0.f) {   // uniform
#pragma unroll
      for (int i = 0; i < kFT; ++i)
#pragma unroll
        for (int j = 0; j < kFT; ++j) {
          const int col = n0 + wc + j * 16 + r;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = m0 + wr + i * 16 + q * 4 + v;
            const bool ok = row < t.m && col < t.n;
            cv[i][j][v] = Cbase[t.c + (ok ? int64_t(row) * t.ldc + col : 0)];
          }
        }
    }
  }
#pragma unroll
  for (int i = 0; i < kFT; ++i)
#pragma unroll
    for (int j = 0; j < kFT; ++j) {
      const int col = n0 + wc + j * 16 + r;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wr + i * 16 + q * 4 + v;
        if (row < t.m && col < t.n) {
          float val = t.alpha * acc[i][j][v];
          if constexpr (!PREC) {
            if (t.beta != 0.f) val += t.beta * cv[i][j][v];
          }
          D[int64_t(row) * ldd + col] = val;
        }
      }
    }
}

// Gauss-Jordan inverse of one leaf (FP32), in place in registers: thread
// (c, g) holds column c of rows g, g + 4, g + 8, ... of the leaf padded to
// 128 x 128 with the identity (the padding stays the identity, so it needs
// no bounds checks).  At step k the pivot row is scaled by 1/p (its pivot
// entry becomes 1/p) and every other row i loses X[i][k] times it (its
// entry in column k becomes -X[i][k]/p).  With row k and column k zeroed
// first and -1 stored as row k's entry of the column, every entry takes the
// same update x -= col[r] * row[c] (row[k] = 1/p, row[c] = X[k][c]/p).  Row
// k and column k go through LDS, double-buffered by step parity, so one
// barrier per step suffices: a buffer is written again two steps later,
// after every thread has passed the barrier that follows its last read.
constexpr int kLeafThreads = 1024;
constexpr int kLeafGroups = kLeafThreads / 128;      // row groups
constexpr int kLeafSlots = 128 / kLeafGroups;        // rows held per thread
static_assert(kLeafMax < 128, "a leaf fits the padded 128 x 128 layout");
__global__ __launch_bounds__(kLeafThreads) void k_schur_leaf(const LeafTask* __restrict__ tasks,
                                                             float* __restrict__ arena) {
  // column k by row group: rows g + 8 j at g * 16 + j, so that a thread
  // reads its 16 entries as four 16-byte loads
  __shared__ float rowb[2][128];
  __shared__ __align__(16) float colb[2][128];
  const LeafTask t = tasks[blockIdx.x];
  const int n = t.n;
  const int c = threadIdx.x & 127, g = threadIdx.x >> 7;
  float x[kLeafSlots];
#pragma unroll
  for (int j = 0; j < kLeafSlots; ++j) {
    const int r = g + kLeafGroups * j;
    x[j] = (c < n && r < n) ? arena[t.in + int64_t(r) * t.ldi + c] : (r == c ? 1.0f : 0.0f);
  }
  for (int k = 0; k < n; ++k) {
    float* rowk = rowb[k & 1];
    float* colk = colb[k & 1];
    const bool owner = g == (k & (kLeafGroups - 1));  // holds row k, in slot jk
    const int jk = k / kLeafGroups;
    if (c == k) {
#pragma unroll
      for (int j = 0; j < kLeafSlots; ++j) colk[g * kLeafSlots + j] = (owner && j == jk) ? -1.0f : x[j];
    }
    if (owner) {
#pragma unroll
      for (int j = 0; j < kLeafSlots; ++j)
        if (j == jk) rowk[c] = x[j];
    }
    if (c == k) {
#pragma unroll
      for (int j = 0; j < kLeafSlots; ++j) x[j] = 0.0f;
    }
    if (owner) {
#pragma unroll
      for (int j = 0; j < kLeafSlots; ++j)
        if (j == jk) x[j] = 0.0f;
    }
    __syncthreads();
    const float inv = 1.0f / rowk[k];
    const float rk = (c == k ? 1.0f : rowk[c]) * inv;
#pragma unroll
    for (int j = 0; j < kLeafSlots; ++j) x[j] = fma(-colk[g * kLeafSlots + j], rk, x[j]);
  }
  if (c < n) {
#pragma unroll
    for (int j = 0; j < kLeafSlots; ++j) {
      const int r = g + kLeafGroups * j;
      if (r < n) arena[t.out + int64_t(r) * t.ldo + c] = x[j];
    }
  }
}

// Partial <R_j, Z_j> per CG row tile (FP64), long-row slots zeroed.
__global__ __launch_bounds__(kBlock) void k_schur_rz(int n_tiles, const int32_t* __restrict__ tile_r0,
                                                     const int32_t* __restrict__ tile_r1, int n_long,
                                                     const float* __restrict__ R, int64_t ldr,
                                                     const float* __restrict__ Z, int64_t ldz, int nrhs,
                                                     double* __restrict__ part, Gate gate) {
  if (gate.skip()) return;
  __shared__ double red[4][kWave];
  const int lane = threadIdx.x % kWave, grp = threadIdx.x / kWave;
  const int col = blockIdx.y * kWave + lane;
  const int t = blockIdx.x;
  double acc = 0.0;
  if (col < nrhs)
    for (int r = tile_r0[t] + grp; r < tile_r1[t]; r += 4)
      acc += double(R[int64_t(r) * ldr + col]) * double(Z[int64_t(r) * ldz + col]);
  red[grp][lane] = acc;
  __syncthreads();
  if (grp == 0 && col < nrhs) part[int64_t(t) * nrhs + col] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
  if (blockIdx.y == 0) {
    const int64_t total = int64_t(n_long) * nrhs;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x)
      part[int64_t(n_tiles) * nrhs + i] = 0.0;
  }
}

// ---------------------------------------------------------------- plan --

struct Phase {
  int32_t tile0 = 0, tiles = 0, leaf0 = 0, leaves = 0, leaf_n = 0;
};

// Workspace of the block inverse, kept by the handle (buffers only grow).
struct Schur {
  int nb = 0, min_block = 0, max_n = 0;
  std::vector<int32_t> off;
  std::vector<int64_t> moff, ioff;  // arena offsets of M_bb and of its inverse
  int64_t inv_elems = 0, arena_elems = 0;
  std::vector<Phase> phases;
  int32_t n_tiles = 0, n_leaves = 0, n_tasks = 0, max_leaf = 0;
  double flops = 0.0;               // algorithmic flops of the products (2 m n k each)
  DevBuf arena, meta, pmeta;
  const GemmTask* d_tasks = nullptr;
  const int32_t* d_tile_task = nullptr;
  const int32_t* d_tile_mn = nullptr;
  const LeafTask* d_leaves = nullptr;
  const int32_t* d_boff = nullptr;
  const int64_t* d_moff = nullptr;
  // preconditioner products for p_nrhs columns
  int p_nrhs = -1;
  int32_t p_tiles = 0;
  const GemmTask* p_tasks = nullptr;
  const int32_t* p_tile_task = nullptr;
  const int32_t* p_tile_mn = nullptr;
  // the inverse's launches recorded as a HIP graph, replayed while the key
  // (buffers, plan, lambda) is unchanged
  uint64_t plan_gen = 0;
  hipStream_t cap = nullptr;
  hipGraphExec_t graph = nullptr;
  std::vector<uint64_t> graph_key;
};

void schur_delete(void* p) {
  Schur* S = static_cast<Schur*>(p);
  S->arena.release();
  S->meta.release();
  S->pmeta.release();
  if (S->graph) (void)hipGraphExecDestroy(S->graph);
  if (S->cap) (void)hipStreamDestroy(S->cap);
  delete S;
}

Schur& schur_of(hgl_handle* h) {
  if (!h->schur_ws) {
    Schur* S = new Schur();
    attach(h, S->arena, S->meta, S->pmeta);
    h->schur_ws = S;
    h->schur_free = &schur_delete;
  }
  return *static_cast<Schur*>(h->schur_ws);
}

struct Planner {
  int min_block;
  int64_t top = 0;
  std::vector<std::vector<GemmTask>> g;
  std::vector<std::vector<LeafTask>> l;
  double flops = 0.0;

  int64_t alloc(int64_t elems) {
    const int64_t at = top;
    top += (elems + 63) / 64 * 64;
    return at;
  }
  void gemm(int p, int64_t a, int lda, int64_t b, int ldb, int64_t c, int ldc, int64_t d, int ldd, int m, int n,
            int k, float alpha, float beta) {
    if (int(g.size()) <= p) g.resize(p + 1);
    g[p].push_back(GemmTask{a, b, c, d, lda, ldb, ldc, ldd, m, n, k, alpha, beta});
    flops += 2.0 * m * n * k;
  }
  // Inverse of the n x n view (in, ldi) into the view (out, ldo), starting
  // at phase p0; returns the first phase after it.
  int node(int64_t in, int ldi, int64_t out, int ldo, int n, int p0) {
    // a smallest submatrix of the tessellation (n < 2 min_block) is a leaf
    // when its registers allow; a larger one is inverted exactly by going on
    // with the construction below it
    if (n < 2 * min_block && n <= kLeafMax) {
      if (int(l.size()) <= p0) l.resize(p0 + 1);
      l[p0].push_back(LeafTask{in, out, ldi, ldo, n, 0});
      return p0 + 1;
    }
    const int n1 = n / 2, n2 = n - n1;
    const int64_t W1 = alloc(int64_t(n1) * n1), W2 = alloc(int64_t(n2) * n2);
    const int64_t T1 = alloc(int64_t(n1) * n2), T2 = alloc(int64_t(n2) * n1), T3 = alloc(int64_t(n1) * n2);
    const int64_t Z1 = alloc(int64_t(n1) * n1), Z2 = alloc(int64_t(n2) * n2);
    const int64_t x11 = in, x12 = in + n1, x21 = in + int64_t(n1) * ldi, x22 = x21 + n1;
    const int p1 = std::max(node(x11, ldi, W1, n1, n1, p0), node(x22, ldi, W2, n2, n2, p0));
    gemm(p1, x12, ldi, W2, n2, 0, 0, T1, n2, n1, n2, n2, 1.f, 0.f);    // T1 = X12 W2
    gemm(p1, x21, ldi, W1, n1, 0, 0, T2, n1, n2, n1, n1, 1.f, 0.f);    // T2 = X21 W1
    gemm(p1, W1, n1, x12, ldi, 0, 0, T3, n2, n1, n2, n1, 1.f, 0.f);    // T3 = W1 X12
    gemm(p1 + 1, T1, n2, x21, ldi, x11, ldi, Z1, n1, n1, n1, n2, -1.f, 1.f);  // Z1 = X11 - T1 X21
    gemm(p1 + 1, T2, n1, x12, ldi, x22, ldi, Z2, n2, n2, n2, n1, -1.f, 1.f);  // Z2 = X22 - T2 X12
    const int64_t o11 = out, o12 = out + n1, o21 = out + int64_t(n1) * ldo, o22 = o21 + n1;
    const int p2 = std::max(node(Z1, n1, o11, ldo, n1, p1 + 2), node(Z2, n2, o22, ldo, n2, p1 + 2));
    gemm(p2, T3, n2, o22, ldo, 0, 0, o12, ldo, n1, n2, n2, -1.f, 0.f);  // top right = -T3 Z2^-1
    gemm(p2, o22, ldo, T2, n1, 0, 0, o21, ldo, n2, n1, n2, -1.f, 0.f);  // bottom left = -Z2^-1 T2
    return p2 + 1;
  }
};

void add_tiles(const GemmTask& t, int32_t task, std::vector<int32_t>& tt, std::vector<int32_t>& tmn) {
  const int tm = (t.m + kGT - 1) / kGT, tn = (t.n + kGT - 1) / kGT;
  for (int i = 0; i < tm; ++i)
    for (int j = 0; j < tn; ++j) {
      tt.push_back(task);
      tmn.push_back((i << 16) | j);
    }
}

template <class T>
size_t put(std::vector<char>& host, const std::vector<T>& v) {
  const size_t at = (host.size() + 255) / 256 * 256;
  host.resize(at + sizeof(T) * v.size());
  if (!v.empty()) std::memcpy(host.data() + at, v.data(), sizeof(T) * v.size());
  return at;
}

int check_offsets(int n_blocks, const int32_t* offs, int min_block) {
  HGL_CHECK_ARG(n_blocks >= 1 && offs != nullptr, "need at least one block");
  HGL_CHECK_ARG(offs[0] == 0, "block offsets must start at 0");
  HGL_CHECK_ARG(min_block >= kMinBlockLo && min_block <= kMaxBlock, "min_block must be in [%d, %d]", kMinBlockLo,
                kMaxBlock);
  for (int b = 0; b < n_blocks; ++b) {
    const int n = offs[b + 1] - offs[b];
    HGL_CHECK_ARG(n >= 1, "block %d is empty or offsets decrease", b);
    HGL_CHECK_ARG(n <= kMaxBlock, "block %d has %d rows, more than %d", b, n, kMaxBlock);
  }
  return HGL_OK;
}

int check_blocks(hgl_handle* h, int n_blocks, const int32_t* offs, int min_block) {
  HGL_CHECK_ARG(h != nullptr, "handle must not be NULL");
  HGL_CHECK_ARG(h->G == 1, "the block inverse needs a single-graph handle");
  HGL_TRY(check_offsets(n_blocks, offs, min_block));
  HGL_CHECK_ARG(offs[n_blocks] == h->N, "block offsets must cover [0, N)");
  return HGL_OK;
}

// The phases of all blocks' inverses: host only.
struct Plan {
  std::vector<GemmTask> tasks;
  std::vector<LeafTask> leaves;
  std::vector<int32_t> tt, tmn;  // per tile: task, (tile row << 16) | tile column
  std::vector<Phase> phases;
  std::vector<int64_t> moff, ioff;
  int64_t inv_elems = 0, arena_elems = 0;
  int max_n = 0, max_leaf = 0;
  double flops = 0.0;
};

int make_plan(int n_blocks, const int32_t* offs, int min_block, Plan& out) {
  Planner P{min_block};
  out.moff.assign(n_blocks, 0);
  out.ioff.assign(n_blocks, 0);
  out.max_n = 0;
  for (int b = 0; b < n_blocks; ++b) {
    const int n = offs[b + 1] - offs[b];
    out.max_n = std::max(out.max_n, n);
    out.ioff[b] = P.top;
    P.top += int64_t(n) * n;  // inverses packed first: one copy gives them all
  }
  out.inv_elems = P.top;
  P.top = (P.top + 63) / 64 * 64;
  for (int b = 0; b < n_blocks; ++b) {
    const int n = offs[b + 1] - offs[b];
    out.moff[b] = P.alloc(int64_t(n) * n);
  }
  for (int b = 0; b < n_blocks; ++b) {
    const int n = offs[b + 1] - offs[b];
    P.node(out.moff[b], n, out.ioff[b], n, n, 0);
  }
  const int n_phases = int(std::max(P.g.size(), P.l.size()));
  P.g.resize(n_phases);
  P.l.resize(n_phases);
  out.tasks.clear();
  out.leaves.clear();
  out.tt.clear();
  out.tmn.clear();
  out.phases.assign(n_phases, Phase{});
  out.max_leaf = 0;
  for (int p = 0; p < n_phases; ++p) {
    Phase& ph = out.phases[p];
    ph.tile0 = int32_t(out.tt.size());
    // Tiles in XCD order: the dispatcher deals workgroup w to XCD w mod 8,
    // so the phase's products are dealt to the XCDs (most tiles first, each
    // to the least loaded) and the launch interleaves the XCDs' lists: all
    // tiles of a product then run on one XCD, whose L2 keeps its operands'
    // panels.  Short lists are padded with empty tiles (product -1).
    std::vector<std::vector<int32_t>> xt(kXcd), xmn(kXcd);
    std::vector<int64_t> load(kXcd, 0);
    std::vector<int32_t> order(P.g[p].size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = int32_t(i);
    auto ntile = [&](const GemmTask& t) { return int64_t((t.m + kGT - 1) / kGT) * ((t.n + kGT - 1) / kGT); };
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return ntile(P.g[p][x]) > ntile(P.g[p][y]); });
    const int32_t task0 = int32_t(out.tasks.size());
    for (int32_t i : order) {
      const int x = int(std::min_element(load.begin(), load.end()) - load.begin());
      add_tiles(P.g[p][i], task0 + i, xt[x], xmn[x]);
      load[x] += ntile(P.g[p][i]) * P.g[p][i].k;
    }
    for (const GemmTask& t : P.g[p]) out.tasks.push_back(t);
    size_t len = 0;
    for (const auto& v : xt) len = std::max(len, v.size());
    for (size_t j = 0; j < len; ++j)
      for (int x = 0; x < kXcd; ++x) {
        out.tt.push_back(j < xt[x].size() ? xt[x][j] : -1);
        out.tmn.push_back(j < xmn[x].size() ? xmn[x][j] : 0);
      }
    ph.tiles = int32_t(out.tt.size()) - ph.tile0;
    ph.leaf0 = int32_t(out.leaves.size());
    for (const LeafTask& t : P.l[p]) {
      out.leaves.push_back(t);
      ph.leaf_n = std::max(ph.leaf_n, t.n);
    }
    ph.leaves = int32_t(out.leaves.size()) - ph.leaf0;
    out.max_leaf = std::max(out.max_leaf, ph.leaf_n);
  }
  out.arena_elems = P.top;
  out.flops = P.flops;
  if (out.max_leaf > kLeafMax) {
    set_error("a leaf of %d rows exceeds %d", out.max_leaf, kLeafMax);
    return HGL_EUNSUPPORTED;
  }
  return HGL_OK;
}

// Plan and upload the task lists (skipped when the blocks and min_block are
// those of the previous plan).
int schur_plan(Schur& S, int n_blocks, const int32_t* offs, int min_block, hipStream_t s) {
  if (S.nb == n_blocks && S.min_block == min_block && std::equal(offs, offs + n_blocks + 1, S.off.begin()) &&
      S.meta.p)
    return HGL_OK;
  S.nb = 0;
  Plan P;
  HGL_TRY(make_plan(n_blocks, offs, min_block, P));
  std::vector<int32_t> boff(offs, offs + n_blocks + 1);
  std::vector<char> host;
  const size_t at_tasks = put(host, P.tasks), at_tt = put(host, P.tt), at_tmn = put(host, P.tmn);
  const size_t at_leaves = put(host, P.leaves), at_boff = put(host, boff), at_moff = put(host, P.moff);
  HGL_TRY(S.meta.reserve(host.size() + 256));
  HGL_HIP(hipMemcpyAsync(S.meta.p, host.data(), host.size(), hipMemcpyHostToDevice, s));
  HGL_HIP(hipStreamSynchronize(s));
  HGL_TRY(S.arena.reserve(sizeof(float) * size_t(P.arena_elems)));
  char* base = static_cast<char*>(S.meta.p);
  S.d_tasks = reinterpret_cast<const GemmTask*>(base + at_tasks);
  S.d_tile_task = reinterpret_cast<const int32_t*>(base + at_tt);
  S.d_tile_mn = reinterpret_cast<const int32_t*>(base + at_tmn);
  S.d_leaves = reinterpret_cast<const LeafTask*>(base + at_leaves);
  S.d_boff = reinterpret_cast<const int32_t*>(base + at_boff);
  S.d_moff = reinterpret_cast<const int64_t*>(base + at_moff);
  S.off = boff;
  S.moff = P.moff;
  S.ioff = P.ioff;
  S.phases = P.phases;
  S.inv_elems = P.inv_elems;
  S.arena_elems = P.arena_elems;
  S.max_n = P.max_n;
  S.n_tiles = int32_t(P.tt.size());
  S.n_leaves = int32_t(P.leaves.size());
  S.n_tasks = int32_t(P.tasks.size());
  S.max_leaf = P.max_leaf;
  S.flops = P.flops;
  S.min_block = min_block;
  S.p_nrhs = -1;
  S.nb = n_blocks;
  ++S.plan_gen;
  return HGL_OK;
}

template <class K>
int allow_lds(K kernel, size_t bytes) {
  if (bytes > 160 * 1024) {
    set_error("kernel needs %zu bytes of LDS", bytes);
    return HGL_EUNSUPPORTED;
  }
  if (bytes > 64 * 1024)
    HGL_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                int(bytes)));
  return HGL_OK;
}

// Extract every M_bb and invert it through the phases: every launch on st.
int schur_launches(hgl_handle* h, Schur& S, double lambda, hipStream_t st) {
  const double a = 1.0 + 1.0 / lambda, b = 1.0 / lambda;
  float* arena = S.arena.as<float>();
  const size_t ex_lds = sizeof(double) * 4 * size_t(S.max_n);
  launch(h, kProfExtract, k_schur_extract, dim3((S.max_n + 3) / 4, S.nb), dim3(kBlock), uint32_t(ex_lds), st,
         S.d_boff, S.d_moff, h->vtx_ptr, h->vtx_edge, h->edge_ptr, h->edge_vtx, h->s64, h->c64, a, b, arena,
         S.max_n);
  HGL_HIP(hipGetLastError());
  for (const Phase& ph : S.phases) {
    if (ph.leaves > 0) {
      launch(h, kProfLeaf, k_schur_leaf, dim3(ph.leaves), dim3(kLeafThreads), 0, st, S.d_leaves + ph.leaf0, arena);
      HGL_HIP(hipGetLastError());
    }
    if (ph.tiles > 0) {
      launch(h, kProfGemm, k_schur_gemm<false>, dim3(ph.tiles), dim3(kBlock), 0, st, S.d_tasks,
             S.d_tile_task + ph.tile0, S.d_tile_mn + ph.tile0, static_cast<const float*>(arena),
             static_cast<const float*>(arena), static_cast<const float*>(arena), arena, int64_t(0), int64_t(0), Gate{});
      HGL_HIP(hipGetLastError());
    }
  }
  return HGL_OK;
}

// The launches of schur_launches, recorded once as a HIP graph on a
// capture stream and replayed on s while every value they bake in (buffer
// addresses, the plan, lambda) is unchanged; direct launches while kernel
// timing is on.  The graph holds kernels only (no memory set or copy nodes).
int schur_run(hgl_handle* h, Schur& S, double lambda, hipStream_t s) {
  HGL_TRY(allow_lds(k_schur_extract, sizeof(double) * 4 * size_t(S.max_n)));
  if (h->prof_on) return schur_launches(h, S, lambda, s);
  uint64_t lam_bits;
  std::memcpy(&lam_bits, &lambda, sizeof(lam_bits));
  auto u = [](const void* p) { return uint64_t(reinterpret_cast<uintptr_t>(p)); };
  const std::vector<uint64_t> key = {u(S.arena.p), u(S.meta.p), S.plan_gen, lam_bits, u(h->vtx_ptr),
                                     u(h->vtx_edge), u(h->edge_ptr), u(h->edge_vtx), u(h->s64), u(h->c64)};
  if (!S.graph || key != S.graph_key) {
    if (S.graph) {
      HGL_HIP(hipGraphExecDestroy(S.graph));
      S.graph = nullptr;
    }
    if (!S.cap) HGL_HIP(hipStreamCreateWithFlags(&S.cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HGL_HIP(hipStreamBeginCapture(S.cap, hipStreamCaptureModeThreadLocal));
    const int rc = schur_launches(h, S, lambda, S.cap);
    const hipError_t e = hipStreamEndCapture(S.cap, &g);
    if (rc != HGL_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    HGL_HIP(e);
    const hipError_t e2 = hipGraphInstantiate(&S.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HGL_HIP(e2);
    S.graph_key = key;
  }
  HGL_HIP(hipGraphLaunch(S.graph, s));
  return HGL_OK;
}

// The preconditioner's products Z_b = M_bb^-1 R_b for nrhs columns.
int schur_prec_tasks(Schur& S, int nrhs, hipStream_t s) {
  if (S.p_nrhs == nrhs) return HGL_OK;
  std::vector<GemmTask> tasks;
  std::vector<int32_t> tt, tmn;
  for (int b = 0; b < S.nb; ++b) {
    const int n = S.off[b + 1] - S.off[b];
    const GemmTask t{S.ioff[b], S.off[b], 0, S.off[b], n, 0, 0, 0, n, nrhs, n, 1.f, 0.f};
    add_tiles(t, int32_t(tasks.size()), tt, tmn);
    tasks.push_back(t);
  }
  std::vector<char> host;
  const size_t at_tasks = put(host, tasks), at_tt = put(host, tt), at_tmn = put(host, tmn);
  HGL_TRY(S.pmeta.reserve(host.size() + 256));
  HGL_HIP(hipMemcpyAsync(S.pmeta.p, host.data(), host.size(), hipMemcpyHostToDevice, s));
  HGL_HIP(hipStreamSynchronize(s));
  char* base = static_cast<char*>(S.pmeta.p);
  S.p_tasks = reinterpret_cast<const GemmTask*>(base + at_tasks);
  S.p_tile_task = reinterpret_cast<const int32_t*>(base + at_tt);
  S.p_tile_mn = reinterpret_cast<const int32_t*>(base + at_tmn);
  S.p_tiles = int32_t(tt.size());
  S.p_nrhs = nrhs;
  return HGL_OK;
}

struct SchurPrec {
  hgl_handle* h;
  Schur* S;
};

int schur_prec_f32(void* ctx, const float* R, int64_t ldr, float* Z, int64_t ldz, double* part, int nrhs, Gate gate,
                   hipStream_t s) {
  SchurPrec* P = static_cast<SchurPrec*>(ctx);
  Schur& S = *P->S;
  hgl_handle* h = P->h;
  if (nrhs != S.p_nrhs) {
    set_error("block inverse products prepared for %d columns, asked for %d", S.p_nrhs, nrhs);
    return HGL_EINVAL;
  }
  prof_begin(h, kProfPrecond, s);
  launch(h, -1, k_schur_gemm<true>, dim3(S.p_tiles), dim3(kBlock), 0, s, S.p_tasks, S.p_tile_task, S.p_tile_mn,
         static_cast<const float*>(S.arena.as<float>()), R, static_cast<const float*>(nullptr), Z, ldr, ldz, gate);
  HGL_HIP(hipGetLastError());
  if (part) {
    launch(h, -1, k_schur_rz, dim3(h->n_tiles, (nrhs + kWave - 1) / kWave), dim3(kBlock), 0, s, h->n_tiles, h->tile_r0,
           h->tile_r1, h->n_long, R, ldr, static_cast<const float*>(Z), ldz, nrhs, part, gate);
    HGL_HIP(hipGetLastError());
  }
  prof_end(h, s);
  return HGL_OK;
}

int schur_prec_f64(void*, const double*, int64_t, double*, int64_t, double*, int, Gate, hipStream_t) {
  set_error("the Schur block inverse preconditions FP32 CG only");
  return HGL_EUNSUPPORTED;
}

}  // namespace
}  // namespace hgl

using namespace hgl;

extern "C" int hgl_block_schur_plan(int32_t n_blocks, const int32_t* block_offsets_host, int32_t min_block,
                                    int64_t* counts7, int64_t* tasks, int64_t* leaves, int32_t* phases,
                                    int64_t* tiles, int64_t* moff) {
  clear_error();
  HGL_TRY(check_offsets(n_blocks, block_offsets_host, min_block));
  HGL_CHECK_ARG(counts7 != nullptr, "counts7 must not be NULL");
  Plan P;
  HGL_TRY(make_plan(n_blocks, block_offsets_host, min_block, P));
  const int64_t c[7] = {int64_t(P.tasks.size()), int64_t(P.leaves.size()), int64_t(P.phases.size()), P.arena_elems,
                        P.inv_elems,          int64_t(P.tt.size()),     int64_t(P.flops)};
  std::copy(c, c + 7, counts7);
  if (tasks)
    for (size_t i = 0; i < P.tasks.size(); ++i) {
      const GemmTask& t = P.tasks[i];
      const int64_t row[13] = {t.a, t.b, t.c, t.d, t.lda, t.ldb, t.ldc, t.ldd, t.m, t.n, t.k,
                               int64_t(t.alpha), int64_t(t.beta)};
      std::copy(row, row + 13, tasks + 13 * i);
    }
  if (leaves)
    for (size_t i = 0; i < P.leaves.size(); ++i) {
      const LeafTask& t = P.leaves[i];
      const int64_t row[5] = {t.in, t.out, t.ldi, t.ldo, t.n};
      std::copy(row, row + 5, leaves + 5 * i);
    }
  if (phases)
    for (size_t i = 0; i < P.phases.size(); ++i) {
      const Phase& p = P.phases[i];
      const int32_t row[5] = {p.tile0, p.tiles, p.leaf0, p.leaves, p.leaf_n};
      std::copy(row, row + 5, phases + 5 * i);
    }
  if (tiles)
    for (size_t i = 0; i < P.tt.size(); ++i) {
      tiles[2 * i] = P.tt[i];
      tiles[2 * i + 1] = P.tmn[i];
    }
  if (moff) std::copy(P.moff.begin(), P.moff.end(), moff);
  return HGL_OK;
}

extern "C" int hgl_block_schur_inverse(hgl_handle* h, double lambda, int32_t n_blocks,
                                       const int32_t* block_offsets_host, int32_t min_block, float* inv_out,
                                       double* flops_out, hipStream_t s) {
  clear_error();
  enter(h, s);
  HGL_TRY(check_blocks(h, n_blocks, block_offsets_host, min_block));
  HGL_CHECK_ARG(lambda > 0.0 && std::isfinite(lambda), "lambda must be > 0");
  Schur& S = schur_of(h);
  HGL_TRY(schur_plan(S, n_blocks, block_offsets_host, min_block, s));
  HGL_TRY(schur_run(h, S, lambda, s));
  if (inv_out)
    HGL_HIP(hipMemcpyAsync(inv_out, S.arena.p, sizeof(float) * size_t(S.inv_elems), hipMemcpyDeviceToDevice, s));
  if (flops_out) *flops_out = S.flops;
  HGL_HIP(hipStreamSynchronize(s));
  return HGL_OK;
}

extern "C" int hgl_block_schur_invert(hgl_handle* h, double lambda, int32_t n_blocks,
                                      const int32_t* block_offsets_host, int32_t min_block, double refine_tol,
                                      int32_t max_refine, int32_t chunk, const float* Y, int64_t ldy, float* F,
                                      int64_t ldf, int32_t nrhs, int32_t* iters_host, double* relres_host,
                                      hipStream_t s) {
  clear_error();
  enter(h, s);
  HGL_TRY(check_blocks(h, n_blocks, block_offsets_host, min_block));
  HGL_CHECK_ARG(lambda > 0.0 && std::isfinite(lambda), "lambda must be > 0");
  HGL_CHECK_ARG(Y && F && nrhs >= 1 && ldy >= nrhs && ldf >= nrhs, "bad Y/F/nrhs/leading dimensions");
  HGL_CHECK_ARG(nrhs <= (1 << 21), "nrhs must be <= %d", 1 << 21);
  HGL_CHECK_ARG(refine_tol > 0.0 && max_refine >= 0 && chunk >= 0, "need refine_tol > 0, max_refine >= 0, chunk >= 0");
  Schur& S = schur_of(h);
  HGL_TRY(schur_plan(S, n_blocks, block_offsets_host, min_block, s));
  HGL_TRY(schur_prec_tasks(S, nrhs, s));
  HGL_TRY(schur_run(h, S, lambda, s));
  SchurPrec sp{h, &S};
  Precond pc;
  pc.ctx = &sp;
  pc.apply_f32 = &schur_prec_f32;
  pc.apply_f64 = &schur_prec_f64;
  auto u = [](const void* p) { return uint64_t(reinterpret_cast<uintptr_t>(p)); };
  pc.key = {u(S.arena.p), u(S.pmeta.p), uint64_t(S.p_tiles), uint64_t(nrhs), u(S.meta.p), uint64_t(S.nb), 0, 0};
  hgl_cg_opts co{};
  co.mode = HGL_CG_F32_F64DOT_RR;
  co.tol = refine_tol;
  co.max_iter = max_refine;
  co.x0_given = 0;
  co.rr_period = 0;
  co.chunk = chunk;
  const double lams[1] = {lambda};
  const int st = cg_run(h, lams, &co, Y, ldy, F, ldf, nrhs, iters_host, relres_host, &pc, s);
  HGL_HIP(hipStreamSynchronize(s));
  return st;
}
