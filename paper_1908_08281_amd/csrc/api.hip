// Handle lifecycle, hypergraph build (section 2 of the paper: incidence,
// degrees, scales) and validation.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "common.h"

namespace hgl {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
void clear_error() { g_err[0] = 0; }

int Mem::alloc(void** p, size_t bytes) {
  *p = nullptr;
  bytes = std::max<size_t>(bytes, 256);
  if (al.alloc) {
    *p = al.alloc(bytes, al.ctx, stream);
    if (!*p) {
      set_error("the caller's allocator returned NULL for %zu bytes", bytes);
      return HGL_ENOMEM;
    }
    return HGL_OK;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    set_error("hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    return HGL_ENOMEM;
  }
  return HGL_OK;
}

void Mem::release(void* p) {
  if (!p) return;
  if (al.alloc) {
    if (al.free) al.free(p, al.ctx, stream);
  } else {
    (void)hipFree(p);
  }
}

static int raw_alloc(void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    set_error("hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    return HGL_ENOMEM;
  }
  return HGL_OK;
}

int DevBuf::reserve(size_t n) {
  if (n <= bytes) return HGL_OK;
  release();
  size_t want = std::max<size_t>(n, 256);
  int rc = mem ? mem->alloc(&p, want) : raw_alloc(&p, want);
  if (rc < 0) {
    p = nullptr;
    return rc;
  }
  bytes = want;
  return HGL_OK;
}

void DevBuf::release() {
  if (p) {
    if (mem) mem->release(p);
    else (void)hipFree(p);
  }
  p = nullptr;
  bytes = 0;
}

template <class T>
static int dev_alloc(hgl_handle* h, T** p, size_t count) {
  void* q = nullptr;
  const int rc = h->mem.alloc(&q, std::max<size_t>(count * sizeof(T), 4));
  *p = static_cast<T*>(q);
  return rc;
}

int ensure_pinned(hgl_handle* h, size_t n) {
  if (!h->pinned_i) HGL_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->pinned_i), 64 * sizeof(int32_t)));
  if (n > h->pinned_d_len) {
    if (h->pinned_d) (void)hipHostFree(h->pinned_d);
    h->pinned_d = nullptr;
    h->pinned_d_len = 0;
    HGL_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->pinned_d), n * sizeof(double)));
    h->pinned_d_len = n;
  }
  return HGL_OK;
}

// ------------------------------------------------------------ kernel timing --

hipEvent_t prof_event(hgl_handle* h) {
  if (!h->prof_pool.empty()) {
    hipEvent_t e = h->prof_pool.back();
    h->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void prof_begin(hgl_handle* h, int kind, hipStream_t) {
  if (h->prof_on) h->prof_kind = kind;
}

void prof_end(hgl_handle* h, hipStream_t) { h->prof_kind = -1; }

static void prof_collect(hgl_handle* h) {
  if (h->prof_pending.empty()) return;
  (void)hipDeviceSynchronize();
  for (auto& p : h->prof_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
      h->prof_ms[p.first] += ms;
      h->prof_launches[p.first] += 1;
    }
    h->prof_pool.push_back(p.second.first);
    h->prof_pool.push_back(p.second.second);
  }
  h->prof_pending.clear();
}

static bool aligned(const void* p, int bytes) {
  return (reinterpret_cast<uintptr_t>(p) % bytes) == 0;
}

ColShape pick_shape(int k, int elem_bytes, std::initializer_list<const void*> ptrs,
                    std::initializer_list<int64_t> lds) {
  ColShape cs;
  int vmax = elem_bytes == 4 ? 4 : 2;  // 16-byte vector loads at most
  int V = vmax;
  while (V > 1) {
    bool ok = (k % V) == 0;
    for (int64_t ld : lds) ok = ok && (ld % V) == 0;
    for (const void* p : ptrs) ok = ok && (p == nullptr || aligned(p, V * elem_bytes));
    if (ok) break;
    V >>= 1;
  }
  int ncv = (k + V - 1) / V;
  int GL = 4;
  while (GL < ncv && GL < 64) GL <<= 1;
  cs.GL = GL;
  cs.V = V;
  cs.slabs = (k + cs.width() - 1) / cs.width();
  return cs;
}

// ---------------------------------------------------------------- kernels --

enum : int { kErrEmpty = 1, kErrRange = 2, kErrOrder = 4, kErrWeight = 8, kErrPtr = 16 };

__global__ void k_validate(int32_t E, int64_t nnz, const int32_t* __restrict__ edge_ptr,
                           const int32_t* __restrict__ edge_vtx, const double* __restrict__ w,
                           const int32_t* __restrict__ vtx_off, const int32_t* __restrict__ edge_off,
                           int32_t G, int32_t* __restrict__ err) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0 && (edge_ptr[0] != 0 || int64_t(edge_ptr[E]) != nnz)) {
    atomicOr(&err[0], kErrPtr);
    atomicMin(&err[1], 0);
  }
  if (e >= E) return;
  int code = 0;
  double we = w[e];
  if (!(we >= 0.0) || !isfinite(we)) code |= kErrWeight;
  int64_t b = edge_ptr[e], en = edge_ptr[e + 1];
  if (b < 0 || en > nnz || en < b) {
    code |= kErrPtr;
  } else if (en == b) {
    code |= kErrEmpty;
  } else {
    // graph of this edge: largest g with edge_off[g] <= e
    int lo = 0, hi = G - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (edge_off[mid] <= e) lo = mid; else hi = mid - 1;
    }
    int32_t v0 = vtx_off[lo], v1 = vtx_off[lo + 1];
    int32_t prev = -1;
    for (int64_t j = b; j < en; ++j) {
      int32_t v = edge_vtx[j];
      if (v < v0 || v >= v1) code |= kErrRange;
      if (j > b && v <= prev) code |= kErrOrder;
      prev = v;
    }
  }
  if (code) {
    atomicOr(&err[0], code);
    atomicMin(&err[1], e);
  }
}

__global__ void k_validate_w(int32_t E, const double* __restrict__ w, int32_t* __restrict__ err) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double we = w[e];
  if (!(we >= 0.0) || !isfinite(we)) {
    atomicOr(&err[0], kErrWeight);
    atomicMin(&err[1], e);
  }
}

// ------------------------------------------------------ exclusive scans --
// out[i] = sum_{j < i} in[i] for int32 arrays (in place allowed): each
// workgroup scans a tile of kScanTile entries (kScanItems consecutive
// entries per thread, then a wave prefix and a prefix over the waves) and
// writes its total; one workgroup scans the tile totals; a last pass adds
// each tile's offset.  Integer sums: exact, so the result does not depend
// on the order.
constexpr int kScanThreads = 256, kScanItems = 8, kScanTile = kScanThreads * kScanItems;

// Exclusive prefix of v over the workgroup's threads; the workgroup total in
// *total.  Every thread must call it.
__device__ __forceinline__ int32_t block_exclusive(int32_t v, int32_t* lds /* [kScanThreads / kWave] */,
                                                   int32_t* total) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  int32_t x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int32_t y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  if (lane == kWave - 1) lds[wave] = x;
  __syncthreads();
  int32_t before = 0, tot = 0;
  for (int w = 0; w < kScanThreads / kWave; ++w) {
    const int32_t t = lds[w];
    if (w < wave) before += t;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return before + x - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const int32_t* in, int32_t* out, int64_t n,
                                                             int32_t* __restrict__ tile_sums) {
  __shared__ int32_t lds[kScanThreads / kWave];
  const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  int32_t x[kScanItems];
  int32_t sum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    x[i] = base + i < n ? in[base + i] : 0;
    sum += x[i];
  }
  int32_t total = 0;
  int32_t run = block_exclusive(sum, lds, &total);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += x[i];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the tile totals in place, tile by tile
// with a carry.
__global__ __launch_bounds__(kScanThreads) void k_scan_top(int32_t* __restrict__ sums, int64_t nt) {
  __shared__ int32_t lds[kScanThreads / kWave];
  int32_t carry = 0;
  for (int64_t b0 = 0; b0 < nt; b0 += kScanTile) {
    const int64_t base = b0 + int64_t(threadIdx.x) * kScanItems;
    int32_t x[kScanItems];
    int32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      x[i] = base + i < nt ? sums[base + i] : 0;
      sum += x[i];
    }
    int32_t total = 0;
    int32_t run = carry + block_exclusive(sum, lds, &total);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      if (base + i < nt) sums[base + i] = run;
      run += x[i];
    }
    carry += total;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int32_t* __restrict__ out, int64_t n,
                                                           const int32_t* __restrict__ tile_off) {
  const int32_t add = tile_off[blockIdx.x];
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  for (int i = threadIdx.x; i < kScanTile; i += kScanThreads)
    if (base + i < n) out[base + i] += add;
}

// ------------------------------------------------ vertex-major transpose --

// deg[v] += 1 for every incidence (v, e).
__global__ void k_degree_count(int32_t E, const int32_t* __restrict__ edge_ptr,
                               const int32_t* __restrict__ edge_vtx, int32_t* __restrict__ deg) {
  const int e = blockIdx.x * (blockDim.x / 16) + threadIdx.x / 16;
  const int lane = threadIdx.x % 16;
  if (e >= E) return;
  for (int j = edge_ptr[e] + lane; j < edge_ptr[e + 1]; j += 16) atomicAdd(&deg[edge_vtx[j]], 1);
}

// Every incidence (v, e) goes to a free place of vertex v's segment
// [vtx_ptr[v], vtx_ptr[v+1]) of tmp (row[] records v there); the order
// inside a segment is whatever the atomics give (the ranking pass below
// fixes it).
__global__ void k_scatter_edges(int32_t E, const int32_t* __restrict__ edge_ptr,
                                const int32_t* __restrict__ edge_vtx, const int32_t* __restrict__ vtx_ptr,
                                int32_t* __restrict__ cursor, int32_t* __restrict__ tmp, int32_t* __restrict__ row) {
  const int e = blockIdx.x * (blockDim.x / 16) + threadIdx.x / 16;
  const int lane = threadIdx.x % 16;
  if (e >= E) return;
  for (int j = edge_ptr[e] + lane; j < edge_ptr[e + 1]; j += 16) {
    const int32_t v = edge_vtx[j];
    const int32_t pos = vtx_ptr[v] + atomicAdd(&cursor[v], 1);
    tmp[pos] = e;
    row[pos] = v;
  }
}

// The hyperedges of a vertex are distinct, so an entry's place in the sorted
// segment is the number of smaller entries in it: one thread per entry
// counts over its row's segment (the lanes of a wave mostly share a row, so
// their reads of the segment coincide).
__global__ __launch_bounds__(256) void k_rank(int64_t nnz, const int32_t* __restrict__ vtx_ptr,
                                              const int32_t* __restrict__ tmp, const int32_t* __restrict__ row,
                                              int32_t* __restrict__ vtx_edge) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const int32_t v = row[i];
  const int32_t b = vtx_ptr[v], en = vtx_ptr[v + 1];
  const int32_t x = tmp[i];
  int32_t r = 0;
  for (int32_t j = b; j < en; ++j) r += tmp[j] < x ? 1 : 0;
  vtx_edge[b + r] = x;
}

// dv[v] = sum of w_e over the hyperedges of v (the vertex degree of eq. 1),
// one wave per vertex: lane l takes entries l, l+64, ... with four loads in
// flight, then a fixed xor-shuffle tree (deterministic).  s = dv^-1/2, and 0
// for an isolated vertex (dv = 0).
__global__ __launch_bounds__(256) void k_degrees(int32_t N, const int32_t* __restrict__ vtx_ptr,
                                                 const int32_t* __restrict__ vtx_edge, const double* __restrict__ w,
                                                 double* __restrict__ dv, double* __restrict__ s64,
                                                 float* __restrict__ s32) {
  const int v = blockIdx.x * 4 + threadIdx.x / 64, lane = threadIdx.x % 64;
  if (v >= N) return;  // uniform per wave
  const int en = vtx_ptr[v + 1];
  double d = 0.0;
  int j = vtx_ptr[v] + lane;
  for (; j + 3 * 64 < en; j += 4 * 64) {
    const double w0 = w[vtx_edge[j]], w1 = w[vtx_edge[j + 64]];
    const double w2 = w[vtx_edge[j + 128]], w3 = w[vtx_edge[j + 192]];
    d += ((w0 + w1) + w2) + w3;
  }
  for (; j < en; j += 64) d += w[vtx_edge[j]];
  for (int off = 32; off >= 1; off >>= 1) d += __shfl_xor(d, off, 64);
  if (lane == 0) {
    dv[v] = d;
    const double sv = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    s64[v] = sv;
    s32[v] = float(sv);
  }
}

__global__ void k_edge_scales(int32_t E, const int32_t* __restrict__ edge_ptr,
                              const double* __restrict__ w, double* __restrict__ c64,
                              float* __restrict__ c32) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double c = w[e] / double(edge_ptr[e + 1] - edge_ptr[e]);
  c64[e] = c;
  c32[e] = float(c);
}

// Hub rows (more than kLongRow hyperedges) are split into chunks of at most
// kChunk.  A row of at least kBucketRow hyperedges is first cut where its
// (increasing) hyperedge ids cross into the next eighth of [0, E): every
// chunk then reads Z rows of one eighth only, and the chunk's workgroup is
// placed on the matching XCD (chunk_order), whose L2 so serves one eighth of
// Z.  Eighth x of [0, E) starts at ceil(x E / 8).
__device__ __forceinline__ int32_t eighth_start(int x, int32_t E) {
  return int32_t((int64_t(x) * E + kXcd - 1) / kXcd);
}

// First position in [b, en) whose hyperedge id is >= e (ids increase).
__device__ __forceinline__ int32_t lower_pos(const int32_t* __restrict__ ids, int32_t b, int32_t en, int32_t e) {
  while (b < en) {
    const int32_t m = b + (en - b) / 2;
    if (ids[m] < e) b = m + 1;
    else en = m;
  }
  return b;
}

__global__ void k_long_flags(int32_t N, int32_t E, const int32_t* __restrict__ vtx_ptr,
                             const int32_t* __restrict__ vtx_edge, int32_t* __restrict__ is_long,
                             int32_t* __restrict__ nch) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const int32_t b = vtx_ptr[v], en = vtx_ptr[v + 1], d = en - b;
  const bool L = d > kLongRow;
  is_long[v] = L ? 1 : 0;
  int n = 0;
  if (L && d >= kBucketRow) {
    int32_t p0 = b;
    for (int x = 0; x < kXcd; ++x) {
      const int32_t p1 = x + 1 < kXcd ? lower_pos(vtx_edge, p0, en, eighth_start(x + 1, E)) : en;
      n += (p1 - p0 + kChunk - 1) / kChunk;
      p0 = p1;
    }
  } else if (L) {
    n = (d + kChunk - 1) / kChunk;
  }
  nch[v] = n;
}

// chunk_eighth[c]: the eighth of [0, E) whose Z rows chunk c reads, or -1
// (a row below kBucketRow: any XCD).
__global__ void k_long_fill(int32_t N, int32_t E, const int32_t* __restrict__ vtx_ptr,
                            const int32_t* __restrict__ vtx_edge, const int32_t* __restrict__ is_long,
                            const int32_t* __restrict__ slot_of, const int32_t* __restrict__ chunk_of,
                            int32_t* __restrict__ long_row, int32_t* __restrict__ long_chunk0,
                            int32_t* __restrict__ chunk_slot, int32_t* __restrict__ chunk_begin,
                            int32_t* __restrict__ chunk_end, int32_t* __restrict__ chunk_eighth) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N || !is_long[v]) return;
  int slot = slot_of[v];
  int c = chunk_of[v];
  long_row[slot] = v;
  long_chunk0[slot] = c;
  const int32_t b = vtx_ptr[v], en = vtx_ptr[v + 1];
  const bool bucketed = en - b >= kBucketRow;
  int32_t p0 = b;
  for (int x = 0; x < (bucketed ? kXcd : 1); ++x) {
    const int32_t p1 =
        bucketed && x + 1 < kXcd ? lower_pos(vtx_edge, p0, en, eighth_start(x + 1, E)) : en;
    for (int32_t j = p0; j < p1; j += kChunk, ++c) {
      chunk_slot[c] = slot;
      chunk_begin[c] = j;
      chunk_end[c] = min(j + kChunk, p1);
      chunk_eighth[c] = bucketed ? x : -1;
    }
    p0 = p1;
  }
}

__global__ void k_long_edge_flags(int32_t E, const int32_t* __restrict__ edge_ptr, int32_t* __restrict__ is_long) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  is_long[e] = edge_ptr[e + 1] - edge_ptr[e] > kLongEdge ? 1 : 0;
}

__global__ void k_long_edge_fill(int32_t E, const int32_t* __restrict__ is_long, const int32_t* __restrict__ slot_of,
                                 int32_t* __restrict__ long_edge) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < E && is_long[e]) long_edge[slot_of[e]] = e;
}

static int blocks_for(int64_t n, int per) { return int((n + per - 1) / per); }

static int check_error_words(const int32_t* err_host) {
  if (err_host[0] == 0) return HGL_OK;
  int c = err_host[0];
  set_error("invalid hypergraph (first bad hyperedge %d):%s%s%s%s%s", err_host[1],
            (c & kErrPtr) ? " edge_ptr not a valid CSR offset array;" : "",
            (c & kErrEmpty) ? " empty hyperedge;" : "",
            (c & kErrRange) ? " vertex id outside [0,N) (or outside its graph);" : "",
            (c & kErrOrder) ? " vertex ids not strictly increasing (repeated vertex);" : "",
            (c & kErrWeight) ? " weight negative or not finite;" : "");
  return HGL_EINVAL;
}

static int compute_scales(hgl_handle* h, hipStream_t s) {
  if (h->N > 0)
    hipLaunchKernelGGL(k_degrees, dim3(blocks_for(h->N, 4)), dim3(256), 0, s, h->N, h->vtx_ptr,
                       h->vtx_edge, h->w, h->dv, h->s64, h->s32);
  if (h->E > 0)
    hipLaunchKernelGGL(k_edge_scales, dim3(blocks_for(h->E, 256)), dim3(256), 0, s, h->E,
                       h->edge_ptr, h->w, h->c64, h->c32);
  HGL_HIP(hipGetLastError());
  return HGL_OK;
}

static void free_handle(hgl_handle* h) {
  if (!h) return;
  void* ptrs[] = {h->edge_ptr, h->edge_vtx, h->vtx_ptr, h->vtx_edge, h->w, h->dv, h->s64, h->c64,
                  h->s32, h->c32, h->tile_r0, h->tile_r1, h->tile_seg, h->long_row,
                  h->chunk_slot, h->chunk_begin, h->chunk_end, h->long_chunk0,
                  h->seg_slots, h->long_seg, h->long_edge, h->etile_e0, h->etile_e1, h->seg_eslots,
                  h->chunk_order};
  for (void* p : ptrs) h->mem.release(p);
  DevBuf* bufs[] = {&h->ws_z, &h->ws_z64, &h->ws_chunk, &h->ws_part, &h->ws_part2,
                    &h->ws_vec, &h->ws_state, &h->ws_misc};
  for (DevBuf* b : bufs) b->release();
  for (auto& b : h->ws_extra) b.release();
  h->ws_ab.release();
  h->wg_tab.release();
  if (h->rsvd_free) h->rsvd_free(h->rsvd_ws);
  if (h->schur_free) h->schur_free(h->schur_ws);
  if (h->cg_graph) (void)hipGraphExecDestroy(h->cg_graph);
  if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
  if (h->pinned_i) (void)hipHostFree(h->pinned_i);
  if (h->pinned_d) (void)hipHostFree(h->pinned_d);
  for (auto& p : h->prof_pending) {
    (void)hipEventDestroy(p.second.first);
    (void)hipEventDestroy(p.second.second);
  }
  for (hipEvent_t e : h->prof_pool) (void)hipEventDestroy(e);
  delete h;
}

// Temporaries of one build, taken from the handle's memory source and
// returned in one place (before the handle itself on failure).
struct Temps {
  hgl_handle* h;
  std::vector<void*> ps;
  template <class T>
  int get(T** p, size_t count) {
    void* q = nullptr;
    const int rc = h->mem.alloc(&q, std::max<size_t>(count * sizeof(T), 4));
    *p = static_cast<T*>(q);
    if (rc == HGL_OK) ps.push_back(q);
    return rc;
  }
  void release() {
    for (void* q : ps) h->mem.release(q);
    ps.clear();
  }
};

// out[0 .. n-1] = exclusive prefix sums of in[0 .. n-1] (in place allowed).
static int scan_exclusive(Temps& tmp, const int32_t* in, int32_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return HGL_OK;
  const int64_t nt = (n + kScanTile - 1) / kScanTile;
  int32_t* sums = nullptr;
  HGL_TRY(tmp.get(&sums, size_t(nt)));
  hipLaunchKernelGGL(k_scan_tiles, dim3(unsigned(nt)), dim3(kScanThreads), 0, s, in, out, n, sums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, sums, nt);
  hipLaunchKernelGGL(k_scan_add, dim3(unsigned(nt)), dim3(kScanThreads), 0, s, out, n,
                     static_cast<const int32_t*>(sums));
  HGL_HIP(hipGetLastError());
  return HGL_OK;
}

static void attach_all(hgl_handle* h) {
  attach(h, h->ws_z, h->ws_z64, h->ws_chunk, h->ws_part, h->ws_part2, h->ws_vec, h->ws_state, h->ws_misc,
         h->ws_ab, h->wg_tab);
  for (auto& b : h->ws_extra) b.mem = &h->mem;
}

static int build(int32_t G, const int32_t* vtx_off_host, const int32_t* edge_off_host, int64_t nnz,
                 const int32_t* edge_ptr, const int32_t* edge_vtx, const double* w, const hgl_allocator* al,
                 hgl_handle** out, hipStream_t s) {
  HGL_CHECK_ARG(out != nullptr, "out must not be NULL");
  *out = nullptr;
  HGL_CHECK_ARG(G >= 1, "number of graphs must be >= 1 (got %d)", G);
  HGL_CHECK_ARG(vtx_off_host && edge_off_host, "offset arrays must not be NULL");
  HGL_CHECK_ARG(vtx_off_host[0] == 0 && edge_off_host[0] == 0, "offsets must start at 0");
  for (int g = 0; g < G; ++g) {
    HGL_CHECK_ARG(vtx_off_host[g + 1] >= vtx_off_host[g] && edge_off_host[g + 1] >= edge_off_host[g],
                  "offsets must be non-decreasing (graph %d)", g);
  }
  int32_t N = vtx_off_host[G], E = edge_off_host[G];
  HGL_CHECK_ARG(N >= 1, "N must be >= 1");
  HGL_CHECK_ARG(E >= 0 && nnz >= 0 && nnz < (int64_t(1) << 31), "E, nnz out of range");
  HGL_CHECK_ARG(E == 0 || (edge_ptr && edge_vtx && w), "edge_ptr, edge_vtx, w must not be NULL");
  HGL_CHECK_ARG(nnz >= E, "nnz (%lld) < E (%d): some hyperedge would be empty", (long long)nnz, E);
  HGL_CHECK_ARG(!al || al->alloc, "an allocator must have an alloc function");

  hgl_handle* h = new hgl_handle();
  if (al) h->mem.al = *al;
  h->mem.stream = s;
  attach_all(h);
  h->N = N;
  h->E = E;
  h->G = G;
  h->nnz = nnz;
  (void)hipGetDevice(&h->device);
  h->vtx_off.assign(vtx_off_host, vtx_off_host + G + 1);
  h->edge_off.assign(edge_off_host, edge_off_host + G + 1);
  Temps tmp{h, {}};

  auto fail = [&](int code) {
    (void)hipStreamSynchronize(s);  // queued work may still use the temporaries
    tmp.release();
    free_handle(h);
    return code;
  };
#define B_TRY(expr)              \
  do {                           \
    int _s = (expr);             \
    if (_s < 0) return fail(_s); \
  } while (0)
#define B_HIP(call)                                                                   \
  do {                                                                                \
    hipError_t _e = (call);                                                           \
    if (_e != hipSuccess) {                                                           \
      set_error("%s failed: %s", #call, hipGetErrorString(_e));                       \
      return fail(HGL_EDEVICE);                                                       \
    }                                                                                 \
  } while (0)

  B_TRY(dev_alloc(h, &h->edge_ptr, E + 1));
  B_TRY(dev_alloc(h, &h->edge_vtx, nnz));
  B_TRY(dev_alloc(h, &h->vtx_ptr, N + 1));
  B_TRY(dev_alloc(h, &h->vtx_edge, nnz));
  B_TRY(dev_alloc(h, &h->w, E));
  B_TRY(dev_alloc(h, &h->dv, N));
  B_TRY(dev_alloc(h, &h->s64, N));
  B_TRY(dev_alloc(h, &h->c64, E));
  B_TRY(dev_alloc(h, &h->s32, N));
  B_TRY(dev_alloc(h, &h->c32, E));
  B_TRY(ensure_pinned(h, 64));

  if (E > 0) {
    B_HIP(hipMemcpyAsync(h->edge_ptr, edge_ptr, sizeof(int32_t) * (E + 1), hipMemcpyDeviceToDevice, s));
    if (nnz > 0)
      B_HIP(hipMemcpyAsync(h->edge_vtx, edge_vtx, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, s));
    B_HIP(hipMemcpyAsync(h->w, w, sizeof(double) * E, hipMemcpyDeviceToDevice, s));
  } else {
    B_HIP(hipMemsetAsync(h->edge_ptr, 0, sizeof(int32_t), s));
  }

  // ---- validation (device), before any use of the indices
  {
    int32_t* d_off = nullptr;
    B_TRY(tmp.get(&d_off, 2 * size_t(G) + 4));
    int32_t* d_err = d_off + 2 * G + 2;
    // offsets and the error words' start values, staged in one host vector
    // (the stream is synchronised before it goes out of scope)
    std::vector<int32_t> hv(2 * size_t(G) + 4);
    std::copy(vtx_off_host, vtx_off_host + G + 1, hv.begin());
    std::copy(edge_off_host, edge_off_host + G + 1, hv.begin() + G + 1);
    hv[2 * G + 2] = 0;
    hv[2 * G + 3] = 0x7fffffff;
    B_HIP(hipMemcpyAsync(d_off, hv.data(), sizeof(int32_t) * hv.size(), hipMemcpyHostToDevice, s));
    if (E > 0)
      hipLaunchKernelGGL(k_validate, dim3(blocks_for(E, 256)), dim3(256), 0, s, E, nnz, h->edge_ptr,
                         h->edge_vtx, h->w, d_off, d_off + G + 1, G, d_err);
    B_HIP(hipGetLastError());
    B_HIP(hipMemcpyAsync(h->pinned_i, d_err, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    B_HIP(hipStreamSynchronize(s));  // hv goes out of scope; the error words are read
    int st = check_error_words(h->pinned_i);
    if (st < 0) return fail(st);
  }

  // ---- vertex-major transpose: degree counts -> offsets (scan) -> each
  // incidence scattered into its vertex's segment -> each segment put in
  // increasing hyperedge order by ranking
  std::vector<int32_t> chunk_eighth_host;
  {
    int32_t* deg = nullptr;    // [N+1] degree, then the scatter cursor
    int32_t* etmp = nullptr;   // [nnz] scattered hyperedge ids
    int32_t* erow = nullptr;   // [nnz] their vertex
    B_TRY(tmp.get(&deg, size_t(N) + 1));
    B_TRY(tmp.get(&etmp, size_t(std::max<int64_t>(nnz, 1))));
    B_TRY(tmp.get(&erow, size_t(std::max<int64_t>(nnz, 1))));
    B_HIP(hipMemsetAsync(deg, 0, sizeof(int32_t) * (size_t(N) + 1), s));
    if (E > 0)
      hipLaunchKernelGGL(k_degree_count, dim3(blocks_for(E, 16)), dim3(256), 0, s, E, h->edge_ptr, h->edge_vtx,
                         deg);
    B_HIP(hipGetLastError());
    B_TRY(scan_exclusive(tmp, deg, h->vtx_ptr, int64_t(N) + 1, s));
    if (nnz > 0) {
      B_HIP(hipMemsetAsync(deg, 0, sizeof(int32_t) * (size_t(N) + 1), s));
      hipLaunchKernelGGL(k_scatter_edges, dim3(blocks_for(E, 16)), dim3(256), 0, s, E, h->edge_ptr, h->edge_vtx,
                         h->vtx_ptr, deg, etmp, erow);
      hipLaunchKernelGGL(k_rank, dim3(blocks_for(nnz, 256)), dim3(256), 0, s, nnz, h->vtx_ptr,
                         static_cast<const int32_t*>(etmp), static_cast<const int32_t*>(erow), h->vtx_edge);
      B_HIP(hipGetLastError());
    }
  }

  // ---- hub rows -> chunks (the large ones cut by eighth of [0, E))
  {
    int32_t* tmpi = nullptr;
    B_TRY(tmp.get(&tmpi, 4 * (size_t(N) + 1)));
    int32_t* is_long = tmpi;
    int32_t* nch = tmpi + (N + 1);
    int32_t* slot_of = tmpi + 2 * (N + 1);
    int32_t* chunk_of = tmpi + 3 * (N + 1);
    B_HIP(hipMemsetAsync(tmpi, 0, sizeof(int32_t) * 4 * (size_t(N) + 1), s));
    hipLaunchKernelGGL(k_long_flags, dim3(blocks_for(N, 256)), dim3(256), 0, s, N, E, h->vtx_ptr, h->vtx_edge,
                       is_long, nch);
    B_HIP(hipGetLastError());
    B_TRY(scan_exclusive(tmp, is_long, slot_of, int64_t(N) + 1, s));
    B_TRY(scan_exclusive(tmp, nch, chunk_of, int64_t(N) + 1, s));
    B_HIP(hipMemcpyAsync(h->pinned_i, slot_of + N, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    B_HIP(hipMemcpyAsync(h->pinned_i + 1, chunk_of + N, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    B_HIP(hipStreamSynchronize(s));
    h->n_long = h->pinned_i[0];
    h->n_chunks = h->pinned_i[1];
    int32_t* chunk_eighth = nullptr;
    B_TRY(tmp.get(&chunk_eighth, size_t(h->n_chunks) + 1));
    B_TRY(dev_alloc(h, &h->long_row, h->n_long));
    B_TRY(dev_alloc(h, &h->long_chunk0, h->n_long + 1));
    B_TRY(dev_alloc(h, &h->chunk_slot, h->n_chunks));
    B_TRY(dev_alloc(h, &h->chunk_begin, h->n_chunks));
    B_TRY(dev_alloc(h, &h->chunk_end, h->n_chunks));
    hipLaunchKernelGGL(k_long_fill, dim3(blocks_for(N, 256)), dim3(256), 0, s, N, E, h->vtx_ptr, h->vtx_edge,
                       is_long, slot_of, chunk_of, h->long_row, h->long_chunk0, h->chunk_slot, h->chunk_begin,
                       h->chunk_end, chunk_eighth);
    B_HIP(hipGetLastError());
    h->pinned_i[2] = h->n_chunks;
    B_HIP(hipMemcpyAsync(h->long_chunk0 + h->n_long, h->pinned_i + 2, sizeof(int32_t),
                         hipMemcpyHostToDevice, s));
    // per-graph slot ranges: long rows are listed in increasing vertex id, so
    // each graph's long rows are contiguous
    std::vector<int32_t> lr(h->n_long);
    chunk_eighth_host.assign(h->n_chunks, -1);
    if (h->n_long)
      B_HIP(hipMemcpyAsync(lr.data(), h->long_row, 4 * size_t(h->n_long), hipMemcpyDeviceToHost, s));
    if (h->n_chunks)
      B_HIP(hipMemcpyAsync(chunk_eighth_host.data(), chunk_eighth, 4 * size_t(h->n_chunks),
                           hipMemcpyDeviceToHost, s));
    B_HIP(hipStreamSynchronize(s));
    h->seg_slots_host.assign(4 * G, 0);
    int t = 0, l = 0;
    std::vector<int32_t> lseg(h->n_long);
    for (int g = 0; g < G; ++g) {
      // tiles are generated graph by graph, so graph g owns a contiguous range
      int t0 = t;
      t += (vtx_off_host[g + 1] - vtx_off_host[g] + kTileRows - 1) / kTileRows;
      int l0 = l;
      while (l < h->n_long && lr[l] < vtx_off_host[g + 1]) lseg[l++] = g;
      h->seg_slots_host[4 * g + 0] = t0;
      h->seg_slots_host[4 * g + 1] = t;
      h->seg_slots_host[4 * g + 2] = l0;
      h->seg_slots_host[4 * g + 3] = l;
    }
    B_TRY(dev_alloc(h, &h->long_seg, h->n_long));
    if (h->n_long)
      B_HIP(hipMemcpyAsync(h->long_seg, lseg.data(), 4 * size_t(h->n_long), hipMemcpyHostToDevice, s));
    B_HIP(hipStreamSynchronize(s));
  }
  B_TRY(compute_scales(h, s));

  // ---- row tiles (segment-aligned) for the row-streaming kernels
  {
    std::vector<int32_t> r0, r1, sg;
    for (int g = 0; g < G; ++g)
      for (int32_t r = vtx_off_host[g]; r < vtx_off_host[g + 1]; r += kTileRows) {
        r0.push_back(r);
        r1.push_back(std::min(r + kTileRows, vtx_off_host[g + 1]));
        sg.push_back(g);
      }
    h->n_tiles = int32_t(r0.size());
    for (int g = 0; g < G; ++g) {
      h->seg_slots_host[4 * g + 2] += h->n_tiles;
      h->seg_slots_host[4 * g + 3] += h->n_tiles;
    }
    B_TRY(dev_alloc(h, &h->tile_r0, r0.size()));
    B_TRY(dev_alloc(h, &h->tile_r1, r0.size()));
    B_TRY(dev_alloc(h, &h->tile_seg, r0.size()));
    B_TRY(dev_alloc(h, &h->seg_slots, 4 * G));
    B_HIP(hipMemcpyAsync(h->tile_r0, r0.data(), 4 * r0.size(), hipMemcpyHostToDevice, s));
    B_HIP(hipMemcpyAsync(h->tile_r1, r1.data(), 4 * r1.size(), hipMemcpyHostToDevice, s));
    B_HIP(hipMemcpyAsync(h->tile_seg, sg.data(), 4 * sg.size(), hipMemcpyHostToDevice, s));
    B_HIP(hipMemcpyAsync(h->seg_slots, h->seg_slots_host.data(), 16 * size_t(G), hipMemcpyHostToDevice, s));
    B_HIP(hipStreamSynchronize(s));  // host vectors go out of scope
  }

  // ---- dispatch order of the chunk workgroups: workgroup n_tiles + j runs
  // on XCD (n_tiles + j) mod kXcd; a chunk that reads one eighth of Z goes to
  // that eighth's XCD while such chunks remain, the rest fill in where their
  // own list is empty.  Padding to a multiple of kXcd keeps the placement for
  // every column slab of the grid.
  {
    std::vector<std::vector<int32_t>> lists(kXcd + 1);
    for (int32_t c = 0; c < h->n_chunks; ++c) {
      const int x = chunk_eighth_host[c];
      lists[x >= 0 ? x : kXcd].push_back(c);
    }
    std::vector<size_t> at(kXcd + 1, 0);
    std::vector<int32_t> order;
    order.reserve(h->n_chunks + 2 * kXcd);
    auto left = [&](int x) { return lists[x].size() - at[x]; };
    int32_t placed = 0;
    while (placed < h->n_chunks) {
      const int xcd = int((int64_t(h->n_tiles) + int64_t(order.size())) % kXcd);
      int from = -1;
      if (left(xcd) > 0) {
        from = xcd;
      } else if (left(kXcd) > 0) {
        from = kXcd;  // a chunk with no eighth of its own
      } else {
        for (int x = 0; x < kXcd; ++x)
          if (left(x) > 0 && (from < 0 || left(x) > left(from))) from = x;
      }
      order.push_back(lists[from][at[from]++]);
      ++placed;
    }
    while ((int64_t(h->n_tiles) + int64_t(order.size())) % kXcd != 0) order.push_back(-1);
    h->n_dispatch = int32_t(order.size());
    B_TRY(dev_alloc(h, &h->chunk_order, order.size()));
    if (!order.empty())
      B_HIP(hipMemcpyAsync(h->chunk_order, order.data(), 4 * order.size(), hipMemcpyHostToDevice, s));
    B_HIP(hipStreamSynchronize(s));
  }

  // ---- long hyperedges (one workgroup each in the edge gather)
  if (E > 0) {
    int32_t* tmpi = nullptr;
    B_TRY(tmp.get(&tmpi, 2 * (size_t(E) + 1)));
    int32_t* is_long = tmpi;
    int32_t* slot_of = tmpi + (E + 1);
    B_HIP(hipMemsetAsync(tmpi, 0, sizeof(int32_t) * 2 * (size_t(E) + 1), s));
    hipLaunchKernelGGL(k_long_edge_flags, dim3(blocks_for(E, 256)), dim3(256), 0, s, E, h->edge_ptr, is_long);
    B_HIP(hipGetLastError());
    B_TRY(scan_exclusive(tmp, is_long, slot_of, int64_t(E) + 1, s));
    B_HIP(hipMemcpyAsync(h->pinned_i, slot_of + E, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    B_HIP(hipStreamSynchronize(s));
    h->n_long_edge = h->pinned_i[0];
    B_TRY(dev_alloc(h, &h->long_edge, h->n_long_edge));
    hipLaunchKernelGGL(k_long_edge_fill, dim3(blocks_for(E, 256)), dim3(256), 0, s, E, is_long, slot_of,
                       h->long_edge);
    B_HIP(hipGetLastError());
  }
  // ---- edge tiles (graph-aligned) of the edge gather, and per graph the
  // slot ranges of its partial sums: tiles, then long hyperedges (listed in
  // increasing id, so each graph's are contiguous)
  {
    std::vector<int32_t> e0, e1;
    for (int g = 0; g < G; ++g)
      for (int32_t e = edge_off_host[g]; e < edge_off_host[g + 1]; e += kEdgeTile) {
        e0.push_back(e);
        e1.push_back(std::min(e + kEdgeTile, edge_off_host[g + 1]));
      }
    h->n_etiles = int32_t(e0.size());
    B_TRY(dev_alloc(h, &h->etile_e0, e0.size()));
    B_TRY(dev_alloc(h, &h->etile_e1, e1.size()));
    if (!e0.empty()) {
      B_HIP(hipMemcpyAsync(h->etile_e0, e0.data(), 4 * e0.size(), hipMemcpyHostToDevice, s));
      B_HIP(hipMemcpyAsync(h->etile_e1, e1.data(), 4 * e1.size(), hipMemcpyHostToDevice, s));
    }
    std::vector<int32_t> le(h->n_long_edge);
    if (h->n_long_edge)
      B_HIP(hipMemcpyAsync(le.data(), h->long_edge, 4 * size_t(h->n_long_edge), hipMemcpyDeviceToHost, s));
    B_HIP(hipStreamSynchronize(s));
    h->seg_eslots_host.assign(4 * G, 0);
    int t = 0, l = 0;
    for (int g = 0; g < G; ++g) {
      const int t0 = t, l0 = l;
      t += (edge_off_host[g + 1] - edge_off_host[g] + kEdgeTile - 1) / kEdgeTile;
      while (l < h->n_long_edge && le[l] < edge_off_host[g + 1]) ++l;
      h->seg_eslots_host[4 * g + 0] = t0;
      h->seg_eslots_host[4 * g + 1] = t;
      h->seg_eslots_host[4 * g + 2] = h->n_etiles + l0;
      h->seg_eslots_host[4 * g + 3] = h->n_etiles + l;
    }
    B_TRY(dev_alloc(h, &h->seg_eslots, 4 * G));
    B_HIP(hipMemcpyAsync(h->seg_eslots, h->seg_eslots_host.data(), 16 * size_t(G), hipMemcpyHostToDevice, s));
  }
  B_HIP(hipStreamSynchronize(s));
  tmp.release();
#undef B_TRY
#undef B_HIP
  *out = h;
  return HGL_OK;
}

}  // namespace hgl

using namespace hgl;

extern "C" int hgl_version(void) { return 100; }

extern "C" const char* hgl_last_error(void) { return g_err; }

extern "C" int hgl_build_laplacian(int32_t N, int32_t E, int64_t nnz, const int32_t* edge_ptr,
                                   const int32_t* edge_vtx, const double* w, const hgl_allocator* al,
                                   hgl_handle** out, hipStream_t stream) {
  clear_error();
  int32_t vo[2] = {0, N}, eo[2] = {0, E};
  HGL_CHECK_ARG(N >= 1 && E >= 0, "need N >= 1 and E >= 0 (got N=%d, E=%d)", N, E);
  return build(1, vo, eo, nnz, edge_ptr, edge_vtx, w, al, out, stream);
}

extern "C" int hgl_build_laplacian_batched(int32_t G, const int32_t* vtx_offsets_host,
                                           const int32_t* edge_offsets_host, int64_t nnz,
                                           const int32_t* edge_ptr, const int32_t* edge_vtx,
                                           const double* w, const hgl_allocator* al, hgl_handle** out,
                                           hipStream_t stream) {
  clear_error();
  return build(G, vtx_offsets_host, edge_offsets_host, nnz, edge_ptr, edge_vtx, w, al, out, stream);
}

extern "C" int hgl_set_weights(hgl_handle* h, const double* w, hipStream_t s) {
  clear_error();
  HGL_CHECK_ARG(h != nullptr, "handle is NULL");
  HGL_CHECK_ARG(h->E == 0 || w != nullptr, "w is NULL");
  enter(h, s);
  if (h->E == 0) return HGL_OK;
  // the error words live in the handle's small workspace
  HGL_TRY(h->ws_misc.reserve(64));
  int32_t* d_err = h->ws_misc.as<int32_t>();
  h->pinned_i[0] = 0;
  h->pinned_i[1] = 0x7fffffff;
  HGL_HIP(hipMemcpyAsync(d_err, h->pinned_i, 2 * sizeof(int32_t), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_validate_w, dim3(blocks_for(h->E, 256)), dim3(256), 0, s, h->E, w, d_err);
  HGL_HIP(hipGetLastError());
  HGL_HIP(hipMemcpyAsync(h->pinned_i + 2, d_err, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HGL_HIP(hipStreamSynchronize(s));
  HGL_TRY(check_error_words(h->pinned_i + 2));
  HGL_HIP(hipMemcpyAsync(h->w, w, sizeof(double) * h->E, hipMemcpyDeviceToDevice, s));
  return compute_scales(h, s);
}

extern "C" void hgl_destroy(hgl_handle* h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  free_handle(h);
}

extern "C" int hgl_get_sizes(const hgl_handle* h, int32_t* N, int32_t* E, int64_t* nnz, int32_t* G) {
  clear_error();
  HGL_CHECK_ARG(h != nullptr, "handle is NULL");
  if (N) *N = h->N;
  if (E) *E = h->E;
  if (nnz) *nnz = h->nnz;
  if (G) *G = h->G;
  return HGL_OK;
}

extern "C" int hgl_get_partition(const hgl_handle* h, int32_t* n_tiles, int32_t* n_hub_rows,
                                 int32_t* n_hub_chunks, int32_t* n_long_edges) {
  clear_error();
  HGL_CHECK_ARG(h != nullptr, "handle is NULL");
  if (n_tiles) *n_tiles = h->n_tiles;
  if (n_hub_rows) *n_hub_rows = h->n_long;
  if (n_hub_chunks) *n_hub_chunks = h->n_chunks;
  if (n_long_edges) *n_long_edges = h->n_long_edge;
  return HGL_OK;
}

extern "C" int hgl_get_gather_shape(const hgl_handle* h, int32_t* shape6) {
  clear_error();
  HGL_CHECK_ARG(h != nullptr, "handle is NULL");
  HGL_CHECK_ARG(shape6 != nullptr, "shape6 is NULL");
  for (int i = 0; i < 6; ++i) shape6[i] = h->last_shape[i];
  return HGL_OK;
}

extern "C" int hgl_get_cg_stats(const hgl_handle* h, int32_t* stats4) {
  clear_error();
  HGL_CHECK_ARG(h != nullptr, "handle is NULL");
  HGL_CHECK_ARG(stats4 != nullptr, "stats4 is NULL");
  for (int i = 0; i < 4; ++i) stats4[i] = h->last_cg[i];
  return HGL_OK;
}

extern "C" int hgl_profile(hgl_handle* h, int32_t enable) {
  clear_error();
  HGL_CHECK_ARG(h != nullptr, "handle is NULL");
  prof_collect(h);
  for (int i = 0; i < kProfKinds; ++i) {
    h->prof_launches[i] = 0;
    h->prof_ms[i] = 0.0;
  }
  h->prof_on = enable != 0;
  h->prof_mask = enable == 1 ? 0xffffffffu : (uint32_t(enable) & 0xffffu);
  h->prof_every = enable == 1 ? 1u : std::max(1u, (uint32_t(enable) >> 16) & 0xffu);
  for (int i = 0; i < kProfKinds; ++i) h->prof_count[i] = 0;
  return HGL_OK;
}

extern "C" int hgl_profile_read(hgl_handle* h, int32_t kind, int64_t* launches, double* ms) {
  clear_error();
  HGL_CHECK_ARG(h != nullptr, "handle is NULL");
  HGL_CHECK_ARG(kind >= 0 && kind < kProfKinds, "unknown kernel kind %d", kind);
  prof_collect(h);
  if (launches) *launches = h->prof_launches[kind];
  if (ms) *ms = h->prof_ms[kind];
  return HGL_OK;
}

extern "C" int hgl_get_operator(const hgl_handle* h, double* dv, double* s, double* c,
                                int32_t* vtx_ptr, int32_t* vtx_edge, hipStream_t st) {
  clear_error();
  HGL_CHECK_ARG(h != nullptr, "handle is NULL");
  auto D2D = hipMemcpyDeviceToDevice;
  if (dv) HGL_HIP(hipMemcpyAsync(dv, h->dv, sizeof(double) * h->N, D2D, st));
  if (s) HGL_HIP(hipMemcpyAsync(s, h->s64, sizeof(double) * h->N, D2D, st));
  if (c && h->E) HGL_HIP(hipMemcpyAsync(c, h->c64, sizeof(double) * h->E, D2D, st));
  if (vtx_ptr) HGL_HIP(hipMemcpyAsync(vtx_ptr, h->vtx_ptr, sizeof(int32_t) * (h->N + 1), D2D, st));
  if (vtx_edge && h->nnz) HGL_HIP(hipMemcpyAsync(vtx_edge, h->vtx_edge, sizeof(int32_t) * h->nnz, D2D, st));
  return HGL_OK;
}
