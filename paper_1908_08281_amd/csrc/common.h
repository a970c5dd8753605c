// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <tuple>
#include <type_traits>
#include <cstdio>
#include <string>
#include <vector>

#include "hgl.h"

namespace hgl {

// ---------------------------------------------------------------- errors --

void set_error(const char* fmt, ...);
void clear_error();

struct Status {
  int code = HGL_OK;
};

// Return on a HIP error with HGL_EDEVICE and the runtime's message.
#define HGL_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t _e = (call);                                                            \
    if (_e != hipSuccess) {                                                            \
      ::hgl::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(_e), __FILE__, \
                       __LINE__);                                                      \
      return HGL_EDEVICE;                                                              \
    }                                                                                  \
  } while (0)

#define HGL_CHECK_ARG(cond, ...)   \
  do {                             \
    if (!(cond)) {                 \
      ::hgl::set_error(__VA_ARGS__); \
      return HGL_EINVAL;           \
    }                              \
  } while (0)

#define HGL_TRY(...)              \
  do {                            \
    int _s = (__VA_ARGS__);       \
    if (_s < 0) return _s;        \
  } while (0)

// ------------------------------------------------------------- constants --

constexpr int kBlock = 256;        // threads per workgroup: 4 waves of 64
constexpr int kWave = 64;
constexpr int kTileRows = 32;      // rows per tile of the row-streaming kernels
constexpr int kLongRow = 32;       // vertex rows with more hyperedges are split
constexpr int kChunk = 128;        // hyperedges per chunk of a split vertex row
constexpr int kBucketRow = 256;    // hub rows with this many hyperedges are split by eighth of [0, E)
constexpr int kXcd = 8;            // XCDs of the device; workgroup w runs on XCD w mod 8
constexpr int kStageIdx = 2048;    // hyperedge ids of a tile staged in LDS
constexpr int kGather = 8;         // gathered rows in flight per lane group
constexpr int kLongEdge = 32;      // hyperedges with more members get a whole workgroup
constexpr int kEdgeTile = 32;      // hyperedges per workgroup of the edge gather
constexpr int kEdgeStageIdx = 1024;  // member ids of an edge tile staged in LDS
constexpr int kProfKinds = 16;     // kernel kinds of the timing counters

// ------------------------------------------------------ device buffers --

// Device memory source of a handle: the caller's allocator (hgl_allocator),
// or hipMalloc / hipFree when none was given.  `stream` is the stream of the
// call in progress: allocations are made for it and frees are ordered on it.
struct Mem {
  hgl_allocator al{};
  hipStream_t stream = nullptr;
  int alloc(void** p, size_t bytes);
  void release(void* p);
};

// Grow-only device buffer; its memory comes from `mem` (hipMalloc if null).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  Mem* mem = nullptr;
  int reserve(size_t n);
  void release();
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// ------------------------------------------------------------- the handle --

}  // namespace hgl

struct hgl_handle {
  int32_t N = 0, E = 0, G = 1;
  int64_t nnz = 0;
  int device = 0;
  hgl::Mem mem;  // every device allocation of the handle goes through it

  // structure (device)
  int32_t* edge_ptr = nullptr;   // [E+1]
  int32_t* edge_vtx = nullptr;   // [nnz]
  int32_t* vtx_ptr = nullptr;    // [N+1]
  int32_t* vtx_edge = nullptr;   // [nnz]

  // weights and scales (device)
  double* w = nullptr;           // [E]
  double* dv = nullptr;          // [N]
  double* s64 = nullptr;         // [N]
  double* c64 = nullptr;         // [E]
  float* s32 = nullptr;          // [N]
  float* c32 = nullptr;          // [E]

  // segments (graphs of a batched handle); host copies
  std::vector<int32_t> vtx_off, edge_off;   // [G+1]

  // row tiles for row-streaming kernels, segment-aligned (device)
  int32_t n_tiles = 0;
  int32_t* tile_r0 = nullptr;    // [n_tiles] first row
  int32_t* tile_r1 = nullptr;    // [n_tiles] one past last row
  int32_t* tile_seg = nullptr;   // [n_tiles]

  // vertex rows with more than kLongRow hyperedges, split into chunks (device)
  int32_t n_long = 0;
  int32_t n_chunks = 0;
  int32_t* long_row = nullptr;       // [n_long] vertex id, increasing
  int32_t* long_seg = nullptr;       // [n_long] graph of the row
  int32_t* chunk_slot = nullptr;     // [n_chunks] index into long_row
  int32_t* chunk_begin = nullptr;    // [n_chunks] position in vtx_edge
  int32_t* chunk_end = nullptr;      // [n_chunks]
  int32_t* long_chunk0 = nullptr;    // [n_long+1] first chunk of each long row
  // dispatch order of the chunk workgroups of a vertex gather: workgroup
  // n_tiles + j takes chunk chunk_order[j] (-1: none), so that a chunk that
  // reads one eighth of Z runs on that eighth's XCD; n_dispatch >= n_chunks
  // makes n_tiles + n_dispatch a multiple of kXcd
  int32_t n_dispatch = 0;
  int32_t* chunk_order = nullptr;    // [n_dispatch]

  // hyperedges with more than kLongEdge members, increasing id (device)
  int32_t n_long_edge = 0;
  int32_t* long_edge = nullptr;      // [n_long_edge]

  // edge tiles of the edge gather: kEdgeTile consecutive hyperedges of one
  // graph (device); per graph the slot ranges {t0, t1, l0, l1} of the edge
  // gather's partial sums over tiles + long hyperedges (device [G*4], host)
  int32_t n_etiles = 0;
  int32_t* etile_e0 = nullptr;       // [n_etiles]
  int32_t* etile_e1 = nullptr;       // [n_etiles]
  int32_t* seg_eslots = nullptr;
  std::vector<int32_t> seg_eslots_host;

  // per segment: partial-slot ranges {t0, t1, l0, l1} (device, [G*4]) over
  // tiles + long rows
  int32_t* seg_slots = nullptr;
  std::vector<int32_t> seg_slots_host;

  // scratch owned by the handle
  hgl::DevBuf ws_z, ws_z64, ws_chunk, ws_part, ws_part2, ws_vec, ws_state, ws_misc;
  hgl::DevBuf ws_extra[8];
  hgl::DevBuf ws_ab;                 // per-graph (1 + 1/lambda, 1/lambda)
  hgl::DevBuf wg_tab;                // one-workgroup CG: per-graph share tables and descriptors
  int32_t wg_lds = -1;               // one-workgroup CG: LDS bytes of the largest graph (-1: not built, -2: refused)
  std::vector<double> ab_cache;      // lambdas held in ws_ab

  // block rSVD workspace (owned, freed by rsvd_free)
  void* rsvd_ws = nullptr;
  void (*rsvd_free)(void*) = nullptr;
  // Schur-complement block inverse workspace (owned, freed by schur_free)
  void* schur_ws = nullptr;
  void (*schur_free)(void*) = nullptr;

  // kernel timing (diagnostics)
  bool prof_on = false;
  uint32_t prof_mask = 0;                             // kinds whose launches are stamped
  uint32_t prof_every = 1;                            // stamp every n-th launch of such a kind
  uint64_t prof_count[hgl::kProfKinds] = {0};         // launches seen per kind
  std::vector<hipEvent_t> prof_pool;                 // free events
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_pending;
  int64_t prof_launches[hgl::kProfKinds] = {0};
  double prof_ms[hgl::kProfKinds] = {0};
  int prof_kind = -1;                                // open kind (prof_begin), or -1
  // autotuned column shapes: {k, element size, base V} -> {GL, V, slabs} of
  // the edge gather, then of the vertex gather
  std::vector<std::array<int, 9>> tuned;
  // column shapes {GL, V, slabs} of the edge, then the vertex gather of the
  // latest CG solve
  int32_t last_shape[6] = {0, 0, 0, 0, 0, 0};
  // latest CG solve: {iterations enqueued, chunks, check steps, check steps
  // after which columns went on iterating}
  int32_t last_cg[4] = {0, 0, 0, 0};
  // CG iterations captured as a HIP graph (first chunk of a solve), replayed
  // while the solve's arguments stay the same
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t cg_graph = nullptr;
  std::vector<uint64_t> cg_graph_key;
  int32_t* pinned_i = nullptr;   // host-pinned readback words
  double* pinned_d = nullptr;
  size_t pinned_d_len = 0;
};

namespace hgl {

// The stream of the API call in progress (allocations through the handle's
// allocator are made for it).
inline void enter(hgl_handle* h, hipStream_t s) {
  if (h) h->mem.stream = s;
}

// Point a workspace's buffers at the handle's memory source.
template <class... B>
inline void attach(hgl_handle* h, B&... bufs) {
  ((bufs.mem = &h->mem), ...);
}

// Partial-slot count of the reductions: one per tile, one per long row.
inline int n_slots(const hgl_handle* h) { return h->n_tiles + h->n_long; }

int ensure_pinned(hgl_handle* h, size_t n_doubles);

// Launch shape of the column dimension: GL lanes per row, V elements per lane.
struct ColShape {
  int GL = 64;
  int V = 1;
  int slabs = 1;
  int width() const { return GL * V; }
};
ColShape pick_shape(int k, int elem_bytes, std::initializer_list<const void*> ptrs,
                    std::initializer_list<int64_t> lds);

// Column shapes of the two operator gathers.
struct GatherShapes {
  ColShape edge, vertex;
};

// Operands of the fused CG step (VMode::Step); unused by the other modes.
template <class T>
struct UpdArgs {
  T* F = nullptr;
  int64_t ldf = 0;
  T* R = nullptr;
  int64_t ldr = 0;
  const double* alpha = nullptr;  // [G*k]
};

// Autotuner: the column shapes under which the edge gather (with its
// hyperedge partials) and the vertex gather (as the fused CG step) each run
// fastest for k columns of the given element size, among the shapes that
// `base` (pick_shape's, with the widest valid vector) admits: narrower
// vectors, fewer lanes per row with more column slabs.  Timed once on X
// (N x k, leading dimension ldx) with scratch Z (E x k), u.F and u.R
// (u.alpha must be zero, so that F and R keep their values), epart and part,
// then cached in the handle under (k, element size, base vector width).
template <class T>
GatherShapes tune_shapes(hgl_handle* h, int k, const ColShape& base, const T* X, int64_t ldx, T* Z,
                         UpdArgs<T> u, double* epart, double* part, const double* a_seg, const double* b_seg,
                         hipStream_t s);

// Early-exit gate of a kernel launched inside the CG loop: the kernel does
// nothing when *active == 0 (no column iterates) or when it is a
// conditional residual pass (*flag == 0 and not periodic).
struct Gate {
  const int32_t* active = nullptr;
  const int32_t* flag = nullptr;
  int32_t periodic = 1;
  __device__ __forceinline__ bool skip() const {
    if (active && *active == 0) return true;
    if (flag && !periodic && *flag == 0) return true;
    return false;
  }
};

int upload_ab(hgl_handle* h, const double* lambdas_host, hipStream_t st);

// Kernel timing: bracket one launch of a kernel kind (no-ops unless enabled).
enum ProfKind { kProfEdge = 0, kProfVertex = 1, kProfUpdate = 2, kProfDirection = 3,
                kProfReduce = 4, kProfResidEdge = 5, kProfResidVertex = 6, kProfStart = 7,
                kProfPrecond = 8, kProfGemm = 9, kProfQr = 10, kProfEig = 11, kProfExtract = 12,
                kProfGrad = 13, kProfFinish = 14, kProfLeaf = 15 };
void prof_begin(hgl_handle* h, int kind, hipStream_t s);
void prof_end(hgl_handle* h, hipStream_t s);
hipEvent_t prof_event(hgl_handle* h);

// Launch one kernel.  While timing is enabled and a kind is open (prof_begin,
// or `kind` >= 0), the dispatch carries start/stop events that the runtime
// stamps at this kernel's own start and end, credited to that kind.
template <class F, class... Args>
inline void launch(const hgl_handle* hc, int kind, F kernel, dim3 grid, dim3 block, uint32_t shm, hipStream_t s,
                   Args... args) {
  hgl_handle* h = const_cast<hgl_handle*>(hc);
  const int kd = kind >= 0 ? kind : h->prof_kind;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->prof_on && kd >= 0 && ((h->prof_mask >> kd) & 1u) && (h->prof_count[kd]++ % h->prof_every) == 0) {
    e0 = prof_event(h);
    e1 = prof_event(h);
  }
  if (e0 && e1) {
    hipExtLaunchKernelGGL(kernel, grid, block, shm, s, e0, e1, 0, args...);
    h->prof_pending.push_back({kd, {e0, e1}});
  } else {
    // plain launch (also what stream capture records into a graph)
    auto actual = std::tuple<Args...>{args...};
    auto formal = validateArgsCountType(kernel, actual);
    void* kargs[sizeof...(Args) > 0 ? sizeof...(Args) : 1];
    pArgs<0>(formal, kargs);
    hipLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, kargs, shm, s);
  }
}

// Preconditioner for the CG driver: Z = P^-1 R (k columns), with partial
// inner products <R_j, Z_j> per row tile written to part (nullable).
// `key` holds what its launches bake in besides R, Z and part (buffer
// addresses, grid sizes, scalar arguments): a recorded CG graph is replayed
// only while the key is unchanged.
struct Precond {
  void* ctx = nullptr;
  int (*apply_f32)(void*, const float*, int64_t, float*, int64_t, double*, int, Gate, hipStream_t) = nullptr;
  int (*apply_f64)(void*, const double*, int64_t, double*, int64_t, double*, int, Gate, hipStream_t) = nullptr;
  std::array<uint64_t, 8> key{};
};

// The CG / preconditioned CG driver behind hgl_cg_solve (cg.hip).
int cg_run(hgl_handle* h, const double* lambdas, const hgl_cg_opts* o, const void* Y, int64_t ldy, void* F,
           int64_t ldf, int k, int32_t* iters_host, double* relres_host, const Precond* prec, hipStream_t s);

// Operator application pieces (spmm.hip).
enum class VMode { Apply = 0, ApplyDot = 1, Resid = 2, Step = 3 };


// Z = C H' S P: edge-major gather.  TIn = type of P, TAcc = type of Z.
// part (nullable): FP64 partial sums of sum_e c_e |(H' S P)_e|^2 per column,
// slot-major over the edge slots (edge tiles, then long hyperedges).
template <class TIn, class TAcc>
int launch_spmm_edge(const hgl_handle* h, const TIn* P, int64_t ldp, TAcc* Z, int64_t ldz,
                     int k, const ColShape& cs, Gate gate, hipStream_t s, double* part = nullptr);

// Edge-slot count of the edge gather's partial sums.
inline int n_eslots(const hgl_handle* h) { return h->n_etiles + h->n_long_edge; }

// Vertex-major gather + epilogue.  Apply: Out = a X - b s H Z (X may be null
// for a = 0).  ApplyDot: same
// and partial <X, Out> per column.  Resid: Out = Y - (a X - b s H Z) with FP64
// accumulation and partial <Out, Out>.  Step (T = TZ, X = P): with Q = a P -
// b s H Z kept in registers, u.F += alpha P, u.R -= alpha Q and partial
// <R, R> of the new R.  a, b per segment (device, [G]).  chunk_buf
// (nullable): the hub rows' chunk partials (n_chunks x k of TZ) in the
// caller's memory instead of the handle's workspace.
template <class T, class TZ>
int launch_spmm_vertex(const hgl_handle* h, VMode mode, const T* X, int64_t ldx, const TZ* Z,
                       int64_t ldz, const T* Y, int64_t ldy, T* Out, int64_t ldo,
                       const double* a_seg, const double* b_seg, double* part, int k,
                       const ColShape& cs, Gate gate, hipStream_t s, UpdArgs<T> u = {},
                       TZ* chunk_buf = nullptr);

}  // namespace hgl
