// Device helpers shared by the kernels: vector row access and block reductions.
#pragma once

#include "common.h"

namespace hgl {

template <class T, int V>
struct alignas(sizeof(T) * V) VecT {
  T v[V];
};

template <int V, class T>
__device__ __forceinline__ void load_row(const T* __restrict__ p, T (&x)[V]) {
  VecT<T, V> t = *reinterpret_cast<const VecT<T, V>*>(p);
#pragma unroll
  for (int i = 0; i < V; ++i) x[i] = t.v[i];
}

template <int V, class T>
__device__ __forceinline__ void store_row(T* __restrict__ p, const T (&x)[V]) {
  VecT<T, V> t;
#pragma unroll
  for (int i = 0; i < V; ++i) t.v[i] = x[i];
  *reinterpret_cast<VecT<T, V>*>(p) = t;
}

// acc += sum_{j in [jb, je)} Z[idx[j], col .. col+V-1], kGather rows in
// flight: every batch issues all its loads before the sums (masked past je,
// so a short row costs one round trip), and the batch is summed in a fixed
// order.
template <int V, class TZ>
__device__ __forceinline__ void gather_rows(const TZ* __restrict__ Z, int64_t ldz,
                                            const int32_t* __restrict__ idx, int jb, int je, int col,
                                            TZ (&acc)[V]) {
  for (int j = jb; j < je; j += kGather) {
    int e[kGather];
#pragma unroll
    for (int u = 0; u < kGather; ++u) e[u] = j + u < je ? idx[j + u] : -1;
    TZ z[kGather][V];
#pragma unroll
    for (int u = 0; u < kGather; ++u) {
      if (e[u] >= 0) {
        load_row<V>(Z + int64_t(e[u]) * ldz + col, z[u]);
      } else {
#pragma unroll
        for (int i = 0; i < V; ++i) z[u][i] = TZ(0);
      }
    }
#pragma unroll
    for (int i = 0; i < V; ++i) {
      TZ sum = z[0][i];
#pragma unroll
      for (int u = 1; u < kGather; ++u) sum += z[u][i];
      acc[i] += sum;
    }
  }
}

// Sum, over the groups of a 256-thread block, of per-lane values x[V] whose
// column is (lane within its GL-wide group, i).  The result for column
// tid = lane*V + i (tid < GL*V) is returned in thread tid.  Fixed order, so
// deterministic.  Every thread of the block must call it.
template <int GL, int V, class T>
__device__ __forceinline__ T block_colsum(T (&x)[V], T* lds /* [4 * GL * V] */) {
#pragma unroll
  for (int off = GL; off < kWave; off <<= 1) {
#pragma unroll
    for (int i = 0; i < V; ++i) x[i] += __shfl_xor(x[i], off, kWave);
  }
  const int wave = threadIdx.x / kWave, lw = threadIdx.x % kWave;
  if (lw < GL) {
#pragma unroll
    for (int i = 0; i < V; ++i) lds[wave * GL * V + lw * V + i] = x[i];
  }
  __syncthreads();
  T r = T(0);
  if (threadIdx.x < GL * V) {
    const int t = threadIdx.x;
    r = ((lds[t] + lds[GL * V + t]) + lds[2 * GL * V + t]) + lds[3 * GL * V + t];
  }
  __syncthreads();
  return r;
}

// Dispatch a lambda templated on (GL, V) for the runtime shape.
#define HGL_DISPATCH_SHAPE(cs, ELEM_BYTES, BODY)                                 \
  [&]() -> int {                                                                \
    switch ((cs).GL * 8 + (cs).V) {                                             \
      case 64 * 8 + 4: if constexpr (ELEM_BYTES * 4 <= 16) { constexpr int GL = 64, V = 4; BODY; } break; \
      case 64 * 8 + 2: { constexpr int GL = 64, V = 2; BODY; } break;           \
      case 64 * 8 + 1: { constexpr int GL = 64, V = 1; BODY; } break;           \
      case 32 * 8 + 4: if constexpr (ELEM_BYTES * 4 <= 16) { constexpr int GL = 32, V = 4; BODY; } break; \
      case 32 * 8 + 2: { constexpr int GL = 32, V = 2; BODY; } break;           \
      case 32 * 8 + 1: { constexpr int GL = 32, V = 1; BODY; } break;           \
      case 16 * 8 + 4: if constexpr (ELEM_BYTES * 4 <= 16) { constexpr int GL = 16, V = 4; BODY; } break; \
      case 16 * 8 + 2: { constexpr int GL = 16, V = 2; BODY; } break;           \
      case 16 * 8 + 1: { constexpr int GL = 16, V = 1; BODY; } break;           \
      case 8 * 8 + 4: if constexpr (ELEM_BYTES * 4 <= 16) { constexpr int GL = 8, V = 4; BODY; } break; \
      case 8 * 8 + 2: { constexpr int GL = 8, V = 2; BODY; } break;             \
      case 8 * 8 + 1: { constexpr int GL = 8, V = 1; BODY; } break;             \
      case 4 * 8 + 4: if constexpr (ELEM_BYTES * 4 <= 16) { constexpr int GL = 4, V = 4; BODY; } break; \
      case 4 * 8 + 2: { constexpr int GL = 4, V = 2; BODY; } break;             \
      case 4 * 8 + 1: { constexpr int GL = 4, V = 1; BODY; } break;             \
      default: break;                                                           \
    }                                                                           \
    ::hgl::set_error("unsupported column shape GL=%d V=%d", (cs).GL, (cs).V);  \
    return HGL_EUNSUPPORTED;                                                    \
  }()

}  // namespace hgl
