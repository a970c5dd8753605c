// Device helpers shared by the kernels: vector row access and block reductions.
#pragma once

#include <type_traits>

#include "common.h"

namespace hgl {

template <class T, int V>
struct alignas(sizeof(T) * V) VecT {
  T v[V];
};

// Cross-lane reductions on DPP moves: a DPP operand is read in the same VALU
// instruction, where __shfl_xor goes through ds_bpermute, an LDS round trip
// per step.  GFX9 dpp_ctrl codes used: quad_perm [1,0,3,2] (0xB1) and
// [2,3,0,1] (0x4E), row_half_mirror (lane i of 8 reads lane 7 - i, 0x141),
// row_mirror (lane i of 16 reads lane 15 - i, 0x140).  The row helpers read
// only lanes of the caller's own row of 16, so a branch that is uniform per
// row may call them; the wave helpers need every lane active.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF,
                                                               false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = __builtin_amdgcn_update_dpp(0, int(uint32_t(u)), CTRL, 0xF, 0xF, false);
  const uint32_t hi = __builtin_amdgcn_update_dpp(0, int(uint32_t(u >> 32)), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}

__device__ __forceinline__ float readlane_f(float x, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
}

__device__ __forceinline__ double readlane_d(double x, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = __builtin_amdgcn_readlane(int(uint32_t(u)), l);
  const uint32_t hi = __builtin_amdgcn_readlane(int(uint32_t(u >> 32)), l);
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}

// Every lane of a row of 16 gets op over the row.  Each step combines a lane
// with its partner's partial of the same size, so the lanes of a row end with
// bit-identical results (op commutative).
template <class T, class Op>
__device__ __forceinline__ T row16_reduce(T x, Op op) {
  if constexpr (sizeof(T) == 8) {
    x = op(x, dpp_d<0xB1>(x));
    x = op(x, dpp_d<0x4E>(x));
    x = op(x, dpp_d<0x141>(x));
    return op(x, dpp_d<0x140>(x));
  } else {
    x = op(x, dpp_f<0xB1>(x));
    x = op(x, dpp_f<0x4E>(x));
    x = op(x, dpp_f<0x141>(x));
    return op(x, dpp_f<0x140>(x));
  }
}

// Every lane gets op over the wave: rows by DPP, then the four rows' results
// read as scalars and combined as (r0 op r1) op (r2 op r3).
template <class T, class Op>
__device__ __forceinline__ T wave_reduce(T x, Op op) {
  x = row16_reduce(x, op);
  if constexpr (sizeof(T) == 8)
    return op(op(readlane_d(x, 0), readlane_d(x, 16)), op(readlane_d(x, 32), readlane_d(x, 48)));
  else
    return op(op(readlane_f(x, 0), readlane_f(x, 16)), op(readlane_f(x, 32), readlane_f(x, 48)));
}

struct OpAdd {
  template <class T>
  __device__ __forceinline__ T operator()(T a, T b) const { return a + b; }
};
struct OpMin {
  __device__ __forceinline__ float operator()(float a, float b) const { return fminf(a, b); }
};
struct OpMax {
  __device__ __forceinline__ float operator()(float a, float b) const { return fmaxf(a, b); }
};

// Every lane of a row of 16 reads lane J of its own row (row_newbcast,
// dpp_ctrl 0x150 + J, GFX90A and later: one v_mov_b64_dpp).
template <int J>
__device__ __forceinline__ double row_bcast_d(double x) {
  static_assert(J >= 0 && J < 16, "lane within a row");
  return __builtin_amdgcn_mov_dpp(x, 0x150 + J, 0xF, 0xF, true);
}

// f(std::integral_constant<int, I>) for I = B .. E-1, so that each call's
// index is a compile-time constant (a DPP control must be one).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

template <class T>
__device__ __forceinline__ T row16_sum(T x) { return row16_reduce(x, OpAdd{}); }
template <class T>
__device__ __forceinline__ T wave_sum_dpp(T x) { return wave_reduce(x, OpAdd{}); }

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
