// Measurement probes: the achievable HBM bandwidth and BF16 MFMA rate of the
// device, the measured denominators that the roofline fractions are also
// reported against (beside the datasheet peaks).  Not part of the method.
#include "common.h"

namespace hgl {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kPeakBlock = 256;

// Stream copy, 16 bytes per lane, grid-stride, four loads in flight per
// lane before their stores.
constexpr int kCopyUnroll = 4;
__global__ __launch_bounds__(kPeakBlock) void k_peak_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                          int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * kPeakBlock;
  int64_t i = int64_t(blockIdx.x) * kPeakBlock + threadIdx.x;
  for (; i + (kCopyUnroll - 1) * stride < n; i += kCopyUnroll * stride) {
    uint4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) dst[i + u * stride] = v[u];
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// Every wave runs 2 iters rounds of four independent
// v_mfma_f32_16x16x32_bf16 on register operands (no memory traffic), then
// stores one value per workgroup only if it equals a sentinel the sums never
// reach, so the chain is kept without a store of consequence.
__global__ __launch_bounds__(kPeakBlock) void k_peak_mfma(float* __restrict__ out, int iters) {
  const int lane = threadIdx.x & 63;
  bf16x8 a, b;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = __bf16(float(lane + i) * 1e-3f);
    b[i] = __bf16(float(i - lane) * 1e-3f);
  }
  const floatx4 z = {0.f, 0.f, 0.f, 0.f};
  floatx4 c0 = z, c1 = z, c2 = z, c3 = z;
#pragma unroll 4
  for (int it = 0; it < 2 * iters; ++it) {
    c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c3, 0, 0, 0);
  }
  const float v = (c0[0] + c1[0]) + (c2[0] + c3[0]);
  if (v == 1.2345e30f) out[blockIdx.x] = v;
}

}  // namespace
}  // namespace hgl

using namespace hgl;

extern "C" int hgl_peak_copy(const void* src, void* dst, int64_t bytes, hipStream_t s) {
  clear_error();
  HGL_CHECK_ARG(src && dst, "src and dst must not be NULL");
  HGL_CHECK_ARG(bytes > 0 && bytes % 16 == 0, "bytes must be a positive multiple of 16");
  HGL_CHECK_ARG(reinterpret_cast<uintptr_t>(src) % 16 == 0 && reinterpret_cast<uintptr_t>(dst) % 16 == 0,
                "src and dst must be 16-byte aligned");
  const int64_t n = bytes / 16;
  const int64_t blocks = std::min<int64_t>((n + kPeakBlock - 1) / kPeakBlock, 256 * 64);
  hipLaunchKernelGGL(k_peak_copy, dim3(unsigned(blocks)), dim3(kPeakBlock), 0, s, static_cast<const uint4*>(src),
                     static_cast<uint4*>(dst), n);
  HGL_HIP(hipGetLastError());
  return HGL_OK;
}

extern "C" int hgl_peak_mfma_bf16(float* out, int32_t workgroups, int32_t iters, hipStream_t s) {
  clear_error();
  HGL_CHECK_ARG(out != nullptr, "out must not be NULL");
  HGL_CHECK_ARG(workgroups >= 1 && iters >= 1, "workgroups and iters must be >= 1");
  hipLaunchKernelGGL(k_peak_mfma, dim3(workgroups), dim3(kPeakBlock), 0, s, out, iters);
  HGL_HIP(hipGetLastError());
  return HGL_OK;
}
