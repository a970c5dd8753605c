// The operator apply Q = (I + L/lambda) P (section 2, eq. 1) for callers that
// cannot allocate device memory: the intermediate Z = C H' S P, the hub rows'
// chunk partials and the per-graph factors (1 + 1/lambda, 1/lambda) live in a
// fixed device array of this file instead of the handle's workspaces.  The
// kernels are those of hgl_apply.
#include <cmath>
#include <mutex>

#include "kernels.h"

namespace hgl {

// Scratch of the no-allocation entry point.  Each device the library runs on
// holds its own copy until the process ends.  In host code the name stands
// for a host-side shadow, never for device memory: every use goes through the
// per-device address that hipGetSymbolAddress returned.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
int scratch_ptr(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d out of range for the scratch table", dev);
    return HGL_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HGL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("hipGetSymbolAddress returned NULL for the scratch array");
      return HGL_EDEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HGL_OK;
}

constexpr size_t round256(size_t n) { return (n + 255) & ~size_t(255); }

// a_seg[g] = 1 + 1/lambda, b_seg[g] = 1/lambda for every graph (a kernel, not
// a memset or copy, so the call stays capturable and needs no pinned staging).
__global__ void k_fill_ab(double* ab, int G, double a, double b) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < G; g += gridDim.x * blockDim.x) {
    ab[g] = a;
    ab[G + g] = b;
  }
}

template <class T>
int apply_noalloc(hgl_handle* h, double lambda, const T* P, int64_t ldp, T* Q, int64_t ldq, int k,
                  hipStream_t st) {
  const size_t ab_bytes = round256(sizeof(double) * 2 * size_t(h->G));
  const size_t z_bytes = round256(sizeof(T) * size_t(h->E) * size_t(k));
  const size_t c_bytes = round256(sizeof(T) * size_t(h->n_chunks) * size_t(k));
  const size_t need = ab_bytes + z_bytes + c_bytes;
  if (need > kScratchBytes) {
    set_error("hgl_apply_noalloc needs %zu bytes of scratch (Z: E x k = %d x %d, hub partials: %d x %d), "
              "more than its fixed %zu",
              need, h->E, k, h->n_chunks, k, kScratchBytes);
    return HGL_EUNSUPPORTED;
  }
  int dev = 0;
  HGL_HIP(hipGetDevice(&dev));
  if (dev != h->device) {
    set_error("the current device (%d) is not the handle's (%d)", dev, h->device);
    return HGL_EINVAL;
  }
  void* base = nullptr;
  HGL_TRY(scratch_ptr(dev, &base));
  unsigned char* b = static_cast<unsigned char*>(base);
  double* ab = reinterpret_cast<double*>(b);
  T* Z = reinterpret_cast<T*>(b + ab_bytes);
  T* chunk = reinterpret_cast<T*>(b + ab_bytes + z_bytes);
  // per-launch timing events would be created on demand: keep them off
  const bool prof = h->prof_on;
  h->prof_on = false;
  int rc = HGL_OK;
  do {
    k_fill_ab<<<1, 64, 0, st>>>(ab, h->G, 1.0 + 1.0 / lambda, 1.0 / lambda);
    if (hipGetLastError() != hipSuccess) {
      set_error("k_fill_ab launch failed");
      rc = HGL_EDEVICE;
      break;
    }
    const ColShape cs = pick_shape(k, sizeof(T), {P, Q}, {ldp, ldq, int64_t(k)});
    rc = launch_spmm_edge<T, T>(h, P, ldp, Z, k, k, cs, Gate{}, st);
    if (rc < 0) break;
    rc = launch_spmm_vertex<T, T>(h, VMode::Apply, P, ldp, Z, k, nullptr, 0, Q, ldq, ab, ab + h->G, nullptr, k,
                                  cs, Gate{}, st, UpdArgs<T>{}, chunk);
  } while (false);
  h->prof_on = prof;
  return rc;
}

}  // namespace
}  // namespace hgl

using namespace hgl;

extern "C" int hgl_apply_noalloc(hgl_handle* h, double lambda, int32_t dt, const void* P, int64_t ldp, void* Q,
                                 int64_t ldq, int32_t k, hipStream_t st) {
  clear_error();
  HGL_CHECK_ARG(h != nullptr, "handle is NULL");
  HGL_CHECK_ARG(lambda > 0.0 && std::isfinite(lambda), "lambda must be > 0 (got %g)", lambda);
  HGL_CHECK_ARG(k >= 1, "k must be >= 1");
  HGL_CHECK_ARG(P && Q, "P and Q must not be NULL");
  HGL_CHECK_ARG(ldp >= k && ldq >= k, "leading dimensions must be >= k");
  HGL_CHECK_ARG(dt == HGL_F64 || dt == HGL_F32, "dtype must be HGL_F64 or HGL_F32");
  if (dt == HGL_F32)
    return apply_noalloc<float>(h, lambda, static_cast<const float*>(P), ldp, static_cast<float*>(Q), ldq, k, st);
  return apply_noalloc<double>(h, lambda, static_cast<const double*>(P), ldp, static_cast<double*>(Q), ldq, k,
                               st);
}
