// hdg_apply_noalloc: the operator apply of hdg_apply with its two per-face
// element contributions (qa, qb: the scratch of that entry point) kept in a
// file-scope device array instead of memory the library allocates, for
// callers that cannot allocate device memory (graph capture, serving loops,
// harnesses that forbid hipMalloc).  The array's device address is taken
// with hipGetSymbolAddress once per device, at the first call on that
// device, and only that address is passed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/hdg.h"
#include "hdg_internal.hpp"
#include "host_util.hpp"

namespace hdg {

constexpr size_t kNoAllocScratchBytes = (size_t)48 << 20;   // 48 MiB per GPU
constexpr int kNoAllocMaxDevices = 64;

// Host code never passes this name to a kernel: it stands for the array on
// the host side only; kernels get the device address from scratch_on.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};

// Device address of `scratch` on the current device (taken once per device).
hdg_status scratch_on(int dev, void** out) {
  if (dev < 0 || dev >= kNoAllocMaxDevices)
    return fail(HDG_EUNSUPPORTED, "device %d beyond the %d devices hdg_apply_noalloc supports",
                dev, kNoAllocMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(HDG_EHIP, "hipGetSymbolAddress of the apply scratch failed: %s",
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return HDG_OK;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

template <typename T>
const T* noalloc_mat(const hdg_ctx* c, int kind);
template <>
const double* noalloc_mat<double>(const hdg_ctx* c, int kind) { return mat64(c, kind); }
template <>
const float* noalloc_mat<float>(const hdg_ctx* c, int kind) { return mat32(c, kind); }

template <typename T>
hdg_status apply_noalloc(hdg_ctx* c, const T* x, T* y, hdg_basis basis, unsigned char* base) {
  const int64_t nff = c->n_free_faces;
  const size_t vec = round256(sizeof(T) * (size_t)c->n_free);
  T* qa = reinterpret_cast<T*>(base);
  T* qb = reinterpret_cast<T*>(base + vec);
  const T* xin = x;
  if (basis == HDG_BASIS_NODAL) {
    T* t = reinterpret_cast<T*>(base + 2 * vec);
    HIP_TRY(launch_face_transform<T>(c->np, noalloc_mat<T>(c, HDG_TO_EIGEN_UNKNOWN), x, nullptr,
                                     t, nff, c->stream));
    xin = t;
  }
  // every free face receives both contributions (the second one zero on a
  // face with one element), so nothing in the scratch needs clearing
  HIP_TRY(launch_elem_apply<T>(c, xin, nullptr, qa, qb, c->stream));
  if (basis == HDG_BASIS_NODAL)
    HIP_TRY(launch_face_transform<T>(c->np, noalloc_mat<T>(c, HDG_TO_NODAL_RESIDUAL), qa, qb, y,
                                     nff, c->stream));
  else
    HIP_TRY(launch_combine<T>(qa, qb, y, c->n_free, c->stream));
  return HDG_OK;
}

}  // namespace
}  // namespace hdg

using namespace hdg;

extern "C" hdg_status hdg_apply_noalloc(hdg_ctx* c, const void* x, void* y, hdg_dtype dtype,
                                        hdg_basis basis) {
  if (!c || !x || !y) return fail(HDG_EINVAL, "NULL argument");
  if (x == y) return fail(HDG_EINVAL, "x and y must not overlap");
  if (dtype != HDG_F64 && dtype != HDG_F32) return fail(HDG_EINVAL, "unknown dtype");
  if (basis != HDG_BASIS_NODAL && basis != HDG_BASIS_EIGEN) return fail(HDG_EINVAL, "unknown basis");
  if (c->n_free == 0) return HDG_OK;
  const size_t elem = dtype == HDG_F64 ? sizeof(double) : sizeof(float);
  const size_t need = (basis == HDG_BASIS_NODAL ? 3 : 2) * round256(elem * (size_t)c->n_free);
  if (need > kNoAllocScratchBytes)
    return fail(HDG_EINVAL,
                "hdg_apply_noalloc needs %zu bytes of scratch for %lld unknowns; its limit is %zu "
                "bytes per GPU",
                need, (long long)c->n_free, kNoAllocScratchBytes);
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != c->device)
    return fail(HDG_EINVAL, "the context lives on device %d, device %d is current", c->device,
                dev);
  void* base = nullptr;
  ST_TRY(scratch_on(dev, &base));
  if (dtype == HDG_F64)
    return apply_noalloc<double>(c, static_cast<const double*>(x), static_cast<double*>(y), basis,
                                 static_cast<unsigned char*>(base));
  return apply_noalloc<float>(c, static_cast<const float*>(x), static_cast<float*>(y), basis,
                              static_cast<unsigned char*>(base));
}
