// Host-side helpers shared by the API translation units: device allocation
// and the HIP / status propagation macros (error reporting: host_setup.hpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/hdg.h"
#include "host_setup.hpp"

namespace hdg {

template <typename T>
hdg_status dalloc(T** p, int64_t n) {
  *p = nullptr;
  if (n <= 0) n = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)n);
  if (e != hipSuccess)
    return fail(HDG_ENOMEM, "hipMalloc of %lld bytes failed: %s", (long long)(sizeof(T) * n),
                hipGetErrorString(e));
  return HDG_OK;
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

}  // namespace hdg

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess)                                                                \
      return ::hdg::fail(HDG_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), \
                         __FILE__, __LINE__);                                            \
  } while (0)

#define ST_TRY(expr)             \
  do {                           \
    hdg_status _s = (expr);      \
    if (_s != HDG_OK) return _s; \
  } while (0)
