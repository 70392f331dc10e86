// Device helpers shared by the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>

#include "hdg_internal.hpp"

namespace hdg {

__host__ __device__ constexpr int round_up64(int v) { return (v + 63) / 64 * 64; }

// Elements per block of the element kernels for n_p points per direction:
// blocks of about 256 threads (n_p^2 threads per element).
__host__ __device__ constexpr int epb_for(int np) {
  return (256 / (np * np)) > 0 ? (256 / (np * np)) : 1;
}
__host__ __device__ constexpr int elem_block_threads(int np) {
  return round_up64(epb_for(np) * np * np);
}

// Workgroups are dispatched round-robin over the 8 XCDs; remap so that each
// XCD processes one contiguous range of block ids (neighbouring elements
// share faces, so their reads hit the same L2).
__device__ inline int xcd_remap(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = bid & 7, k = bid >> 3;
  return (xcd < r) ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block sum for a block of NT threads (NT a multiple of 64); the result is
// valid in thread 0.  sbuf holds NT/64 doubles.
template <int NT>
__device__ inline double block_sum(double v, double* sbuf) {
  v = wave_sum(v);
  constexpr int NW = NT / 64;
  if constexpr (NW == 1) {
    return v;
  } else {
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sbuf[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < NW; ++i) s += sbuf[i];
    }
    __syncthreads();
    return s;
  }
}

__device__ inline void store_partial(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double load_partial(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every block calls this once after thread 0 stored its partial(s); returns
// true in all threads of the block that arrives last.  That block resets the
// counter for the next launch.
__device__ inline bool arrive_last(unsigned* cnt, unsigned nblocks) {
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(cnt, 1u);
    s_last = (prev == nblocks - 1) ? 1 : 0;
    if (s_last) {
      __threadfence();
      __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();
  return s_last != 0;
}

// Deterministic sum of nparts partials with stride `stride` (offset `off`),
// performed by the whole (last) block of NT threads; valid in thread 0.
template <int NT>
__device__ inline double sum_partials(const double* parts, int nparts, int stride, int off,
                                      double* sbuf) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nparts; i += NT) v += load_partial(parts + (size_t)i * stride + off);
  return block_sum<NT>(v, sbuf);
}

// Face id of the face of element (i,j,k) normal to axis a on side s (0 low,
// 1 high).  Sets *is_free.
__device__ inline int64_t face_of(const MeshDev& m, int a, int s, int i, int j, int k,
                                  bool* is_free) {
  if (a == 0) {
    const int pl = i + s;
    if (pl >= 1 && pl <= m.n1 - 1) {
      *is_free = true;
      return m.foff[0] + (pl - 1) + (int64_t)(m.n1 - 1) * (j + (int64_t)m.n2 * k);
    }
    *is_free = false;
    return m.boff[0 + (pl == 0 ? 0 : 1)] + j + (int64_t)m.n2 * k;
  } else if (a == 1) {
    const int pl = j + s;
    if (pl >= 1 && pl <= m.n2 - 1) {
      *is_free = true;
      return m.foff[1] + i + (int64_t)m.n1 * ((pl - 1) + (int64_t)(m.n2 - 1) * k);
    }
    *is_free = false;
    return m.boff[2 + (pl == 0 ? 0 : 1)] + i + (int64_t)m.n1 * k;
  } else {
    const int pl = k + s;
    if (pl >= 1 && pl <= m.n3 - 1) {
      *is_free = true;
      return m.foff[2] + i + (int64_t)m.n1 * (j + (int64_t)m.n2 * (pl - 1));
    }
    *is_free = false;
    return m.boff[4 + (pl == 0 ? 0 : 1)] + i + (int64_t)m.n1 * j;
  }
}

}  // namespace hdg
