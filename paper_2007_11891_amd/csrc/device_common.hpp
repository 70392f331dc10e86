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

// a / b through the hardware reciprocal (about 2^-24 relative error on
// gfx950), one Newton step (reciprocal then within about 2^-48) and one
// residual correction of the quotient, q + r (a - b q) with fused
// multiply-adds, which by that error analysis leaves it within about one ulp
// of the IEEE quotient; not an IEEE division sequence, and not claimed to be
// correctly rounded.
__device__ inline double div_fast(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  const double e = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, e, r);
  const double q = a * r;
  return __builtin_fma(r, __builtin_fma(-b, q, a), q);
}
__device__ inline float div_fast(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

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

// K block sums at once (one LDS exchange): the same tree as block_sum for
// each; the results are valid in thread 0.
template <int NT, int K>
__device__ inline void block_sums(double (&v)[K]) {
  constexpr int NW = NT / 64;
  __shared__ double s_w[K][NW];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if constexpr (NW > 1) {
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) s_w[k][threadIdx.x >> 6] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < NW; ++i) t += s_w[k][i];
        v[k] = t;
      }
    }
    __syncthreads();
  }
}

// Deterministic sum of nparts partials written by an earlier launch, with
// stride `stride` and offset `off`, by a whole block of NT threads.  Every
// block that calls it gets the same value (same order, same tree); the result
// is broadcast to all threads through sbuf.
template <int NT>
__device__ inline double sum_partials(const double* __restrict__ parts, int nparts, int stride,
                                      int off, double* sbuf) {
  // up to 4 loads per thread in flight, then a fixed-order combine
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i0 = threadIdx.x; i0 < nparts; i0 += 4 * NT) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * NT;
      if (i < nparts) v[u] += parts[(size_t)i * stride + off];
    }
  }
  double t = block_sum<NT>((v[0] + v[1]) + (v[2] + v[3]), sbuf);
  __shared__ double s_bcast;
  if (threadIdx.x == 0) s_bcast = t;
  __syncthreads();
  t = s_bcast;
  __syncthreads();
  return t;
}

// Two partial arrays summed in one pass (same order as two sum_partials).
template <int NT>
__device__ inline void sum_partials2(const double* __restrict__ pa, const double* __restrict__ pb,
                                     int nparts, double* sbuf, double* ra, double* rb) {
  double va[4] = {0.0, 0.0, 0.0, 0.0}, vb[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i0 = threadIdx.x; i0 < nparts; i0 += 4 * NT) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * NT;
      if (i < nparts) {
        va[u] += pa[i];
        vb[u] += pb[i];
      }
    }
  }
  double ta = block_sum<NT>((va[0] + va[1]) + (va[2] + va[3]), sbuf);
  double tb = block_sum<NT>((vb[0] + vb[1]) + (vb[2] + vb[3]), sbuf);
  __shared__ double s_bc2[2];
  if (threadIdx.x == 0) {
    s_bc2[0] = ta;
    s_bc2[1] = tb;
  }
  __syncthreads();
  *ra = s_bc2[0];
  *rb = s_bc2[1];
  __syncthreads();
}

// K partial arrays of nparts values each, summed by a whole block of NT
// threads in a fixed order (every block gets the same bits): thread t adds
// entries t + u NT + c 4 NT into accumulator u (chunks c in order), the four
// accumulators combine as (v0 + v1) + (v2 + v3), then a wavefront butterfly,
// then the wavefront sums in order.  The loads of the first chunk are issued
// by `issue`, so that a kernel can put them in flight early and do other
// work before `reduce` (which loads any further chunks and returns the sums
// in every thread).
template <int NT, int K>
struct PartialSums {
  double v[K][4];
  __device__ inline void issue(const double* const* p, int nparts) {
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = (int)threadIdx.x + u * NT;
        v[k][u] = i < nparts ? p[k][i] : 0.0;
      }
  }
  __device__ inline void reduce(const double* const* p, int nparts, double* out) {
    for (int i0 = (int)threadIdx.x + 4 * NT; i0 < nparts; i0 += 4 * NT) {
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + u * NT;
          if (i < nparts) v[k][u] += p[k][i];
        }
    }
    constexpr int NW = NT / 64;
    __shared__ double s_w[K][NW];
    double w[K];
#pragma unroll
    for (int k = 0; k < K; ++k) w[k] = wave_sum((v[k][0] + v[k][1]) + (v[k][2] + v[k][3]));
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) s_w[k][threadIdx.x >> 6] = w[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < NW; ++i) t += s_w[k][i];
      out[k] = t;
    }
    __syncthreads();                         // s_w is reused by the next call
  }
};

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
