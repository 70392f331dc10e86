// Vector kernels of the preconditioned CG on the free trace, face transforms,
// and the diagonal of the transformed operator.
//
// CG (paper: section "Summary of solution method", solver HDG-trans): the
// iteration is split into two launches.  The fused element apply (see
// elem_kernels.hip) forms p = z + beta p_old on the fly, writes p, and
// reduces p.q from element-local quadratic forms.  The update below forms
// alpha = rho / p.q, q = qa + qb, z -= alpha D^-1 q, x += alpha p, and
// reduces r.z and r.r with r = z / D^-1.  The CG carries z = D^-1 r instead
// of r: the element kernel, whose face gather streams memory less
// efficiently, then reads two vectors per face instead of four, and the
// x update moves to this streaming kernel.  All reductions are block
// partials summed in a fixed order.
#include "device_common.hpp"

namespace hdg {

constexpr int kVecThreads = 256;
constexpr int kUnroll = 4;

static inline int vec_blocks(int64_t n, int cap = 2048) {
  int64_t nb = (n + kVecThreads * kUnroll - 1) / (kVecThreads * kUnroll);
  if (nb > cap) nb = cap;
  if (nb < 1) nb = 1;
  return (int)nb;
}

// ------------------------------------------------------------------ CG ----
// Update of iteration k: alpha_k = rho_k / (p_k . q_k) with p.q summed from
// the apply's partials; z -= alpha D^-1 q with q = qa + qb; x += alpha p_k;
// partials of r.z and r.r for the next apply.  Block 0 publishes slot A.
template <typename T>
__global__ void __launch_bounds__(kVecThreads)
cg_update_kernel(int64_t n, const T* __restrict__ qa, const T* __restrict__ qb, T* __restrict__ z,
                 const T* __restrict__ dinv, T* __restrict__ x, const T* __restrict__ p0,
                 const T* __restrict__ p1, double* __restrict__ partials, int pmax, int n_apply,
                 CgScalars* sc) {
  __shared__ double s_red[kVecThreads / 64];
  // scalar reads of slot B (a struct copy here costs a large serialisation)
  const int done = sc->B.done;
  if (done) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->A.done = done;
      sc->A.rr = sc->B.rr;
    }
    return;
  }
  const int k = sc->B.iter;
  const double rho = sc->B.rho;
  const T* __restrict__ p = (k & 1) ? p1 : p0;   // p_k, written by the apply of iteration k
  // kUnroll independent entries per thread, all loads issued before use; the
  // partials' loads and the first group's go out before the partial sums
  const int64_t stride = (int64_t)gridDim.x * kVecThreads;
  int64_t g0 = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  T va[kUnroll], vb[kUnroll], vz[kUnroll], vd[kUnroll], vx[kUnroll], vp[kUnroll];
  auto load = [&](int64_t base) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t g = base + u * stride;
      if (g < n) {
        va[u] = qa[g];
        vb[u] = qb[g];
        vz[u] = z[g];
        vd[u] = dinv[g];
        vx[u] = x[g];
        vp[u] = p[g];
      }
    }
  };
  const double* pp[1] = {partials + (size_t)(k & 1) * pmax};
  PartialSums<kVecThreads, 1> ps;
  ps.issue(pp, n_apply);
  if (g0 < n) load(g0);
  double pq;
  ps.reduce(pp, n_apply, &pq);
  const double alpha = rho / pq;
  if (!(pq > 0.0) || !isfinite(alpha)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->A.done = 3;
      sc->A.alpha = 0.0;
      sc->A.pq = pq;
    }
    return;
  }
  const T a = (T)alpha;
  T rz_t = 0, rr_t = 0;
  for (; g0 < n; g0 += kUnroll * stride) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t g = g0 + u * stride;
      if (g < n) {
        const T zn = vz[u] - a * (vd[u] * (va[u] + vb[u]));
        z[g] = zn;
        x[g] = vx[u] + a * vp[u];
        const T rn = div_fast(zn, vd[u]);
        rz_t += zn * rn;
        rr_t += rn * rn;
      }
    }
    if (g0 + kUnroll * stride < n) load(g0 + kUnroll * stride);
  }
  double sums[2] = {(double)rz_t, (double)rr_t};
  block_sums<kVecThreads, 2>(sums);
  const int k1 = (k + 1) & 1;
  if (threadIdx.x == 0) {
    partials[(size_t)(2 + k1) * pmax + blockIdx.x] = sums[0];
    partials[(size_t)(4 + k1) * pmax + blockIdx.x] = sums[1];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // rho_k becomes the previous rho of iteration k+1
    sc->A.rho = rho;
    sc->A.alpha = alpha;
    sc->A.pq = pq;
    sc->A.rr_stop = sc->B.rr_stop;
    sc->A.rr = sc->B.rr;
    sc->A.iter = k + 1;
    sc->A.done = 0;
  }
}

// z = D^-1 b (r = b), x = 0, p_{-1} = 0, and the partials of b.D^-1 b and
// b.b that the first apply sums (they play the role of the update of
// iteration -1).
template <typename T>
__global__ void __launch_bounds__(kVecThreads)
cg_init_kernel(int64_t n, const T* __restrict__ b, T* __restrict__ z, T* __restrict__ x,
               T* __restrict__ p1, const T* __restrict__ dinv, double* __restrict__ partials,
               int pmax) {
  __shared__ double s_red[kVecThreads / 64];
  T rz_t = 0, rr_t = 0;
  for (int64_t g = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * kVecThreads) {
    const T v = b[g];
    const T zv = dinv[g] * v;
    z[g] = zv;
    x[g] = 0;
    p1[g] = 0;
    rz_t += v * zv;
    rr_t += v * v;
  }
  const double brz = block_sum<kVecThreads>((double)rz_t, s_red);
  const double brr = block_sum<kVecThreads>((double)rr_t, s_red);
  if (threadIdx.x == 0) {
    partials[(size_t)2 * pmax + blockIdx.x] = brz;
    partials[(size_t)4 * pmax + blockIdx.x] = brr;
  }
}

// Continuation of a CG on a replaced residual (reliable update of the mixed-
// precision solver): z = D^-1 b, x = 0, the previous direction rescaled,
// and the r.z / r.r partials the next apply sums (state slot `slot`).
template <typename T>
__global__ void __launch_bounds__(kVecThreads)
cg_continue_kernel(int64_t n, const T* __restrict__ b, T* __restrict__ z, T* __restrict__ x,
                   T* __restrict__ p_prev, T pscale, const T* __restrict__ dinv,
                   double* __restrict__ partials, int pmax, int slot) {
  __shared__ double s_red[kVecThreads / 64];
  T rz_t = 0, rr_t = 0;
  for (int64_t g = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * kVecThreads) {
    const T v = b[g];
    const T zv = dinv[g] * v;
    z[g] = zv;
    x[g] = 0;
    p_prev[g] *= pscale;
    rz_t += v * zv;
    rr_t += v * v;
  }
  const double brz = block_sum<kVecThreads>((double)rz_t, s_red);
  const double brr = block_sum<kVecThreads>((double)rr_t, s_red);
  if (threadIdx.x == 0) {
    partials[(size_t)(2 + slot) * pmax + blockIdx.x] = brz;
    partials[(size_t)(4 + slot) * pmax + blockIdx.x] = brr;
  }
}

template <typename T>
hipError_t launch_cg_continue(const hdg_ctx*, CgWork<T>& w, const T* b, int iter, double pscale,
                              hipStream_t s) {
  T* p_prev = (iter & 1) ? w.p[0] : w.p[1];   // p_{k-1}: the input direction of iteration k
  hipLaunchKernelGGL((cg_continue_kernel<T>), dim3(w.update_blocks), dim3(kVecThreads), 0, s, w.n,
                     b, w.z, w.x, p_prev, (T)pscale, w.dinv, w.partials, w.pmax, iter & 1);
  return hipGetLastError();
}
template hipError_t launch_cg_continue<double>(const hdg_ctx*, CgWork<double>&, const double*, int,
                                               double, hipStream_t);
template hipError_t launch_cg_continue<float>(const hdg_ctx*, CgWork<float>&, const float*, int,
                                              double, hipStream_t);

// One-kernel CG: z_0 = D^-1 b (r_0 = b), x = 0, p_{-1} = s_{-1} = 0.  The
// first iteration launch applies the operator to z_0 and reduces r.z, r.r.
template <typename T>
__global__ void __launch_bounds__(kVecThreads)
cgcg_init_kernel(int64_t n, const T* __restrict__ b, T* __restrict__ z0, T* __restrict__ x,
                 T* __restrict__ p1, T* __restrict__ s1, const T* __restrict__ dinv) {
  for (int64_t g = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * kVecThreads) {
    z0[g] = dinv[g] * b[g];
    x[g] = 0;
    p1[g] = 0;
    s1[g] = 0;
  }
}

template <typename T>
hipError_t launch_cgcg_init(const hdg_ctx*, CgWork<T>& w, const T* b, hipStream_t s) {
  hipLaunchKernelGGL((cgcg_init_kernel<T>), dim3(w.update_blocks), dim3(kVecThreads), 0, s, w.n, b,
                     w.zz[0], w.x, w.p[1], w.s[1], w.dinv);
  return hipGetLastError();
}
template hipError_t launch_cgcg_init<double>(const hdg_ctx*, CgWork<double>&, const double*,
                                             hipStream_t);
template hipError_t launch_cgcg_init<float>(const hdg_ctx*, CgWork<float>&, const float*,
                                            hipStream_t);

template <typename T>
hipError_t launch_cg_update(const hdg_ctx* c, CgWork<T>& w, hipStream_t s) {
  hipLaunchKernelGGL((cg_update_kernel<T>), dim3(w.update_blocks), dim3(kVecThreads), 0, s, w.n,
                     w.qa, w.qb, w.z, w.dinv, w.x, w.p[0], w.p[1], w.partials, w.pmax,
                     w.apply_blocks, w.sc);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_cg_init(const hdg_ctx*, CgWork<T>& w, const T* b, hipStream_t s) {
  hipLaunchKernelGGL((cg_init_kernel<T>), dim3(w.update_blocks), dim3(kVecThreads), 0, s, w.n, b,
                     w.z, w.x, w.p[1], w.dinv, w.partials, w.pmax);
  return hipGetLastError();
}

template hipError_t launch_cg_update<double>(const hdg_ctx*, CgWork<double>&, hipStream_t);
template hipError_t launch_cg_update<float>(const hdg_ctx*, CgWork<float>&, hipStream_t);
template hipError_t launch_cg_init<double>(const hdg_ctx*, CgWork<double>&, const double*,
                                           hipStream_t);
template hipError_t launch_cg_init<float>(const hdg_ctx*, CgWork<float>&, const float*,
                                          hipStream_t);

// ------------------------------------------------------------ combine ----
template <typename T>
__global__ void __launch_bounds__(kVecThreads)
combine_kernel(int64_t n, const T* __restrict__ qa, const T* __restrict__ qb, T* __restrict__ y) {
  for (int64_t g = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * kVecThreads)
    y[g] = qa[g] + qb[g];
}

template <typename T>
hipError_t launch_combine(const T* qa, const T* qb, T* y, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((combine_kernel<T>), dim3(vec_blocks(n, 8192)), dim3(kVecThreads), 0, s, n,
                     qa, qb, y);
  return hipGetLastError();
}
template hipError_t launch_combine<double>(const double*, const double*, double*, int64_t,
                                           hipStream_t);
template hipError_t launch_combine<float>(const float*, const float*, float*, int64_t,
                                          hipStream_t);

// out[0] = sum of n partials (one block, fixed order)
__global__ void __launch_bounds__(kVecThreads)
reduce_partials_kernel(const double* __restrict__ parts, int n, double* __restrict__ out) {
  __shared__ double s_red[kVecThreads / 64];
  const double v = sum_partials<kVecThreads>(parts, n, 1, 0, s_red);
  if (threadIdx.x == 0) out[0] = v;
}

// r = b - (qa + qb); out[0] = ||r||^2 (FP64)
__global__ void __launch_bounds__(kVecThreads)
residual64_kernel(int64_t n, const double* __restrict__ b, const double* __restrict__ qa,
                  const double* __restrict__ qb, double* __restrict__ r, double* partials) {
  __shared__ double s_red[kVecThreads / 64];
  double acc = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * kVecThreads) {
    const double v = b[g] - (qa[g] + qb[g]);
    r[g] = v;
    acc += v * v;
  }
  const double bs = block_sum<kVecThreads>(acc, s_red);
  if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

hipError_t launch_residual64(const double* b, const double* qa, const double* qb, double* r,
                             int64_t n, double* partials, double* out, int nblocks,
                             hipStream_t s) {
  hipLaunchKernelGGL(residual64_kernel, dim3(nblocks), dim3(kVecThreads), 0, s, n, b, qa, qb, r,
                     partials);
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(kVecThreads), 0, s, partials, nblocks,
                     out);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kVecThreads)
dot64_kernel(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
             double* partials) {
  __shared__ double s_red[kVecThreads / 64];
  double acc = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * kVecThreads)
    acc += a[g] * b[g];
  const double bs = block_sum<kVecThreads>(acc, s_red);
  if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

hipError_t launch_dot64(const double* a, const double* b, int64_t n, double* partials,
                        double* out, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(dot64_kernel, dim3(nblocks), dim3(kVecThreads), 0, s, n, a, b, partials);
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(kVecThreads), 0, s, partials, nblocks,
                     out);
  return hipGetLastError();
}

// --------------------------------------------------------------- misc ----
// Plain copy (reference kernel of known traffic for counter calibration).
__global__ void copy64_kernel(int64_t n, const double* __restrict__ in, double* __restrict__ out) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x)
    out[g] = in[g];
}
// CG state before a solve, from kernel arguments (no host buffer to keep
// alive, so the host needs no synchronisation before the next upload).
__global__ void state_reset_kernel(CgScalars* sc, double rtol2, int maxit) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    CgScalars s{};
    s.A.rtol2 = rtol2;
    s.A.maxit = maxit;
    s.A.rho = 1.0;
    *sc = s;
  }
}
hipError_t launch_state_reset(CgScalars* sc, double rtol2, int maxit, hipStream_t s) {
  hipLaunchKernelGGL(state_reset_kernel, dim3(1), dim3(64), 0, s, sc, rtol2, maxit);
  return hipGetLastError();
}

__global__ void add64_kernel(int64_t n, const double* __restrict__ in, double* __restrict__ out) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x)
    out[g] += in[g];
}
hipError_t launch_add64(const double* in, double* out, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(add64_kernel, dim3(vec_blocks(n, 8192)), dim3(kVecThreads), 0, s, n, in,
                     out);
  return hipGetLastError();
}

hipError_t launch_copy64(const double* in, double* out, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(copy64_kernel, dim3(vec_blocks(n, 8192)), dim3(kVecThreads), 0, s, n, in,
                     out);
  return hipGetLastError();
}

__global__ void cast_scale_kernel(int64_t n, const double* __restrict__ in, float* __restrict__ out,
                                  double scale) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x)
    out[g] = (float)(in[g] * scale);
}
hipError_t launch_cast_scale_64_32(const double* in, float* out, double scale, int64_t n,
                                   hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cast_scale_kernel, dim3(vec_blocks(n, 8192)), dim3(kVecThreads), 0, s, n, in,
                     out, scale);
  return hipGetLastError();
}

__global__ void axpy_32_64_kernel(int64_t n, const float* __restrict__ in, double* __restrict__ out,
                                  double scale) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x)
    out[g] += scale * (double)in[g];
}
hipError_t launch_axpy_32_64(const float* in, double* out, double scale, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_32_64_kernel, dim3(vec_blocks(n, 8192)), dim3(kVecThreads), 0, s, n, in,
                     out, scale);
  return hipGetLastError();
}

template <typename T>
__global__ void fill_kernel(int64_t n, T* __restrict__ out, T v) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x)
    out[g] = v;
}
hipError_t launch_fill64(double* out, double v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((fill_kernel<double>), dim3(vec_blocks(n, 8192)), dim3(kVecThreads), 0, s, n,
                     out, v);
  return hipGetLastError();
}
hipError_t launch_fill32(float* out, float v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((fill_kernel<float>), dim3(vec_blocks(n, 8192)), dim3(kVecThreads), 0, s, n,
                     out, v);
  return hipGetLastError();
}

__global__ void recip_kernel(int64_t n, const double* __restrict__ diag, float* __restrict__ d32,
                             double* __restrict__ d64) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x) {
    const double v = 1.0 / diag[g];
    d64[g] = v;
    d32[g] = (float)v;
  }
}
hipError_t launch_recip_64_32(const double* diag, float* dinv32, double* dinv64, int64_t n,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(recip_kernel, dim3(vec_blocks(n, 8192)), dim3(kVecThreads), 0, s, n, diag,
                     dinv32, dinv64);
  return hipGetLastError();
}

// ------------------------------------------------------ face transform ----
// out_face = (A x A) (in_face [+ in2_face]) on n_p x n_p faces, A row-major
// (out[a] = sum_b A[a*n_p+b] in[b]) applied along both tangential axes.
template <typename T, int NP>
__global__ void __launch_bounds__(320)
face_transform_kernel(const T* __restrict__ A, const T* __restrict__ in, const T* __restrict__ in2,
                      T* __restrict__ out, int64_t n_faces) {
  constexpr int NF = NP * NP;
  constexpr int FPB = (256 / NF) > 0 ? 256 / NF : 1;
  __shared__ T s_in[FPB][NF];
  __shared__ T s_t[FPB][NF];
  const int slot = threadIdx.x / NF;
  const int lt = threadIdx.x - slot * NF;
  const int64_t f = (int64_t)blockIdx.x * FPB + slot;
  const bool active = slot < FPB && f < n_faces;
  if (active) {
    T v = in[f * NF + lt];
    if (in2) v += in2[f * NF + lt];
    s_in[slot][lt] = v;
  }
  __syncthreads();
  const int qa = lt % NP, qb = lt / NP;
  if (active) {
    // along the first tangential axis: t[a, c] = sum_b A[a,b] in[b, c]
    T acc = 0;
#pragma unroll
    for (int b = 0; b < NP; ++b) acc += A[qa * NP + b] * s_in[slot][b + NP * qb];
    s_t[slot][lt] = acc;
  }
  __syncthreads();
  if (active) {
    // along the second tangential axis: out[a, c] = sum_d A[c,d] t[a, d]
    T acc = 0;
#pragma unroll
    for (int dd = 0; dd < NP; ++dd) acc += A[qb * NP + dd] * s_t[slot][qa + NP * dd];
    out[f * NF + lt] = acc;
  }
}

template <typename T, int NP>
static hipError_t launch_ft_np(const T* A, const T* in, const T* in2, T* out, int64_t n_faces,
                               hipStream_t s) {
  constexpr int NF = NP * NP;
  constexpr int FPB = (256 / NF) > 0 ? 256 / NF : 1;
  const int64_t nb = (n_faces + FPB - 1) / FPB;
  if (nb == 0) return hipSuccess;
  constexpr int NTH = (FPB * NF + 63) / 64 * 64;
  hipLaunchKernelGGL((face_transform_kernel<T, NP>), dim3((unsigned)nb), dim3(NTH), 0, s, A, in,
                     in2, out, n_faces);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_face_transform(int np, const T* A, const T* in, const T* in2, T* out,
                                 int64_t n_faces, hipStream_t s) {
  switch (np) {
#define HDG_CASE(N) \
  case N: return launch_ft_np<T, N>(A, in, in2, out, n_faces, s);
    HDG_CASE(2) HDG_CASE(3) HDG_CASE(4) HDG_CASE(5) HDG_CASE(6) HDG_CASE(7) HDG_CASE(8)
    HDG_CASE(9) HDG_CASE(10) HDG_CASE(11) HDG_CASE(12) HDG_CASE(13) HDG_CASE(14)
    HDG_CASE(15) HDG_CASE(16) HDG_CASE(17)
#undef HDG_CASE
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_face_transform<double>(int, const double*, const double*, const double*,
                                                  double*, int64_t, hipStream_t);
template hipError_t launch_face_transform<float>(int, const float*, const float*, const float*,
                                                 float*, int64_t, hipStream_t);

// ------------------------------------------------------------ diagonal ----
// diag(K^) at a free face node: sum over the adjacent elements of
//   d_a H_ss - d_a^2 sum_q BS[q,s]^2 / (lambda d0 + d_a Lam[q] + d_b Lam[qb] + d_c Lam[qc])
// with s = 1 for the element below the face and s = 0 for the one above
// (paper: equation (hdg_op_east_east_transformed) and the diagonal
// preconditioner that follows it).  An interior face has two elements, a
// face of a Neumann side one.
__device__ inline double diag_share(const MeshDev& m, const ElemTab<double>& tab, int np, int a,
                                    int ei, int ej, int ek, int s, int qb, int qc) {
  const int64_t e = ei + (int64_t)m.n1 * (ej + (int64_t)m.n2 * ek);
  const double h1 = m.h1[ei], h2 = m.h2[ej], h3 = m.h3[ek];
  const double d0 = h1 * h2 * h3 * 0.125;
  const double dd[3] = {d0 * 4.0 / (h1 * h1), d0 * 4.0 / (h2 * h2), d0 * 4.0 / (h3 * h3)};
  const int b = (a == 0) ? 1 : 0;
  const int c = (a == 2) ? 1 : 2;
  const double base = d0 * m.lam[e] + dd[b] * tab.lam[qb] + dd[c] * tab.lam[qc];
  const double* bs = s ? tab.bs1 : tab.bs0;
  double sum = 0.0;
  for (int q = 0; q < np; ++q) sum += bs[q] * bs[q] / (base + dd[a] * tab.lam[q]);
  return dd[a] * (s ? tab.H11 : tab.H) - dd[a] * dd[a] * sum;
}

__global__ void __launch_bounds__(256)
diag_kernel(const MeshDev m, const ElemTab<double> tab, int np, double* __restrict__ diag) {
  const int nf = np * np;
  const int64_t n = m.n_free_faces * nf;
  const int nel[3] = {m.n1, m.n2, m.n3};
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t fid = g / nf;
    const int lt = (int)(g - fid * nf);
    const int qb = lt % np, qc = lt / np;
    double acc = 0.0;
    if (fid < m.n_int_faces) {
      int a, pl, ti, tj, tk;   // axis, plane, element indices (one replaced by plane)
      if (fid < m.foff[1]) {
        a = 0;
        int64_t loc = fid - m.foff[0];
        pl = (int)(loc % (m.n1 - 1)) + 1;
        loc /= (m.n1 - 1);
        tj = (int)(loc % m.n2);
        tk = (int)(loc / m.n2);
        ti = 0;
      } else if (fid < m.foff[2]) {
        a = 1;
        int64_t loc = fid - m.foff[1];
        ti = (int)(loc % m.n1);
        loc /= m.n1;
        pl = (int)(loc % (m.n2 - 1)) + 1;
        tk = (int)(loc / (m.n2 - 1));
        tj = 0;
      } else {
        a = 2;
        int64_t loc = fid - m.foff[2];
        ti = (int)(loc % m.n1);
        loc /= m.n1;
        tj = (int)(loc % m.n2);
        pl = (int)(loc / m.n2) + 1;
        tk = 0;
      }
      for (int side = 0; side < 2; ++side) {
        // side 0: element below (its high face, s = 1); side 1: element above (s = 0)
        const int ei = (a == 0) ? pl - 1 + side : ti;
        const int ej = (a == 1) ? pl - 1 + side : tj;
        const int ek = (a == 2) ? pl - 1 + side : tk;
        acc += diag_share(m, tab, np, a, ei, ej, ek, 1 - side, qb, qc);
      }
    } else {
      // a face of a Neumann side: find the side, then its one element
      int k = 0;
      for (; k < 5; ++k) {
        if (!((m.neumann >> k) & 1)) continue;
        const int a = k >> 1;
        const int64_t cnt = (int64_t)nel[a == 0 ? 1 : 0] * nel[a == 2 ? 1 : 2];
        if (fid >= m.boff[k] && fid < m.boff[k] + cnt) break;
      }
      const int a = k >> 1, s = k & 1;
      const int64_t loc = fid - m.boff[k];
      const int nb = nel[a == 0 ? 1 : 0];
      const int tb = (int)(loc % nb), tc = (int)(loc / nb);
      const int pos = s ? nel[a] - 1 : 0;
      const int ei = (a == 0) ? pos : tb;
      const int ej = (a == 1) ? pos : (a == 0 ? tb : tc);
      const int ek = (a == 2) ? pos : tc;
      acc = diag_share(m, tab, np, a, ei, ej, ek, s, qb, qc);
    }
    diag[g] = acc;
  }
}

hipError_t launch_diag(const hdg_ctx* c, double* diag, hipStream_t s) {
  const int64_t n = c->n_free;
  if (n == 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 65535) nb = 65535;
  hipLaunchKernelGGL(diag_kernel, dim3((unsigned)nb), dim3(256), 0, s, c->mesh, c->et64, c->np,
                     diag);
  return hipGetLastError();
}

}  // namespace hdg
