// Volume-source element kernels, FP64: right-hand side with the Dirichlet
// lift, recovery of u, and the adjoint gradients.  All use the element
// eigenspace of the fast diagonalisation (paper: section "Sum factorization
// of the HDG operator"), with S_e = S x S x S:
//
//   g   = S_e^T M_e f = d0 (S^T M x S^T M x S^T M) f        (forcing source)
//   g   = S_e^T r     = (S^T x S^T x S^T) r                 (adjoint source)
//   w   = D_Z^-1 (g - B^_e x)                               (x: eigen-basis trace)
//   RHS:      out_{a,s} = -d_a sum_q BS[q,s] w[..q..]       (free faces)
//   recovery: u_e = S_e w
//   adjoint:  a = D_Z^-1 (S_e^T r - B^_e mu),  u_E = D_Z^-1 (S_e^T M_e f - B^_e x)
//             dJ/dlambda_e = -d0 sum a u_E,  dJ/df_e = d0 (M S x M S x M S) a
//
// These run once per solve and cost O(n_p^4) per element (three 1D
// contractions of the n_p^3 cube held in LDS).  One element per block.
#include "device_common.hpp"

namespace hdg {

struct VolArgs {
  const double* f;        // forcing or adjoint source volume
  const double* x_free;   // eigen-basis trace, free faces (may be null = 0)
  const double* x_bdry;   // eigen-basis trace, boundary tail (may be null = 0)
  const double* r2;       // adjoint: dJ/du volume
  const double* mu_free;  // adjoint: eigen-basis adjoint trace
  double* qa;
  double* qb;
  double* out_vol;
  double* out_elem;
  const double* mats;     // St, StM, S, MS (row-major n_p x n_p each)
  int src_is_forcing;     // 1: g = d0 (S^T M)^3 f, 0: g = (S^T)^3 f
};

// cube <- scale * (A x A x A) cube, cube [q3][q2][q1]; NF threads, thread lt
// owns one line per pass.
template <int NP>
__device__ inline void cube_transform(double* cube, const double* __restrict__ A, double scale,
                                      int lt, bool active) {
  constexpr int NF = NP * NP;
#pragma unroll
  for (int axis = 0; axis < 3; ++axis) {
    int base = 0, stride = 1;
    if (axis == 0) { base = NP * lt; stride = 1; }
    else if (axis == 1) { base = (lt % NP) + NF * (lt / NP); stride = NP; }
    else { base = lt; stride = NF; }
    double v[NP];
    if (active) {
#pragma unroll
      for (int b = 0; b < NP; ++b) v[b] = cube[base + stride * b];
    }
    __syncthreads();
    if (active) {
      const double sc = (axis == 2) ? scale : 1.0;
#pragma unroll
      for (int a = 0; a < NP; ++a) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < NP; ++b) acc += A[a * NP + b] * v[b];
        cube[base + stride * a] = sc * acc;
      }
    }
    __syncthreads();
  }
}

template <int NP>
__device__ inline void load_faces(const MeshDev& m, int i, int j, int k, const double* x_free,
                                  const double* x_bdry, int lt, double* s_face, double* xf,
                                  int64_t* fid, bool* ffree) {
  constexpr int NF = NP * NP;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      bool fr;
      const int64_t f = face_of(m, a, s, i, j, k, &fr);
      fid[2 * a + s] = f;
      ffree[2 * a + s] = fr;
      double v = 0.0;
      if (fr) {
        if (x_free) v = x_free[f * NF + lt];
      } else if (x_bdry) {
        v = x_bdry[(f - m.n_free_faces) * NF + lt];
      }
      xf[2 * a + s] = v;
      s_face[(2 * a + s) * NF + lt] = v;
    }
}

// w = (cube - B^ x) / D_Z in place; returns the axis-2 reductions.
template <int NP>
__device__ inline void eig_solve(double* cube, const double* s_face, const double* d,
                                 const ElemTab<double>& tab, int lt, double* r2lo, double* r2hi) {
  constexpr int NF = NP * NP;
  const int q1 = lt % NP, q2 = lt / NP;
  const double c0 = d[1] * tab.bs0[q1], c1 = d[1] * tab.bs1[q1];
  const double c2 = d[2] * tab.bs0[q2], c3 = d[2] * tab.bs1[q2];
  const double x2lo = d[3] * s_face[4 * NF + lt], x2hi = d[3] * s_face[5 * NF + lt];
  const double dij = d[0] + d[1] * tab.lam[q1] + d[2] * tab.lam[q2];
  double lo = 0.0, hi = 0.0;
#pragma unroll
  for (int q3 = 0; q3 < NP; ++q3) {
    double F = c0 * s_face[0 * NF + q2 + NP * q3] + c1 * s_face[1 * NF + q2 + NP * q3] +
               c2 * s_face[2 * NF + q1 + NP * q3] + c3 * s_face[3 * NF + q1 + NP * q3] +
               tab.bs0[q3] * x2lo + tab.bs1[q3] * x2hi;
    const double w = (cube[lt + NF * q3] - F) / (dij + d[3] * tab.lam[q3]);
    cube[lt + NF * q3] = w;
    lo += tab.bs0[q3] * w;
    hi += tab.bs1[q3] * w;
  }
  *r2lo = lo;
  *r2hi = hi;
}

template <int NP, int MODE>
__global__ void __launch_bounds__(round_up64(NP * NP))
volume_kernel(const MeshDev mesh, const ElemTab<double> tab, VolArgs va) {
  constexpr int NF = NP * NP;
  constexpr int NV = NF * NP;
  constexpr int NT = round_up64(NF);
  // dynamic LDS: cube | cube2 (adjoint only) | faces | reduction scratch
  extern __shared__ double s_dyn[];
  double* s_cube = s_dyn;
  double* s_cube2 = s_dyn + NV;
  double* s_face = s_dyn + ((MODE == VOL_ADJ) ? 2 * NV : NV);
  double* s_red = s_face + 6 * NF;

  const int64_t e = blockIdx.x;
  const int lt = threadIdx.x;
  const bool active = lt < NF;
  const int i = (int)(e % mesh.n1);
  const int64_t rest = e / mesh.n1;
  const int j = (int)(rest % mesh.n2);
  const int k = (int)(rest / mesh.n2);
  const double h1 = mesh.h1[i], h2 = mesh.h2[j], h3 = mesh.h3[k];
  const double d0 = h1 * h2 * h3 * 0.125;
  const double d[4] = {d0 * mesh.lam[e], d0 * 4.0 / (h1 * h1), d0 * 4.0 / (h2 * h2),
                       d0 * 4.0 / (h3 * h3)};
  const double* St = va.mats;
  const double* StM = va.mats + NF;
  const double* S = va.mats + 2 * NF;
  const double* MS = va.mats + 3 * NF;

  // source cube(s)
  if (active) {
#pragma unroll
    for (int q3 = 0; q3 < NP; ++q3) {
      s_cube[lt + NF * q3] = va.f[e * NV + lt + NF * q3];
      if constexpr (MODE == VOL_ADJ) s_cube2[lt + NF * q3] = va.r2[e * NV + lt + NF * q3];
    }
  }
  __syncthreads();
  if (MODE == VOL_ADJ || va.src_is_forcing) cube_transform<NP>(s_cube, StM, d0, lt, active);
  else cube_transform<NP>(s_cube, St, 1.0, lt, active);
  if constexpr (MODE == VOL_ADJ) cube_transform<NP>(s_cube2, St, 1.0, lt, active);

  double xf[6];
  int64_t fid[6];
  bool ffree[6];
  double r2lo = 0.0, r2hi = 0.0;
  if (active) load_faces<NP>(mesh, i, j, k, va.x_free, va.x_bdry, lt, s_face, xf, fid, ffree);
  __syncthreads();
  if (active) eig_solve<NP>(s_cube, s_face, d, tab, lt, &r2lo, &r2hi);
  __syncthreads();

  if constexpr (MODE == VOL_RHS) {
    if (active) {
      double out[6];
      {
        const int q2 = lt % NP, q3 = lt / NP;
        const double* u = s_cube + NP * (q2 + NP * q3);
        double lo = 0.0, hi = 0.0;
#pragma unroll
        for (int q1 = 0; q1 < NP; ++q1) { lo += tab.bs0[q1] * u[q1]; hi += tab.bs1[q1] * u[q1]; }
        out[0] = -d[1] * lo;
        out[1] = -d[1] * hi;
      }
      {
        const int q1 = lt % NP, q3 = lt / NP;
        const double* u = s_cube + q1 + NF * q3;
        double lo = 0.0, hi = 0.0;
#pragma unroll
        for (int q2 = 0; q2 < NP; ++q2) { lo += tab.bs0[q2] * u[NP * q2]; hi += tab.bs1[q2] * u[NP * q2]; }
        out[2] = -d[2] * lo;
        out[3] = -d[2] * hi;
      }
      out[4] = -d[3] * r2lo;
      out[5] = -d[3] * r2hi;
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        if (!ffree[f]) continue;
        const int64_t g = fid[f] * NF + lt;
        if (f & 1) va.qa[g] = out[f];
        else va.qb[g] = out[f];
      }
    }
  } else if constexpr (MODE == VOL_RECON) {
    cube_transform<NP>(s_cube, S, 1.0, lt, active);
    if (active) {
#pragma unroll
      for (int q3 = 0; q3 < NP; ++q3) va.out_vol[e * NV + lt + NF * q3] = s_cube[lt + NF * q3];
    }
  } else {  // VOL_ADJ: adjoint cube a from (r2, mu); u_E already in s_cube
    if (active) load_faces<NP>(mesh, i, j, k, va.mu_free, nullptr, lt, s_face, xf, fid, ffree);
    __syncthreads();
    double t0, t1;
    if (active) eig_solve<NP>(s_cube2, s_face, d, tab, lt, &t0, &t1);
    __syncthreads();
    double acc = 0.0;
    if (active) {
#pragma unroll
      for (int q3 = 0; q3 < NP; ++q3) acc += s_cube2[lt + NF * q3] * s_cube[lt + NF * q3];
    }
    const double tot = block_sum<NT>(acc, s_red);
    if (threadIdx.x == 0) va.out_elem[e] = -d0 * tot;
    cube_transform<NP>(s_cube2, MS, d0, lt, active);
    if (active) {
#pragma unroll
      for (int q3 = 0; q3 < NP; ++q3) va.out_vol[e * NV + lt + NF * q3] = s_cube2[lt + NF * q3];
    }
  }
}

template <int NP, int MODE>
static hipError_t launch_vol_mode(const hdg_ctx* c, const VolArgs& va, hipStream_t s) {
  constexpr int NF = NP * NP, NV = NF * NP, NT = round_up64(NF);
  const size_t lds = sizeof(double) * ((MODE == VOL_ADJ ? 2 * NV : NV) + 6 * NF + NT / 64);
  static bool attr_set = false;     // per instantiation; the attribute is per function
  if (!attr_set && lds > 65536) {
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void*>(&volume_kernel<NP, MODE>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    attr_set = true;
  }
  hipLaunchKernelGGL((volume_kernel<NP, MODE>), dim3((unsigned)c->n_elem), dim3(NT), lds, s,
                     c->mesh, c->et64, va);
  return hipGetLastError();
}

template <int NP>
static hipError_t launch_vol_np(const hdg_ctx* c, int mode, const VolArgs& va, hipStream_t s) {
  if (c->n_elem == 0) return hipSuccess;
  if (mode == VOL_RHS) return launch_vol_mode<NP, VOL_RHS>(c, va, s);
  if (mode == VOL_RECON) return launch_vol_mode<NP, VOL_RECON>(c, va, s);
  return launch_vol_mode<NP, VOL_ADJ>(c, va, s);
}

hipError_t launch_volume(const hdg_ctx* c, int mode, int src_is_forcing, const double* f,
                         const double* x_free, const double* x_bdry, const double* r2,
                         const double* mu_free, double* qa, double* qb, double* out_vol,
                         double* out_elem, hipStream_t s) {
  VolArgs va{};
  va.f = f;
  va.x_free = x_free;
  va.x_bdry = x_bdry;
  va.r2 = r2;
  va.mu_free = mu_free;
  va.qa = qa;
  va.qb = qb;
  va.out_vol = out_vol;
  va.out_elem = out_elem;
  va.mats = c->d_mats64;
  va.src_is_forcing = src_is_forcing ? 1 : 0;
  switch (c->np) {
#define HDG_CASE(N) \
  case N: return launch_vol_np<N>(c, mode, va, s);
    HDG_CASE(2) HDG_CASE(3) HDG_CASE(4) HDG_CASE(5) HDG_CASE(6) HDG_CASE(7) HDG_CASE(8)
    HDG_CASE(9) HDG_CASE(10) HDG_CASE(11) HDG_CASE(12) HDG_CASE(13) HDG_CASE(14)
    HDG_CASE(15) HDG_CASE(16) HDG_CASE(17)
#undef HDG_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hdg
