// Volume-source element kernels, FP64: right-hand side with the Dirichlet
// lift, recovery of u, and the adjoint gradients.  All use the element
// eigenspace of the fast diagonalisation (paper: section "Sum factorization
// of the HDG operator"), with S_e = S x S x S:
//
//   g   = S_e^T M_e f = d0 (S^T M x S^T M x S^T M) f        (forcing source)
//   g   = S_e^T r     = (S^T x S^T x S^T) r                 (adjoint source)
//   w   = D_Z^-1 (g - B^_e x)                               (x: eigen-basis trace)
//   RHS:      out_{a,s} = -d_a sum_q BS[q,s] w[..q..] - d_a H01 x_{a,1-s}   (free faces)
//   recovery: u_e = S_e w
//   adjoint:  a = D_Z^-1 (S_e^T r - B^_e mu),  u_E = D_Z^-1 (S_e^T M_e f - B^_e x)
//             dJ/dlambda_e = -d0 sum a u_E,  dJ/df_e = d0 (M S x M S x M S) a
//
// On a face of a Neumann side the right-hand side also carries the face
// integral of mu g_N (the flux row of the element system); in the eigen
// basis that is (h_b h_c / 4) (S^T M x S^T M) g_N, the tail transform of the
// g_N block scaled by the face measure.
//
// The initial-guess flux (section "Summary of solution method", equation
// (fluxu)) of a volume field u with q = grad u: each element adds
//   (tau_e u - q.n + [g_N on a Neumann face]) / (tau_e + tau_neighbour)
// to each of its free faces, tau = 2 tau_hat / h_a, tau_neighbour = 0 on a
// Neumann face; q.n at a face node is (2s - 1) (2 / h_a) sum_k phi_k'(+-1)
// u_k along the normal line.
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
  double tau_hat;         // VOL_HYB: penalty scale
  double dend[2][kMaxNP]; // VOL_HYB: phi_k'(-1), phi_k'(+1) on the reference interval
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
__device__ inline void load_faces(const MeshDev& m, int64_t e, const double* x_free,
                                  const double* x_bdry, int lt, double* s_face, double* xf,
                                  int64_t* fid, bool* ffree, int* nm) {
  constexpr int NF = NP * NP;
  const ElemInfo* ei = m.info + e;
  *nm = ei->nmask;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int64_t id = ei->fid[f];
    const bool fr = id < m.n_free_faces;
    fid[f] = id;
    ffree[f] = fr;
    double v = 0.0;
    if (fr) {
      if (x_free) v = x_free[id * NF + lt];
    } else if (x_bdry) {
      v = x_bdry[(id - m.n_free_faces) * NF + lt];
    }
    xf[f] = v;
    s_face[f * NF + lt] = v;
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

// VOL_HYB: the initial-guess flux contributions of element e (cube = u_e in
// LDS, loaded and synchronised by the caller).  Thread lt holds face node lt
// of every face: (q2,q3), (q1,q3), (q1,q2) for the faces normal to x1, x2, x3.
template <int NP>
__device__ inline void hyb_faces(const MeshDev& m, const VolArgs& va, int64_t e, int i, int j,
                                 int k, const double* cube, int lt, bool active) {
  constexpr int NF = NP * NP;
  if (!active) return;
  const ElemInfo* ei = m.info + e;
  const int nm = ei->nmask;
  const int idx[3] = {i, j, k};
  const int nel[3] = {m.n1, m.n2, m.n3};
  const double* hs[3] = {m.h1, m.h2, m.h3};
  const int r = lt % NP, t = lt / NP;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int base, stride;
    if (a == 0) { base = NP * lt; stride = 1; }
    else if (a == 1) { base = r + NF * t; stride = NP; }
    else { base = lt; stride = NF; }
    double line[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) line[q] = cube[base + stride * q];
    const double h = hs[a][idx[a]];
    const double tau_e = 2.0 * va.tau_hat / h;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int f = 2 * a + s;
      const int64_t id = ei->fid[f];
      if (id >= m.n_free_faces) continue;
      double der = 0.0;
#pragma unroll
      for (int q = 0; q < NP; ++q) der += va.dend[s][q] * line[q];
      const double qn = (s ? 1.0 : -1.0) * (2.0 / h) * der;
      double num = tau_e * line[s ? NP - 1 : 0] - qn;
      double den = tau_e;
      const bool neu = (nm >> f) & 1;
      if (neu) {
        if (va.x_bdry) num += va.x_bdry[(m.n_dir_faces + id - m.n_int_faces) * NF + lt];
      } else {
        const int nb = idx[a] + (s ? 1 : -1);
        if (nb >= 0 && nb < nel[a]) den += 2.0 * va.tau_hat / hs[a][nb];
      }
      const int64_t g = id * NF + lt;
      const double v = num / den;
      if (s) va.qa[g] = v;
      else va.qb[g] = v;
      if (neu) {
        if (s) va.qb[g] = 0.0;
        else va.qa[g] = 0.0;
      }
    }
  }
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
  if constexpr (MODE == VOL_HYB) {
    hyb_faces<NP>(mesh, va, e, i, j, k, s_cube, lt, active);
    return;
  }
  if (MODE == VOL_ADJ || va.src_is_forcing) cube_transform<NP>(s_cube, StM, d0, lt, active);
  else cube_transform<NP>(s_cube, St, 1.0, lt, active);
  if constexpr (MODE == VOL_ADJ) cube_transform<NP>(s_cube2, St, 1.0, lt, active);

  double xf[6];
  int64_t fid[6];
  bool ffree[6];
  int nm = 0;
  double r2lo = 0.0, r2hi = 0.0;
  if (active) load_faces<NP>(mesh, e, va.x_free, va.x_bdry, lt, s_face, xf, fid, ffree, &nm);
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
      const double hh[3] = {h1, h2, h3};
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        if (!ffree[f]) continue;
        const int64_t g = fid[f] * NF + lt;
        // the face term of the lift: with the exact mass H couples the face
        // with the opposite one, which may hold Dirichlet data (xf of a free
        // face is zero here)
        double v = out[f] - d[1 + (f >> 1)] * tab.H01 * xf[f ^ 1];
        const bool neu = (nm >> f) & 1;
        if (neu && va.x_bdry) {   // face integral of mu g_N, eigen basis
          const int a = f >> 1;
          const double area = 0.25 * hh[a == 0 ? 1 : 0] * hh[a == 2 ? 1 : 2];
          v += area * va.x_bdry[(mesh.n_dir_faces + fid[f] - mesh.n_int_faces) * NF + lt];
        }
        if (f & 1) va.qa[g] = v;
        else va.qb[g] = v;
        if (neu) {
          if (f & 1) va.qb[g] = 0.0;
          else va.qa[g] = 0.0;
        }
      }
    }
  } else if constexpr (MODE == VOL_RECON) {
    cube_transform<NP>(s_cube, S, 1.0, lt, active);
    if (active) {
#pragma unroll
      for (int q3 = 0; q3 < NP; ++q3) va.out_vol[e * NV + lt + NF * q3] = s_cube[lt + NF * q3];
    }
  } else {  // VOL_ADJ: adjoint cube a from (r2, mu); u_E already in s_cube
    if (active) load_faces<NP>(mesh, e, va.mu_free, nullptr, lt, s_face, xf, fid, ffree, &nm);
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
  if (mode == VOL_HYB) return launch_vol_mode<NP, VOL_HYB>(c, va, s);
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
  va.tau_hat = c->tau;
  for (int q = 0; q < c->np; ++q) {   // phi_q'(x_i) = D_iq / w_i at the end nodes
    va.dend[0][q] = c->tab.D[q] / c->tab.w[0];
    va.dend[1][q] = c->tab.D[(c->np - 1) * c->np + q] / c->tab.w[c->np - 1];
  }
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
