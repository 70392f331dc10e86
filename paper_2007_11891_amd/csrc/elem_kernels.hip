// Element kernels of the condensed HDG operator in the eigen-face basis
// (paper: algorithm "HDG_Op_3D" for the transformed basis, section "Product
// factorization of the HDG operator").  Per element e with transformed faces
// x_{a,s} (axis a, side s) and metric factors d_0..d_3:
//
//   F[q1,q2,q3] = d1 sum_s BS[q1,s] x_{0,s}[q2,q3] + d2 sum_s BS[q2,s] x_{1,s}[q1,q3]
//               + d3 sum_s BS[q3,s] x_{2,s}[q1,q2]
//   u[q]        = F[q] / (lambda d0 + d1 Lam[q1] + d2 Lam[q2] + d3 Lam[q3])
//   r_{0,s}[q2,q3] = d1 H x_{0,s} - d1 sum_q1 BS[q1,s] u[q1,q2,q3]   (same for axes 1, 2)
//
// The inverse eigenvalues are recomputed in the kernel instead of being
// stored (the paper stored them; see its roofline discussion).
//
// Thread mapping: n_p^2 threads per element, thread (q1,q2) walks q3 and
// keeps the axis-2 reduction in registers; the element's u is staged in LDS
// for the axis-0 and axis-1 reductions.  Each interior face receives one
// contribution from the element below it (written to qa) and one from the
// element above it (qb): plain stores, no atomics, deterministic sums.
#include "device_common.hpp"

namespace hdg {

template <typename T>
struct ApplyIO {
  const T* x_free;   // plain mode: input on free faces
  const T* x_bdry;   // plain mode: input on boundary faces (tail), may be null
  T* qa;
  T* qb;
  // fused CG mode
  const T* r;
  const T* dinv;
  T* p0;
  T* p1;
  T* x;
  double* partials;  // pq[2][pmax] | rz[2][pmax] | rr[2][pmax]
  int pmax;
  int n_upd;         // number of update-kernel partials
  CgScalars* sc;
};

template <typename T>
__device__ inline T elem_div(T a, T b) { return a / b; }

// Geometry of element e: metric factors (paper, section "LDG operator
// structure in three dimensions") and lambda d0.
template <typename T>
__device__ inline void elem_metric(const MeshDev& m, int i, int j, int k, int64_t e, T* d) {
  const double h1 = m.h1[i], h2 = m.h2[j], h3 = m.h3[k];
  const double d0 = h1 * h2 * h3 * 0.125;
  d[0] = (T)(d0 * m.lam[e]);
  d[1] = (T)(d0 * (2.0 / h1) * (2.0 / h1));
  d[2] = (T)(d0 * (2.0 / h2) * (2.0 / h2));
  d[3] = (T)(d0 * (2.0 / h3) * (2.0 / h3));
}

template <typename T, int NP, int MODE>   // MODE 0: plain apply, 1: fused CG apply
__global__ void __launch_bounds__(elem_block_threads(NP))
elem_apply_kernel(const MeshDev mesh, const ElemTab<T> tab, ApplyIO<T> io) {
  constexpr int NF = NP * NP;
  constexpr int EPB = epb_for(NP);
  constexpr int NT = elem_block_threads(NP);
  constexpr int UP = NP * NP * NP + 1;     // u cube pitch per element (odd)
  __shared__ T s_face[EPB][6][NF];
  __shared__ T s_u[EPB][UP];
  __shared__ double s_red[NT / 64];

  T beta = 0, alpha_x = 0;
  int iter = 0;
  bool finish = false;     // converged / capped: only the last x update remains
  if constexpr (MODE == 1) {
    // scalar reads of slot A (a struct copy here costs a large serialisation)
    if (io.sc->A.done) return;             // uniform over the grid
    iter = io.sc->A.iter;
    const double rho_prev = io.sc->A.rho;
    const double rtol2 = io.sc->A.rtol2;
    const int maxit = io.sc->A.maxit;
    double rr_stop = io.sc->A.rr_stop;
    alpha_x = (T)io.sc->A.alpha;
    const int k2 = iter & 1;
    const double* prz = io.partials + (size_t)(2 + k2) * io.pmax;
    const double* prr = io.partials + (size_t)(4 + k2) * io.pmax;
    double rho, rr;
    sum_partials2<NT>(prz, prr, io.n_upd, s_red, &rho, &rr);
    if (iter == 0) rr_stop = rtol2 * rr;
    const double b = (iter == 0) ? 0.0 : rho / rho_prev;
    int done = 0;
    if (!isfinite(rr) || !isfinite(b)) done = 3;
    else if (rr <= rr_stop) done = 1;
    else if (iter >= maxit) done = 2;
    finish = done != 0;
    beta = (T)b;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      io.sc->B.rho = rho;
      io.sc->B.rr = rr;
      io.sc->B.rr_stop = rr_stop;
      io.sc->B.iter = iter;
      io.sc->B.maxit = maxit;
      io.sc->B.rtol2 = rtol2;
      io.sc->B.done = done;
    }
  }
  // search directions ping-pong: iteration k reads p_{k-1} and writes p_k
  const T* p_in = (MODE == 1) ? ((iter & 1) ? io.p0 : io.p1) : nullptr;
  T* p_out = (MODE == 1) ? ((iter & 1) ? io.p1 : io.p0) : nullptr;
  const int tid = threadIdx.x;
  const int slot = tid / NF;
  const int lt = tid - slot * NF;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t e = (int64_t)bid * EPB + slot;
  const bool active = (slot < EPB) && (e < mesh.n_elem);

  int i = 0, j = 0, k = 0;
  T d[4] = {0, 0, 0, 0};
  int64_t fid[6];
  bool ffree[6];
  T xf[6];
  if (active) {
    i = (int)(e % mesh.n1);
    const int64_t rest = e / mesh.n1;
    j = (int)(rest % mesh.n2);
    k = (int)(rest / mesh.n2);
    elem_metric<T>(mesh, i, j, k, e, d);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        bool fr;
        const int64_t f = face_of(mesh, a, s, i, j, k, &fr);
        fid[2 * a + s] = f;
        ffree[2 * a + s] = fr;
        T v = 0;
        if (fr) {
          const int64_t g = f * NF + lt;
          if constexpr (MODE == 0) {
            v = io.x_free[g];
          } else {
            const T pin = p_in[g];
            if (s == 1) io.x[g] += alpha_x * pin;   // the element below the face owns it
            if (!finish) {
              v = io.dinv[g] * io.r[g] + beta * pin;
              if (s == 1) p_out[g] = v;
            }
          }
        } else if (MODE == 0 && io.x_bdry != nullptr) {
          v = io.x_bdry[(f - mesh.n_free_faces) * NF + lt];
        }
        xf[2 * a + s] = v;
        s_face[slot][2 * a + s][lt] = v;
      }
  }
  if constexpr (MODE == 1) {
    if (finish) return;                    // uniform: every block took the same decision
  }
  __syncthreads();

  // ---- expansion into the element eigenspace, division, axis-2 reduction --
  T r2lo = 0, r2hi = 0;
  if (active) {
    const int q1 = lt % NP, q2 = lt / NP;
    const T c0 = d[1] * tab.bs0[q1], c1 = d[1] * tab.bs1[q1];
    const T c2 = d[2] * tab.bs0[q2], c3 = d[2] * tab.bs1[q2];
    const T x2lo = d[3] * xf[4], x2hi = d[3] * xf[5];
    const T dij = d[0] + d[1] * tab.lam[q1] + d[2] * tab.lam[q2];
    const T* f0lo = s_face[slot][0];
    const T* f0hi = s_face[slot][1];
    const T* f1lo = s_face[slot][2];
    const T* f1hi = s_face[slot][3];
#pragma unroll
    for (int q3 = 0; q3 < NP; ++q3) {
      T F = c0 * f0lo[q2 + NP * q3];
      F += c1 * f0hi[q2 + NP * q3];
      F += c2 * f1lo[q1 + NP * q3];
      F += c3 * f1hi[q1 + NP * q3];
      F += tab.bs0[q3] * x2lo;
      F += tab.bs1[q3] * x2hi;
      const T u = elem_div<T>(F, dij + d[3] * tab.lam[q3]);
      s_u[slot][lt + NF * q3] = u;
      r2lo += tab.bs0[q3] * u;
      r2hi += tab.bs1[q3] * u;
    }
  }
  __syncthreads();

  // ---- reductions back to the faces and the face-diagonal term ----------
  double dot = 0.0;
  if (active) {
    T out[6];
    {
      // axis 0: face node (q2,q3) = lt
      const int q2 = lt % NP, q3 = lt / NP;
      const T* u = s_u[slot] + NP * (q2 + NP * q3);
      T lo = 0, hi = 0;
#pragma unroll
      for (int q1 = 0; q1 < NP; ++q1) {
        lo += tab.bs0[q1] * u[q1];
        hi += tab.bs1[q1] * u[q1];
      }
      out[0] = d[1] * (tab.H * xf[0] - lo);
      out[1] = d[1] * (tab.H * xf[1] - hi);
    }
    {
      // axis 1: face node (q1,q3) = lt
      const int q1 = lt % NP, q3 = lt / NP;
      const T* u = s_u[slot] + q1 + NF * q3;
      T lo = 0, hi = 0;
#pragma unroll
      for (int q2 = 0; q2 < NP; ++q2) {
        lo += tab.bs0[q2] * u[NP * q2];
        hi += tab.bs1[q2] * u[NP * q2];
      }
      out[2] = d[2] * (tab.H * xf[2] - lo);
      out[3] = d[2] * (tab.H * xf[3] - hi);
    }
    out[4] = d[3] * (tab.H * xf[4] - r2lo);
    out[5] = d[3] * (tab.H * xf[5] - r2hi);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      if (!ffree[f]) continue;
      const int64_t g = fid[f] * NF + lt;
      if (f & 1) io.qa[g] = out[f];
      else io.qb[g] = out[f];
      if constexpr (MODE == 1) dot += (double)(xf[f] * out[f]);
    }
  }

  if constexpr (MODE == 1) {
    // p.q = sum_e p_e^T K_e p_e: element-local quadratic forms, one partial
    // per block, summed by every block of the update kernel.
    const double bs = block_sum<NT>(dot, s_red);
    if (tid == 0) io.partials[(size_t)(iter & 1) * io.pmax + blockIdx.x] = bs;
  }
}

template <typename T, int NP, int MODE>
static hipError_t launch_apply_np(const hdg_ctx* c, const ElemTab<T>& tab, const ApplyIO<T>& io,
                                  hipStream_t s) {
  constexpr int EPB = epb_for(NP);
  const int nb = (int)((c->n_elem + EPB - 1) / EPB);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL((elem_apply_kernel<T, NP, MODE>), dim3(nb), dim3(elem_block_threads(NP)), 0,
                     s, c->mesh, tab, io);
  return hipGetLastError();
}

template <typename T, int MODE>
static hipError_t launch_apply_dispatch(const hdg_ctx* c, const ElemTab<T>& tab,
                                        const ApplyIO<T>& io, hipStream_t s) {
  switch (c->np) {
#define HDG_CASE(N) \
  case N: return launch_apply_np<T, N, MODE>(c, tab, io, s);
    HDG_CASE(2) HDG_CASE(3) HDG_CASE(4) HDG_CASE(5) HDG_CASE(6) HDG_CASE(7) HDG_CASE(8)
    HDG_CASE(9) HDG_CASE(10) HDG_CASE(11) HDG_CASE(12) HDG_CASE(13) HDG_CASE(14)
    HDG_CASE(15) HDG_CASE(16) HDG_CASE(17)
#undef HDG_CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
static const ElemTab<T>& tab_of(const hdg_ctx* c);
template <>
const ElemTab<double>& tab_of<double>(const hdg_ctx* c) { return c->et64; }
template <>
const ElemTab<float>& tab_of<float>(const hdg_ctx* c) { return c->et32; }

template <typename T>
hipError_t launch_elem_apply(const hdg_ctx* c, const T* x_free, const T* x_bdry, T* qa, T* qb,
                             hipStream_t s) {
  ApplyIO<T> io{};
  io.x_free = x_free;
  io.x_bdry = x_bdry;
  io.qa = qa;
  io.qb = qb;
  return launch_apply_dispatch<T, 0>(c, tab_of<T>(c), io, s);
}

template <typename T>
hipError_t launch_cg_apply(const hdg_ctx* c, CgWork<T>& w, hipStream_t s) {
  ApplyIO<T> io{};
  io.qa = w.qa;
  io.qb = w.qb;
  io.r = w.r;
  io.dinv = w.dinv;
  io.p0 = w.p[0];
  io.p1 = w.p[1];
  io.x = w.x;
  io.partials = w.partials;
  io.pmax = w.pmax;
  io.n_upd = w.update_blocks;
  io.sc = w.sc;
  return launch_apply_dispatch<T, 1>(c, tab_of<T>(c), io, s);
}

template hipError_t launch_elem_apply<double>(const hdg_ctx*, const double*, const double*,
                                              double*, double*, hipStream_t);
template hipError_t launch_elem_apply<float>(const hdg_ctx*, const float*, const float*, float*,
                                             float*, hipStream_t);
template hipError_t launch_cg_apply<double>(const hdg_ctx*, CgWork<double>&, hipStream_t);
template hipError_t launch_cg_apply<float>(const hdg_ctx*, CgWork<float>&, hipStream_t);

int elem_threads(int np, int* epb) {
  *epb = epb_for(np);
  return elem_block_threads(np);
}

}  // namespace hdg
