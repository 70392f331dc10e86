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
// stored (the paper stored them; see its roofline discussion): the kernel is
// bound by memory and instruction issue, and the stored table would double
// the bytes per element at p = 7.
//
// Thread mapping: one thread per face-node column (q1,q2) of an element; it
// walks q3 and keeps the axis-2 reduction in registers, while u is staged in
// LDS for the axis-0 and axis-1 reductions.  For n_p >= 6 each element is
// owned by whole wavefronts (the element data is wave-uniform and read with
// scalar loads); for n_p <= 5 several elements share a wavefront.  Blocks
// loop over a contiguous range of elements so that the grid, and with it the
// number of reduction partials, stays bounded.
// Each interior face receives one contribution from the element below it
// (written to qa) and one from the element above it (qb): plain stores, no
// atomics, deterministic sums.
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

// a / b through the hardware reciprocal, two Newton steps and one residual
// correction (within about one ulp; no IEEE division sequence).
__device__ inline double div_fast(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  double e = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, e, r);
  const double q = a * r;
  return __builtin_fma(r, __builtin_fma(-b, q, a), q);
}
__device__ inline float div_fast(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// CG prologue shared by both mappings: read slot A, sum the update partials
// (r.z and r.r), decide convergence, publish slot B from block 0.
template <typename T, int NT>
__device__ inline void cg_prologue(const ApplyIO<T>& io, double* s_red, int* iter, T* beta,
                                   T* alpha_x, bool* finish, bool* skip) {
  if (io.sc->A.done) {                     // uniform over the grid
    *skip = true;
    return;
  }
  *skip = false;
  const int it = io.sc->A.iter;
  const double rho_prev = io.sc->A.rho;
  const double rtol2 = io.sc->A.rtol2;
  const int maxit = io.sc->A.maxit;
  double rr_stop = io.sc->A.rr_stop;
  *alpha_x = (T)io.sc->A.alpha;
  const int k2 = it & 1;
  double rho, rr;
  sum_partials2<NT>(io.partials + (size_t)(2 + k2) * io.pmax,
                    io.partials + (size_t)(4 + k2) * io.pmax, io.n_upd, s_red, &rho, &rr);
  if (it == 0) rr_stop = rtol2 * rr;
  const double b = (it == 0) ? 0.0 : rho / rho_prev;
  int done = 0;
  if (!isfinite(rr) || !isfinite(b)) done = 3;
  else if (rr <= rr_stop) done = 1;
  else if (it >= maxit) done = 2;
  *finish = done != 0;
  *beta = (T)b;
  *iter = it;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    io.sc->B.rho = rho;
    io.sc->B.rr = rr;
    io.sc->B.rr_stop = rr_stop;
    io.sc->B.iter = it;
    io.sc->B.maxit = maxit;
    io.sc->B.rtol2 = rtol2;
    io.sc->B.done = done;
  }
}

// =============================== group mapping ==============================
// n_p >= 6: each element is owned by a group of whole wavefronts (TPE
// threads, one face-node column per thread), EPB elements per block.  The
// element index is uniform over each wavefront, so the element data comes in
// through scalar loads.  Faces normal to x1 and x2 are staged in LDS; faces
// normal to x3 stay in registers.
template <int NP>
__host__ __device__ constexpr int tpe_for() { return round_up64(NP * NP); }
// u is stored as u[q1 + P (q2 + n_p q3)] with an odd row pitch P so that the
// axis-0 reduction (lanes stride P) is free of LDS bank conflicts
template <int NP>
__host__ __device__ constexpr int upitch() { return NP | 1; }
template <int NP>
__host__ __device__ constexpr int lds_elem_bytes() {
  return (4 * NP * NP + upitch<NP>() * NP * NP + 1) * 8;
}
template <int NP>
__host__ __device__ constexpr int epb_group() {
  constexpr int by_threads = (256 / tpe_for<NP>()) > 0 ? 256 / tpe_for<NP>() : 1;
  constexpr int by_lds = (60000 / lds_elem_bytes<NP>()) > 0 ? 60000 / lds_elem_bytes<NP>() : 1;
  constexpr int e = by_threads < by_lds ? by_threads : by_lds;
  return e > 4 ? 4 : e;
}

template <typename T, int NP, int MODE>   // MODE 0: plain apply, 1: fused CG apply
__global__ void __launch_bounds__(epb_group<NP>() * tpe_for<NP>())
elem_group_kernel(const MeshDev mesh, const ElemTab<T> tab, ApplyIO<T> io, int units_per_block) {
  constexpr int NF = NP * NP;
  constexpr int TPE = tpe_for<NP>();
  constexpr int EPB = epb_group<NP>();
  constexpr int NT = EPB * TPE;
  constexpr int P = upitch<NP>();
  constexpr int UP = P * NF + 1;
  __shared__ T s_face[EPB][4][NF];
  __shared__ T s_u[EPB][UP];
  __shared__ double s_red[NT / 64];

  T beta = 0, alpha_x = 0;
  int iter = 0;
  bool finish = false;
  if constexpr (MODE == 1) {
    bool skip;
    cg_prologue<T, NT>(io, s_red, &iter, &beta, &alpha_x, &finish, &skip);
    if (skip) return;
  }
  const T* p_in = (MODE == 1) ? ((iter & 1) ? io.p0 : io.p1) : nullptr;
  T* p_out = (MODE == 1) ? ((iter & 1) ? io.p1 : io.p0) : nullptr;

  const int slot = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / TPE));
  const int col = (int)(threadIdx.x % TPE);
  const bool colok = col < NF;
  const int q1 = col % NP, q2 = col / NP;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int nff = (int)mesh.n_free_faces;
  double dot = 0.0;

  for (int un = 0; un < units_per_block; ++un) {
    const int e = (bid * units_per_block + un) * EPB + slot;   // wave-uniform
    const bool active = e < mesh.n_elem;
    T d[4] = {0, 0, 0, 0};
    int fid[6];
    T xf[6];
    if (active) {
      const ElemInfo* ei = mesh.info + e;
      d[0] = (T)(ei->d[0] * mesh.lam[e]);
      d[1] = (T)ei->d[1];
      d[2] = (T)ei->d[2];
      d[3] = (T)ei->d[3];
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        fid[f] = ei->fid[f];
        const bool fr = fid[f] < nff;
        T v = 0;
        if (colok) {
          if (fr) {
            const int64_t g = (int64_t)fid[f] * NF + col;
            if constexpr (MODE == 0) {
              v = io.x_free[g];
            } else {
              const T pin = p_in[g];
              if (f & 1) io.x[g] += alpha_x * pin;   // the element below owns the face
              if (!finish) {
                v = io.dinv[g] * io.r[g] + beta * pin;
                if (f & 1) p_out[g] = v;
              }
            }
          } else if (MODE == 0 && io.x_bdry != nullptr) {
            v = io.x_bdry[(int64_t)(fid[f] - nff) * NF + col];
          }
          if (f < 4) s_face[slot][f][col] = v;
        }
        xf[f] = v;
      }
    }
    if constexpr (MODE == 1) {
      if (finish) continue;                // uniform: only the x update remains
    }
    __syncthreads();

    // expansion into the element eigenspace, division, axis-2 reduction
    T r2lo = 0, r2hi = 0;
    if (active && colok) {
      const T* f0lo = s_face[slot][0];
      const T* f0hi = s_face[slot][1];
      const T* f1lo = s_face[slot][2];
      const T* f1hi = s_face[slot][3];
      const T c0 = d[1] * tab.bs0[q1], c1 = d[1] * tab.bs1[q1];
      const T c2 = d[2] * tab.bs0[q2], c3 = d[2] * tab.bs1[q2];
      const T x2lo = d[3] * xf[4], x2hi = d[3] * xf[5];
      const T dij = d[0] + d[1] * tab.lam[q1] + d[2] * tab.lam[q2];
#pragma unroll
      for (int q3 = 0; q3 < NP; ++q3) {
        T F = c0 * f0lo[q2 + NP * q3];
        F += c1 * f0hi[q2 + NP * q3];
        F += c2 * f1lo[q1 + NP * q3];
        F += c3 * f1hi[q1 + NP * q3];
        F += tab.bs0[q3] * x2lo;
        F += tab.bs1[q3] * x2hi;
        const T u = div_fast(F, dij + d[3] * tab.lam[q3]);
        s_u[slot][q1 + P * (q2 + NP * q3)] = u;
        r2lo += tab.bs0[q3] * u;
        r2hi += tab.bs1[q3] * u;
      }
    }
    __syncthreads();

    // reductions back to the faces and the face-diagonal term
    if (active && colok) {
      T out[6];
      {
        // axis 0: face node (q2,q3) = col
        const T* u = s_u[slot] + P * col;
        T lo = 0, hi = 0;
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          lo += tab.bs0[a] * u[a];
          hi += tab.bs1[a] * u[a];
        }
        out[0] = d[1] * (tab.H * xf[0] - lo);
        out[1] = d[1] * (tab.H * xf[1] - hi);
      }
      {
        // axis 1: face node (q1,q3) = col
        const T* u = s_u[slot] + q1 + P * NP * q2;
        T lo = 0, hi = 0;
#pragma unroll
        for (int b = 0; b < NP; ++b) {
          lo += tab.bs0[b] * u[P * b];
          hi += tab.bs1[b] * u[P * b];
        }
        out[2] = d[2] * (tab.H * xf[2] - lo);
        out[3] = d[2] * (tab.H * xf[3] - hi);
      }
      out[4] = d[3] * (tab.H * xf[4] - r2lo);
      out[5] = d[3] * (tab.H * xf[5] - r2hi);
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        if (fid[f] >= nff) continue;
        const int64_t g = (int64_t)fid[f] * NF + col;
        if (f & 1) io.qa[g] = out[f];
        else io.qb[g] = out[f];
        if constexpr (MODE == 1) dot += (double)(xf[f] * out[f]);
      }
    }
    __syncthreads();                        // LDS is reused by the next unit
  }
  if constexpr (MODE == 1) {
    // p.q = sum_e p_e^T K_e p_e: element-local quadratic forms, one partial
    // per block, summed by every block of the update kernel.
    const double bs = block_sum<NT>(dot, s_red);
    if (threadIdx.x == 0) io.partials[(size_t)(iter & 1) * io.pmax + blockIdx.x] = bs;
  }
}

// ============================= packed mapping ===============================
// n_p <= 5: n_p^2 lanes per element, several elements per wavefront.
template <int NP>
__host__ __device__ constexpr int epb_packed() { return 256 / (NP * NP); }
template <int NP>
__host__ __device__ constexpr int packed_threads() { return round_up64(epb_packed<NP>() * NP * NP); }

template <typename T, int NP, int MODE>
__global__ void __launch_bounds__(packed_threads<NP>())
elem_packed_kernel(const MeshDev mesh, const ElemTab<T> tab, ApplyIO<T> io, int units_per_block) {
  constexpr int NF = NP * NP;
  constexpr int EPB = epb_packed<NP>();
  constexpr int NT = packed_threads<NP>();
  constexpr int P = upitch<NP>();
  constexpr int UP = P * NF + 1;
  __shared__ T s_face[EPB][4][NF];
  __shared__ T s_u[EPB][UP];
  __shared__ double s_red[NT / 64];

  T beta = 0, alpha_x = 0;
  int iter = 0;
  bool finish = false;
  if constexpr (MODE == 1) {
    bool skip;
    cg_prologue<T, NT>(io, s_red, &iter, &beta, &alpha_x, &finish, &skip);
    if (skip) return;
  }
  const T* p_in = (MODE == 1) ? ((iter & 1) ? io.p0 : io.p1) : nullptr;
  T* p_out = (MODE == 1) ? ((iter & 1) ? io.p1 : io.p0) : nullptr;

  const int tid = threadIdx.x;
  const int slot = tid / NF;
  const int lt = tid - slot * NF;
  const int q1 = lt % NP, q2 = lt / NP;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int nff = (int)mesh.n_free_faces;
  double dot = 0.0;

  for (int un = 0; un < units_per_block; ++un) {
    const int e = (bid * units_per_block + un) * EPB + slot;
    const bool active = (slot < EPB) && (e < mesh.n_elem);
    T d[4] = {0, 0, 0, 0};
    int fid[6];
    T xf[6];
    if (active) {
      const ElemInfo* ei = mesh.info + e;
      d[0] = (T)(ei->d[0] * mesh.lam[e]);
      d[1] = (T)ei->d[1];
      d[2] = (T)ei->d[2];
      d[3] = (T)ei->d[3];
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        fid[f] = ei->fid[f];
        T v = 0;
        if (fid[f] < nff) {
          const int64_t g = (int64_t)fid[f] * NF + lt;
          if constexpr (MODE == 0) {
            v = io.x_free[g];
          } else {
            const T pin = p_in[g];
            if (f & 1) io.x[g] += alpha_x * pin;
            if (!finish) {
              v = io.dinv[g] * io.r[g] + beta * pin;
              if (f & 1) p_out[g] = v;
            }
          }
        } else if (MODE == 0 && io.x_bdry != nullptr) {
          v = io.x_bdry[(int64_t)(fid[f] - nff) * NF + lt];
        }
        if (f < 4) s_face[slot][f][lt] = v;
        xf[f] = v;
      }
    }
    if constexpr (MODE == 1) {
      if (finish) continue;
    }
    __syncthreads();

    T r2lo = 0, r2hi = 0;
    if (active) {
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
        const T u = div_fast(F, dij + d[3] * tab.lam[q3]);
        s_u[slot][q1 + P * (q2 + NP * q3)] = u;
        r2lo += tab.bs0[q3] * u;
        r2hi += tab.bs1[q3] * u;
      }
    }
    __syncthreads();

    if (active) {
      T out[6];
      {
        const T* u = s_u[slot] + P * lt;
        T lo = 0, hi = 0;
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          lo += tab.bs0[a] * u[a];
          hi += tab.bs1[a] * u[a];
        }
        out[0] = d[1] * (tab.H * xf[0] - lo);
        out[1] = d[1] * (tab.H * xf[1] - hi);
      }
      {
        const T* u = s_u[slot] + q1 + P * NP * q2;
        T lo = 0, hi = 0;
#pragma unroll
        for (int b = 0; b < NP; ++b) {
          lo += tab.bs0[b] * u[P * b];
          hi += tab.bs1[b] * u[P * b];
        }
        out[2] = d[2] * (tab.H * xf[2] - lo);
        out[3] = d[2] * (tab.H * xf[3] - hi);
      }
      out[4] = d[3] * (tab.H * xf[4] - r2lo);
      out[5] = d[3] * (tab.H * xf[5] - r2hi);
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        if (fid[f] >= nff) continue;
        const int64_t g = (int64_t)fid[f] * NF + lt;
        if (f & 1) io.qa[g] = out[f];
        else io.qb[g] = out[f];
        if constexpr (MODE == 1) dot += (double)(xf[f] * out[f]);
      }
    }
    __syncthreads();
  }
  if constexpr (MODE == 1) {
    const double bs = block_sum<NT>(dot, s_red);
    if (tid == 0) io.partials[(size_t)(iter & 1) * io.pmax + blockIdx.x] = bs;
  }
}

// ================================ launch ====================================
constexpr int kApplyGridMax = 2048;

template <int NP>
constexpr bool use_group() { return NP >= 6; }

// units (elements handled concurrently by one block) and the block grid
template <int NP>
static void grid_np(int64_t n_elem, int* nblocks, int* units_per_block) {
  constexpr int E = use_group<NP>() ? epb_group<NP>() : epb_packed<NP>();
  const int64_t units = (n_elem + E - 1) / E;
  if (units == 0) {
    *nblocks = 0;
    *units_per_block = 0;
    return;
  }
  const int64_t g = units < kApplyGridMax ? units : kApplyGridMax;
  const int64_t upb = (units + g - 1) / g;
  *units_per_block = (int)upb;
  *nblocks = (int)((units + upb - 1) / upb);
}

template <typename T, int NP, int MODE>
static hipError_t launch_apply_np(const hdg_ctx* c, const ElemTab<T>& tab, const ApplyIO<T>& io,
                                  hipStream_t s) {
  int nb, upb;
  grid_np<NP>(c->n_elem, &nb, &upb);
  if (nb == 0) return hipSuccess;
  if constexpr (use_group<NP>()) {
    hipLaunchKernelGGL((elem_group_kernel<T, NP, MODE>), dim3(nb),
                       dim3(epb_group<NP>() * tpe_for<NP>()), 0, s, c->mesh, tab, io, upb);
  } else {
    hipLaunchKernelGGL((elem_packed_kernel<T, NP, MODE>), dim3(nb), dim3(packed_threads<NP>()), 0,
                       s, c->mesh, tab, io, upb);
  }
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

int elem_apply_blocks(int np, int64_t n_elem) {
  int nb = 0, upb = 0;
  switch (np) {
#define HDG_CASE(N) \
  case N: grid_np<N>(n_elem, &nb, &upb); break;
    HDG_CASE(2) HDG_CASE(3) HDG_CASE(4) HDG_CASE(5) HDG_CASE(6) HDG_CASE(7) HDG_CASE(8)
    HDG_CASE(9) HDG_CASE(10) HDG_CASE(11) HDG_CASE(12) HDG_CASE(13) HDG_CASE(14)
    HDG_CASE(15) HDG_CASE(16) HDG_CASE(17)
#undef HDG_CASE
    default: return 0;
  }
  return nb;
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

}  // namespace hdg
