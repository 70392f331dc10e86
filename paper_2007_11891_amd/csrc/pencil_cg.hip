// Pencil form of the two-kernel CG (solver HDG-trans: Jacobi-preconditioned
// CG on the transformed condensed operator of algorithm "HDG_Op_3D" in the
// eigen-face basis; paper, sections "Product factorization of the HDG
// operator" and "Summary of solution method"), on the march of
// pencil_unit.hpp: each block marches its columns up x3 through a segment of
// `ks` elements.  Blocks of one XCD work on neighbouring rows of the same
// segment, so the faces they share are read while they sit in that XCD's L2.
//
// Iteration k, element launch: beta_k from the update's r.z partials,
//   p_k = z_k + beta_k p_{k-1},  x += alpha_{k-1} p_{k-1}  (faces it owns),
//   w = K^ p_k  (qa / qb, or the x3 sum in qa),  p_k . w partial per block.
// Update launch: alpha_k = rho_k / (p_k . w), z -= alpha_k D^-1 w,
//   r.z and r.r partials.  The element launch that finds the solve finished
// applies the last x update (x_k = x_{k-1} + alpha_{k-1} p_{k-1}) and stops.
#include <algorithm>

#include "cg_state.hpp"
#include "pencil_unit.hpp"

namespace hdg {

template <typename T>
struct PencilIO {
  const T* z;
  T* p0;              // iteration k reads p_{k-1} from p[(k - 1) & 1] and
  T* p1;              // writes p_k to p[k & 1]
  T* x;
  T* qa;
  T* qb;
  double* partials;   // pq[2][pmax] | rz[2][pmax] | rr[2][pmax]
  int pmax;
  int n_upd;          // partials written by the update launch
  CgScalars* sc;
  int ks;             // elements per segment along x3
  int n_ig;           // slot groups along x1
  int n_seg;          // segments along x3
};

// Elements owned by whole wavefronts: at most 128 VGPRs (four waves per
// SIMD), so that enough blocks per CU are in flight to cover the memory
// latency; elements packed several per wavefront keep more registers per
// lane (their face bookkeeping is per lane).
template <int NP>
constexpr int pencil_min_waves() { return is_group<NP>() ? 4 : 2; }

template <typename T, int NP, int EPB>
__global__ void __launch_bounds__((unit_threads<NP, EPB>()))
__attribute__((amdgpu_waves_per_eu(pencil_min_waves<NP>())))
pencil_apply_kernel(const MeshDev mesh, const ElemTab<T> tab, PencilIO<T> io) {
  constexpr int NT = unit_threads<NP, EPB>();
  __shared__ PencilSmem<T, NP, EPB> sm;
  __shared__ double s_red[NT / 64];
  int iter;
  if (cg_head(io.sc, &iter)) return;
  // block -> (slot group along x1, row along x2, segment along x3), with the
  // XCD remap keeping neighbouring rows of one segment on one XCD
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int ig = bid % io.n_ig;
  const int j = (bid / io.n_ig) % mesh.n2;
  const int seg = bid / (io.n_ig * mesh.n2);
  const int k0 = seg * io.ks;
  const int k1 = min(k0 + io.ks, mesh.n3);
  const UnitLane Ln = unit_lane<NP, EPB>((int)threadIdx.x);
  const int i = ig * EPB + Ln.slot;
  const bool act = Ln.slot < EPB && i < mesh.n1 && Ln.colok;
  const T* __restrict__ z = io.z;
  const T* __restrict__ pin = (iter & 1) ? io.p0 : io.p1;   // p_{k-1}
  T* __restrict__ pout = (iter & 1) ? io.p1 : io.p0;        // p_k
  T* __restrict__ x = io.x;
  T* __restrict__ qa = io.qa;
  T* __restrict__ qb = io.qb;
  const int ic = min(i, mesh.n1 - 1);       // idle slots past the end of x1 mirror the last
  const int rowe = mesh.n1 * j + ic;        // element index at k = 0
  const int plane = mesh.n1 * mesh.n2;

  // the first element's loads go out with the partials' loads
  PencilRow row;
  pencil_row(mesh, ic, j, row);
  PencilLoads<T> L;
  pencil_load<T, NP>(mesh, z, pin, x, row, k0, act, Ln.col, rowe + plane * k0, true, L);
  const int k2 = iter & 1;
  const double* pp[2] = {io.partials + (size_t)(2 + k2) * io.pmax,
                         io.partials + (size_t)(4 + k2) * io.pmax};
  PartialSums<NT, 2> ps;
  ps.issue(pp, io.n_upd);
  if (threadIdx.x < NP) {
    sm.bs[threadIdx.x] = PencilPair<T>{tab.bs0[threadIdx.x], tab.bs1[threadIdx.x]};
    sm.lam[threadIdx.x] = tab.lam[threadIdx.x];
  }
  bool skip;
  T beta;
  cg_scalars<T, NT>(io.sc, io.n_upd, iter, ps, pp, &beta, &skip);
  const T alpha = (T)io.sc->A.alpha;      // alpha_{k-1} (0 before the first update)
  if (skip) {
    // the solve ended at iterate k: x_k = x_{k-1} + alpha_{k-1} p_{k-1}
    pencil_final_x<T, NP>(mesh, row, act, Ln.col, k0, k1, alpha, pin, x);
    return;
  }
  const T H = tab.H, H11 = tab.H11, H01 = tab.H01;
  T carry_p = 0, carry_w = 0;
  double dot = 0.0;
  // past the end of the segment the prefetch reloads the last element
  // (cache hits), so that no load sits behind a branch
  for (int k = k0; k < k1; ++k) {
    const int kn = min(k + 1, k1 - 1);
    pencil_step<T, NP, EPB>(z, pin, pout, x, qa, qb, sm, Ln, act, mesh, row, k, kn,
                            rowe + plane * kn, L, k == k0, k + 1 == k1, alpha, beta, H, H11, H01,
                            carry_p, carry_w, &dot);
  }
  // p_k . K^ p_k from the element-local quadratic forms, one partial per block
  const double bs = block_sum<NT>(dot, s_red);
  if (threadIdx.x == 0) io.partials[(size_t)(iter & 1) * io.pmax + blockIdx.x] = bs;
}

// ================================ update ====================================
constexpr int kPencilVecThreads = 256;
// eight entries per thread in flight (four streams each): with fewer, the
// update's loads per wave do not cover the HBM latency at 512 blocks
constexpr int kPencilUnroll = 8;

// Update of iteration k: alpha_k = rho_k / (p_k . w) with p.w summed from the
// element launch's partials; z -= alpha_k D^-1 w with w = qa + qb, except on
// the faces normal to x3 inside a segment, whose qa already holds the sum;
// r.z and r.r partials for the next element launch.  Block 0 publishes A.
// x3-face DOFs are [x3_lo, x3_hi), in planes of plane_dofs values; plane
// pl = 1 .. n3 - 1 lies on a segment boundary when pl % ks == 0.  32-bit
// offsets within that range (the element launch needs them anyway).
template <typename T>
__global__ void __launch_bounds__(kPencilVecThreads)
pencil_update_kernel(int64_t n, const T* __restrict__ qa, const T* __restrict__ qb,
                     T* __restrict__ z, const T* __restrict__ dinv, double* __restrict__ partials,
                     int pmax, int n_apply, CgScalars* sc, int64_t x3_lo, int64_t x3_hi,
                     uint32_t plane_dofs, float inv_plane, uint32_t ks, float inv_ks) {
  const int done = sc->B.done;
  if (done) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->A.done = done;
      sc->A.rr = sc->B.rr;
      sc->A.iter = sc->B.iter;
    }
    return;
  }
  const int k = sc->B.iter;
  const double rho = sc->B.rho;
  const int64_t stride = (int64_t)gridDim.x * kPencilVecThreads;
  int64_t g0 = (int64_t)blockIdx.x * kPencilVecThreads + threadIdx.x;
  T va[kPencilUnroll], vb[kPencilUnroll], vz[kPencilUnroll], vd[kPencilUnroll];
  // plane q = r / plane_dofs and (q + 1) mod ks by float estimates corrected
  // in 32-bit integers (r < 2^31: the estimate is within one of the quotient)
  auto need_b = [&](int64_t g) -> bool {
    if (g < x3_lo || g >= x3_hi) return true;
    const uint32_t r = (uint32_t)(g - x3_lo);
    uint32_t q = (uint32_t)((float)r * inv_plane);
    if (q * plane_dofs > r) --q;
    else if ((q + 1) * plane_dofs <= r) ++q;
    const uint32_t m = q + 1;
    uint32_t t = (uint32_t)((float)m * inv_ks);
    if (t * ks > m) --t;
    else if ((t + 1) * ks <= m) ++t;
    return m == t * ks;
  };
  auto load = [&](int64_t base) {
#pragma unroll
    for (int u = 0; u < kPencilUnroll; ++u) {
      const int64_t g = base + u * stride;
      vb[u] = 0;
      if (g < n) {
        va[u] = qa[g];
        if (need_b(g)) vb[u] = qb[g];
        vz[u] = z[g];
        vd[u] = dinv[g];
      }
    }
  };
  const double* pp[1] = {partials + (size_t)(k & 1) * pmax};
  PartialSums<kPencilVecThreads, 1> ps;
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
      sc->A.iter = k;
    }
    return;
  }
  const T a = (T)alpha;
  T rz_t = 0, rr_t = 0;
  for (; g0 < n; g0 += kPencilUnroll * stride) {
#pragma unroll
    for (int u = 0; u < kPencilUnroll; ++u) {
      const int64_t g = g0 + u * stride;
      if (g < n) {
        const T zn = vz[u] - a * (vd[u] * (va[u] + vb[u]));
        z[g] = zn;
        const T rn = div_fast(zn, vd[u]);
        rz_t += zn * rn;
        rr_t += rn * rn;
      }
    }
    if (g0 + kPencilUnroll * stride < n) load(g0 + kPencilUnroll * stride);
  }
  double sums[2] = {(double)rz_t, (double)rr_t};
  block_sums<kPencilVecThreads, 2>(sums);
  const int k1 = (k + 1) & 1;
  if (threadIdx.x == 0) {
    partials[(size_t)(2 + k1) * pmax + blockIdx.x] = sums[0];
    partials[(size_t)(4 + k1) * pmax + blockIdx.x] = sums[1];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->A.rho = rho;
    sc->A.alpha = alpha;
    sc->A.pq = pq;
    sc->A.rr_stop = sc->B.rr_stop;
    sc->A.rr = sc->B.rr;
    sc->A.iter = k + 1;
    sc->A.done = 0;
  }
}

// ================================ launch ====================================
// Segment length along x3 and the grid: about `target` blocks, whole
// pencils when the rows alone fill that many.
void pencil_grid(int np, int epb, const int n[3], int ks_req, int* ks, int* n_ig, int* n_seg) {
  (void)np;
  *n_ig = (n[0] + epb - 1) / epb;
  const int64_t rows = (int64_t)(*n_ig) * n[1];
  int k = ks_req;
  if (k <= 0) {
    constexpr int64_t target = 1024;
    const int64_t segs = std::max<int64_t>(1, (target + rows - 1) / rows);
    k = (int)std::max<int64_t>(1, (n[2] + segs - 1) / segs);
  }
  k = std::min(std::max(k, 1), n[2]);
  *ks = k;
  *n_seg = (n[2] + k - 1) / k;
}

template <typename T, int NP, int EPB>
static hipError_t pencil_launch_variant(const hdg_ctx* c, const ElemTab<T>& tab, PencilIO<T> io,
                                        hipStream_t s) {
  int ks, n_ig, n_seg;
  pencil_grid(NP, EPB, c->n, c->pencil_ks, &ks, &n_ig, &n_seg);
  io.ks = ks;
  io.n_ig = n_ig;
  io.n_seg = n_seg;
  const int nb = n_ig * c->n[1] * n_seg;
  hipLaunchKernelGGL((pencil_apply_kernel<T, NP, EPB>), dim3(nb), dim3(unit_threads<NP, EPB>()),
                     0, s, c->mesh, tab, io);
  return hipGetLastError();
}

template <typename T, int NP>
static hipError_t pencil_launch_np(const hdg_ctx* c, const ElemTab<T>& tab, const PencilIO<T>& io,
                                   hipStream_t s) {
  switch (c->tile_variant) {
    case 1: return pencil_launch_variant<T, NP, epb_var<NP, 1>()>(c, tab, io, s);
    case 2: return pencil_launch_variant<T, NP, epb_var<NP, 2>()>(c, tab, io, s);
    default: return pencil_launch_variant<T, NP, epb_var<NP, 0>()>(c, tab, io, s);
  }
}

template <typename T>
static const ElemTab<T>& pencil_tab(const hdg_ctx* c);
template <>
const ElemTab<double>& pencil_tab<double>(const hdg_ctx* c) { return c->et64; }
template <>
const ElemTab<float>& pencil_tab<float>(const hdg_ctx* c) { return c->et32; }

int pencil_blocks(const hdg_ctx* c, int variant) {
  int ks, n_ig, n_seg;
  pencil_grid(c->np, tile_epb(c->np, variant), c->n, c->pencil_ks, &ks, &n_ig, &n_seg);
  return n_ig * c->n[1] * n_seg;
}

template <typename T>
hipError_t launch_pencil_apply(const hdg_ctx* c, CgWork<T>& w, hipStream_t s) {
  PencilIO<T> io{};
  io.z = w.z;
  io.p0 = w.p[0];
  io.p1 = w.p[1];
  io.x = w.x;
  io.qa = w.qa;
  io.qb = w.qb;
  io.partials = w.partials;
  io.pmax = w.pmax;
  io.n_upd = w.update_blocks;
  io.sc = w.sc;
  const ElemTab<T>& tab = pencil_tab<T>(c);
  switch (c->np) {
#define HDG_CASE(N) \
  case N: return pencil_launch_np<T, N>(c, tab, io, s);
    HDG_CASE(2) HDG_CASE(3) HDG_CASE(4) HDG_CASE(5) HDG_CASE(6) HDG_CASE(7) HDG_CASE(8)
    HDG_CASE(9) HDG_CASE(10) HDG_CASE(11) HDG_CASE(12) HDG_CASE(13) HDG_CASE(14)
    HDG_CASE(15) HDG_CASE(16) HDG_CASE(17)
#undef HDG_CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_pencil_update(const hdg_ctx* c, CgWork<T>& w, hipStream_t s) {
  int ks, n_ig, n_seg;
  pencil_grid(c->np, tile_epb(c->np, c->tile_variant), c->n, c->pencil_ks, &ks, &n_ig, &n_seg);
  const int64_t npf = (int64_t)c->np * c->np;
  const int64_t plane = (int64_t)c->n[0] * c->n[1] * npf;
  const int64_t x3_lo = c->mesh.foff[2] * npf;
  const int64_t x3_hi = x3_lo + plane * (c->n[2] - 1);
  hipLaunchKernelGGL((pencil_update_kernel<T>), dim3(w.update_blocks), dim3(kPencilVecThreads), 0,
                     s, w.n, w.qa, w.qb, w.z, w.dinv, w.partials, w.pmax, w.pencil_blocks, w.sc,
                     x3_lo, x3_hi, (uint32_t)plane, 1.0f / (float)plane, (uint32_t)ks,
                     1.0f / (float)ks);
  return hipGetLastError();
}

template hipError_t launch_pencil_apply<double>(const hdg_ctx*, CgWork<double>&, hipStream_t);
template hipError_t launch_pencil_apply<float>(const hdg_ctx*, CgWork<float>&, hipStream_t);
template hipError_t launch_pencil_update<double>(const hdg_ctx*, CgWork<double>&, hipStream_t);
template hipError_t launch_pencil_update<float>(const hdg_ctx*, CgWork<float>&, hipStream_t);

}  // namespace hdg
