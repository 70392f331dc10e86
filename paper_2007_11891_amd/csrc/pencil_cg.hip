// Pencil form of the two-kernel CG (solver HDG-trans: Jacobi-preconditioned
// CG on the transformed condensed operator of algorithm "HDG_Op_3D" in the
// eigen-face basis; paper, sections "Product factorization of the HDG
// operator" and "Summary of solution method").
//
// Each block owns EPB elements side by side along x1 (one slot each) in one
// row (fixed x2 index) and marches them up x3 through a segment of `ks`
// elements.  A thread owns the face-node column (q1, q2) of its slot's
// element, so the face between two consecutive elements of the march (normal
// x3) is the same face-node column for the same thread: its input is loaded
// once and carried in a register, and its two element contributions are
// summed in a register and stored once.  Faces normal to x1 and x2 keep the
// two-contribution layout of the other CG forms (qa from the element below,
// qb from the element above).  Blocks of one XCD work on neighbouring rows of
// the same segment, so the faces they share are read while they sit in that
// XCD's L2.
//
// Iteration k, element launch: beta_k from the update's r.z partials,
//   p_k = z_k + beta_k p_{k-1},  x += alpha_{k-1} p_{k-1}  (faces it owns),
//   w = K^ p_k  (qa / qb, or the x3 sum in qa),  p_k . w partial per block.
// Update launch: alpha_k = rho_k / (p_k . w), z -= alpha_k D^-1 w,
//   r.z and r.r partials.  The element launch that finds the solve finished
// applies the last x update (x_k = x_{k-1} + alpha_{k-1} p_{k-1}) and stops.
//
// A step of the march first consumes the loaded face values of its element
// (p and x updates and their stores, the input staged in LDS), then issues
// the loads of the next element into the same registers, and then runs the
// element arithmetic while those loads are in flight.  The 1D tables sit in
// LDS.
#include <algorithm>

#include "cg_state.hpp"
#include "elem_unit.hpp"

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

// Two values read together from LDS (one 16-byte access in FP64).
template <typename T>
struct alignas(2 * sizeof(T)) PencilPair {
  T lo, hi;
};

template <typename T, int NP, int EPB>
struct PencilSmem {
  PencilPair<T> face[EPB][2][NP * NP];      // faces normal to x1, x2 (input p), low and high
  T u[EPB][upitch<NP>() * NP * NP + 1];     // the element's u in the eigenspace
  PencilPair<T> bs[NP];                     // B_S[k][0], B_S[k][1]
  T lam[NP];
};

// Face ids of one slot's pencil (element (i, j, k) for the k of the march):
// a face normal to x1 or x2 has id A + B k (its plane does not change along
// the march), a face normal to x3 has id x3A + x3B (pl - 1) on the interior
// plane pl, or one of the two boundary ids at the ends.  A face is free when
// its id is below n_free_faces; a free face on the boundary of the box (a
// Neumann side) has this element alone.  32-bit ids and offsets: the host
// runs this form only when every trace offset fits.
struct PencilRow {
  int A[4];            // faces normal to x1, x2 at k = 0
  int x3A;             // interior x3 face of plane 1 (foff[2] + i + n1 j)
  int x3bot, x3top;    // the boundary x3 faces of the column
  int freem, alonem;   // bits 0..3: faces normal to x1, x2; bits 4, 5: the
                       // boundary x3 faces (used at k = 0 and k = n3 - 1)
};

__device__ inline void pencil_row(const MeshDev& m, int i, int j, PencilRow& R) {
  R.freem = R.alonem = 0;
  const int nff = (int)m.n_free_faces;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int pl0 = i + s;
    if (pl0 >= 1 && pl0 <= m.n1 - 1) {
      R.A[s] = (int)m.foff[0] + (pl0 - 1) + (m.n1 - 1) * j;
      R.freem |= 1 << s;
    } else {
      R.A[s] = (int)m.boff[s] + j;
      if (R.A[s] < nff) R.alonem |= 1 << s;
    }
    const int pl1 = j + s;
    if (pl1 >= 1 && pl1 <= m.n2 - 1) {
      R.A[2 + s] = (int)m.foff[1] + i + m.n1 * (pl1 - 1);
      R.freem |= 4 << s;
    } else {
      R.A[2 + s] = (int)m.boff[2 + s] + i;
      if (R.A[2 + s] < nff) R.alonem |= 4 << s;
    }
  }
  const int ij = i + m.n1 * j;
  R.x3A = (int)m.foff[2] + ij;
  R.x3bot = (int)m.boff[4] + ij;
  R.x3top = (int)m.boff[5] + ij;
  if (R.x3bot < nff) R.alonem |= 16;
  if (R.x3top < nff) R.alonem |= 32;
  R.freem |= R.alonem;
}

// Id of face f of the slot's element at k; *fr: free, *al: alone on it.
// Along the march a face normal to x1 moves by (n1 - 1) n2 ids per element
// when interior and by n2 on a side of the box; normal to x2 by n1 (n2 - 1)
// and n1; normal to x3 by n1 n2.
__device__ inline int pencil_fid(const MeshDev& m, const PencilRow& R, int k, int f, bool* fr,
                                 bool* al) {
  if (f < 4) {
    const bool in = (R.freem >> f) & 1 & ~(R.alonem >> f);
    const int step = f < 2 ? (in ? (m.n1 - 1) * m.n2 : m.n2) : (in ? m.n1 * (m.n2 - 1) : m.n1);
    *fr = (R.freem >> f) & 1;
    *al = (R.alonem >> f) & 1;
    return R.A[f] + step * k;
  }
  const int pl = k + (f & 1);                  // plane of the x3 face
  if (pl >= 1 && pl <= m.n3 - 1) {
    *fr = true;
    *al = false;
    return R.x3A + m.n1 * m.n2 * (pl - 1);
  }
  *fr = (R.freem >> f) & 1;
  *al = *fr;
  return f == 4 ? R.x3bot : R.x3top;
}

// Loads of one element of the march (issued one step ahead of their use).
// Every lane loads from a valid address (faces that are not free, and idle
// lanes, read the first free face) and the values of faces it does not use
// are dropped where they are consumed: no conditional load writes a register
// that an earlier load may still be filling.
template <typename T>
struct PencilLoads {
  T z[6], po[6];      // face 4 (low x3) only at the start of a segment
  T xo[6];            // x on the owned faces (high faces; low faces alone on a Neumann side)
  double d[4], lam;   // metric factors d0..d3 and lambda of the element
};

template <typename T, int NP>
__device__ inline void pencil_load(const MeshDev& m, const T* __restrict__ z,
                                   const T* __restrict__ pin, const T* __restrict__ x,
                                   const PencilRow& R, int k, bool act, int col, int e, bool first,
                                   PencilLoads<T>& L) {
  constexpr int NF = NP * NP;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    bool fr, al;
    const int fid = pencil_fid(m, R, k, f, &fr, &al);
    if (f == 4 && !first) {
      L.z[f] = L.po[f] = L.xo[f] = 0;
      continue;
    }
    const bool u = act && fr;
    const int g = (u ? fid * NF : 0) + (act ? col : 0);
    L.z[f] = z[g];
    L.po[f] = pin[g];
    if ((f & 1) || (R.alonem >> f) & 1) L.xo[f] = x[g];
    else L.xo[f] = 0;
  }
  const ElemInfo* ei = m.info + e;      // e is valid for every lane (idle slots clamped)
  L.d[0] = ei->d[0];
  L.d[1] = ei->d[1];
  L.d[2] = ei->d[2];
  L.d[3] = ei->d[3];
  L.lam = m.lam[e];
}

// Element arithmetic on the input p (xf, faces 0..3 staged in LDS by the
// caller before this call): expansion into the element eigenspace, division
// by D_Z, reductions back to the faces, and the face term with the 2 x 2
// matrix H = G + C^T M^-1 C of each axis.  Two barriers per element.
template <typename T, int NP, int EPB>
__device__ inline void pencil_core(PencilSmem<T, NP, EPB>& sm, int sl, int q1, int q2, int col,
                                   bool act, const T* d, const T* xf, T H, T H11, T H01,
                                   T* out) {
  constexpr int P = upitch<NP>();
  __syncthreads();
  T r2lo = 0, r2hi = 0;
  if (act) {
    const PencilPair<T>* f0 = sm.face[sl][0];
    const PencilPair<T>* f1 = sm.face[sl][1];
    const PencilPair<T> b1 = sm.bs[q1], b2 = sm.bs[q2];
    const T c0 = d[1] * b1.lo, c1 = d[1] * b1.hi;
    const T c2 = d[2] * b2.lo, c3 = d[2] * b2.hi;
    const T x2lo = d[3] * xf[4], x2hi = d[3] * xf[5];
    const T dij = d[0] + d[1] * sm.lam[q1] + d[2] * sm.lam[q2];
    T* u = sm.u[sl] + q1 + P * q2;
#pragma unroll 2
    for (int q3 = 0; q3 < NP; ++q3) {
      const PencilPair<T> b = sm.bs[q3];
      const PencilPair<T> a0 = f0[q2 + NP * q3];
      const PencilPair<T> a1 = f1[q1 + NP * q3];
      T F = c0 * a0.lo;
      F += c1 * a0.hi;
      F += c2 * a1.lo;
      F += c3 * a1.hi;
      F += b.lo * x2lo;
      F += b.hi * x2hi;
      const T v = div_fast(F, dij + d[3] * sm.lam[q3]);
      u[P * NP * q3] = v;
      r2lo += b.lo * v;
      r2hi += b.hi * v;
    }
  }
  __syncthreads();
  if (act) {
    T lo = 0, hi = 0;
    const T* ua = sm.u[sl] + P * col;             // axis 0: face node (q2, q3) = col
#pragma unroll 4
    for (int a = 0; a < NP; ++a) {
      const PencilPair<T> b = sm.bs[a];
      lo += b.lo * ua[a];
      hi += b.hi * ua[a];
    }
    out[0] = d[1] * (H * xf[0] + H01 * xf[1] - lo);
    out[1] = d[1] * (H11 * xf[1] + H01 * xf[0] - hi);
    lo = 0;
    hi = 0;
    const T* ub = sm.u[sl] + q1 + P * NP * q2;    // axis 1: face node (q1, q3) = col
#pragma unroll 4
    for (int b = 0; b < NP; ++b) {
      const PencilPair<T> bb = sm.bs[b];
      lo += bb.lo * ub[P * b];
      hi += bb.hi * ub[P * b];
    }
    out[2] = d[2] * (H * xf[2] + H01 * xf[3] - lo);
    out[3] = d[2] * (H11 * xf[3] + H01 * xf[2] - hi);
    out[4] = d[3] * (H * xf[4] + H01 * xf[5] - r2lo);
    out[5] = d[3] * (H11 * xf[5] + H01 * xf[4] - r2hi);
  }
  // no barrier here: the next element stages its faces (read above only
  // before the second barrier) and writes u only after its first barrier,
  // which every wave reaches after finishing these reductions
}

// One element of the march.  In: L holds the loaded values of element k.
// The input p on its faces, p and x on the faces it owns (stored), the input
// staged in LDS; then the loads of element kn into L; then the operator and
// the stores of the contributions.  carry_p / carry_w: p and the
// contribution of the x3 face shared with the previous element of the
// segment (in), and with the next one (out).
template <typename T, int NP, int EPB>
__device__ inline void pencil_step(const T* __restrict__ z, const T* __restrict__ pin,
                                   T* __restrict__ pout, T* __restrict__ x, T* __restrict__ qa,
                                   T* __restrict__ qb, PencilSmem<T, NP, EPB>& sm,
                                   const UnitLane& Ln, bool act, const MeshDev& m,
                                   const PencilRow& R, int k, int kn, int en, PencilLoads<T>& L,
                                   bool first, bool last, T alpha, T beta, T H, T H11, T H01,
                                   T& carry_p, T& carry_w, double* dot) {
  constexpr int NF = NP * NP;
  const int col = Ln.col;
  T xf[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    bool fr, al;
    const int fid = pencil_fid(m, R, k, f, &fr, &al);
    T v = 0;
    if (f == 4 && !first) {
      v = carry_p;
    } else if (act && fr) {
      v = L.z[f] + beta * L.po[f];
      if ((f & 1) || al) {                    // the face is this element's
        pout[fid * NF + col] = v;
        x[fid * NF + col] = L.xo[f] + alpha * L.po[f];
      }
    }
    xf[f] = v;
  }
  if (act) {
    sm.face[Ln.sl][0][col] = PencilPair<T>{xf[0], xf[1]};
    sm.face[Ln.sl][1][col] = PencilPair<T>{xf[2], xf[3]};
  }
  const T d[4] = {(T)(L.d[0] * L.lam), (T)L.d[1], (T)L.d[2], (T)L.d[3]};
  // the next element's loads go out before the arithmetic of this one
  pencil_load<T, NP>(m, z, pin, x, R, kn, act, col, en, false, L);
  T out[6];
  pencil_core<T, NP, EPB>(sm, Ln.sl, Ln.q1, Ln.q2, col, act, d, xf, H, H11, H01, out);
  if (!act) return;
  double acc = 0.0;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    bool fr, al;
    const int fid = pencil_fid(m, R, k, f, &fr, &al);
    if (!fr) continue;
    const int g = fid * NF + col;
    acc += (double)(xf[f] * out[f]);
    if (f < 4) {
      if (f & 1) {
        qa[g] = out[f];
        if (al) qb[g] = 0;
      } else {
        qb[g] = out[f];
        if (al) qa[g] = 0;
      }
    } else if (f == 4) {
      if (!first) {
        qa[g] = out[4] + carry_w;             // both contributions, summed here
      } else {
        qb[g] = out[4];                       // the element below is in another segment
        if (al) qa[g] = 0;
      }
    } else if (last) {
      qa[g] = out[5];                         // the element above is in another segment
      if (al) qb[g] = 0;
    }
  }
  carry_p = xf[5];
  carry_w = out[5];
  *dot += acc;
}

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
    if (!act) return;
    constexpr int NF = NP * NP;
    for (int k = k0; k < k1; ++k) {
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        bool fr, al;
        const int fid = pencil_fid(mesh, row, k, f, &fr, &al);
        if (!fr || !((f & 1) || al)) continue;
        const int g = fid * NF + Ln.col;
        x[g] = x[g] + alpha * pin[g];
      }
    }
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
