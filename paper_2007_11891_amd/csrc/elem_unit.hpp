// One work unit of the condensed HDG operator in the eigen-face basis (paper:
// algorithm "HDG_Op_3D" for the transformed basis, section "Product
// factorization of the HDG operator"), shared by the single-problem element
// kernels and the batched persistent solver.  Per element e with transformed
// faces x_{a,s} (axis a, side s) and metric factors d_0..d_3:
//
//   F[q1,q2,q3] = d1 sum_s BS[q1,s] x_{0,s}[q2,q3] + d2 sum_s BS[q2,s] x_{1,s}[q1,q3]
//               + d3 sum_s BS[q3,s] x_{2,s}[q1,q2]
//   u[q]        = F[q] / (lambda d0 + d1 Lam[q1] + d2 Lam[q2] + d3 Lam[q3])
//   r_{0,s}[q2,q3] = d1 H x_{0,s} - d1 sum_q1 BS[q1,s] u[q1,q2,q3]   (same for axes 1, 2)
//
// The inverse eigenvalues are recomputed instead of stored (the paper stored
// them; its roofline discussion notes that their n_p^3 loads cap the
// intensity).  One thread per face-node column (q1,q2) walks q3 and keeps the
// axis-2 reduction in registers; faces normal to x1, x2 and the element's u
// go through LDS (u with an odd row pitch, so the axis-0 reduction is free of
// bank conflicts).  For n_p = 7, 8 and n_p >= 10 an element is owned by whole
// wavefronts (the element record is wave-uniform; the single-problem kernels
// read it with scalar loads); for n_p <= 6 and n_p = 9 several elements share
// a wavefront.  Each interior face receives
// one contribution from the element below it (qa) and one from the element
// above it (qb): plain stores, no atomics, deterministic sums.
#pragma once
#include "device_common.hpp"

namespace hdg {

// ---- tile shapes ------------------------------------------------------------
// n_p = 6 and 9 pack several elements into a wavefront instead (36 and 81
// threads per element would leave 44 % and 37 % of the lanes of whole
// wavefronts idle; measured 7-15 % faster CG iterations at p = 5 and 8,
// while n_p = 7 measured faster as a group despite its idle lanes)
template <int NP>
__host__ __device__ constexpr bool is_group() { return NP >= 7 && NP != 9; }
template <int NP>  // threads per element
__host__ __device__ constexpr int tpe() { return is_group<NP>() ? round_up64(NP * NP) : NP * NP; }
template <int NP>
__host__ __device__ constexpr int upitch() { return NP | 1; }
template <int NP>  // LDS words of one element (FP64 sizing)
__host__ __device__ constexpr int lds_elem_words() {
  return 4 * NP * NP + upitch<NP>() * NP * NP + 1;
}
// largest elements-per-unit for 256 threads and 60 KB of LDS
template <int NP>
__host__ __device__ constexpr int epb_max() {
  constexpr int by_threads = (256 / tpe<NP>()) > 0 ? 256 / tpe<NP>() : 1;
  constexpr int by_lds = (60000 / (8 * lds_elem_words<NP>())) > 0 ? 60000 / (8 * lds_elem_words<NP>()) : 1;
  constexpr int e = by_threads < by_lds ? by_threads : by_lds;
  return (is_group<NP>() && e > 4) ? 4 : e;
}
// tile variant v = 0, 1, 2: epb_max, epb_max/2, epb_max/4 elements per unit
constexpr int kTileVariants = 3;
template <int NP, int V>
__host__ __device__ constexpr int epb_var() {
  return (epb_max<NP>() >> V) > 0 ? (epb_max<NP>() >> V) : 1;
}
template <int NP, int EPB>
__host__ __device__ constexpr int unit_threads() { return round_up64(EPB * tpe<NP>()); }

// Pointers of one problem (already offset into batched storage).
template <typename T>
struct UnitIO {
  const ElemInfo* info;
  const double* lam;
  int n_elem;
  int nff;                 // number of free faces
  // plain apply
  const T* x_free;
  const T* x_bdry;         // may be null
  T* qa;
  T* qb;
  // fused CG apply (MODE 1): p = z + beta p_old; MODE 3 also makes the
  // previous iteration's x step on the faces the unit owns, x += alpha p_old
  // (alpha and x below), so that the vector update need not touch x and p
  const T* z;              // z = D^-1 r
  const T* p_in;
  T* p_out;
  T beta;
  // one-kernel CG iteration (MODE 2): w = qa_old + qb_old = A z_old,
  //   s = D^-1 w + beta s_old, p = z_old + beta p_old, x += alpha p,
  //   z = z_old - alpha s, then the operator applied to z
  const T* z_old;
  T* z_new;
  const T* s_old;
  T* s_new;
  const T* w_a;
  const T* w_b;
  const T* dinv;
  T* x;
  T alpha;
  bool first;              // first launch: the operator applied to z_old as is
};

// What the 1D tables of a caller can carry: faces on Neumann sides (an
// element alone on a free face) and the exact-mass coupling H01 of opposite
// faces.  A table type that never does (the batched solver's) specialises
// this to drop both from its code paths at compile time.
template <typename Tab>
struct TabTraits {
  static constexpr bool neumann = true;
  static constexpr bool exact_mass = true;
};

template <typename T, int NP, int EPB>
struct UnitSmem {
  T face[EPB][4][NP * NP];
  T u[EPB][upitch<NP>() * NP * NP + 1];
};

// Lane geometry of a work unit: element slot within the unit and face-node
// column (q1, q2) of the thread with block index tid.
struct UnitLane {
  int slot, col, q1, q2, sl;
  bool colok;
};
template <int NP, int EPB>
__device__ inline UnitLane unit_lane(int tid) {
  constexpr int NF = NP * NP;
  constexpr int TPE = tpe<NP>();
  UnitLane L;
  if constexpr (is_group<NP>()) {
    L.slot = __builtin_amdgcn_readfirstlane(tid / TPE);   // wave-uniform
    L.col = tid % TPE;
  } else {
    L.slot = tid / NF;
    L.col = tid % NF;
  }
  L.colok = L.col < NF;
  L.q1 = L.col % NP;
  L.q2 = L.col / NP;
  L.sl = L.slot < EPB ? L.slot : 0;
  return L;
}

// Registers of one unit between its loads and its arithmetic: the element
// record and the raw face values (MODE 0: the input x; MODES 1, 3: z and
// p_old; MODE 3 also x on the three faces the unit owns, c[f / 2]).  MODE 3
// keeps lambda_e apart from d[0] (so that no arithmetic waits on the record
// loads) and the lane's byte offset into the trace vectors of each face.
template <typename T>
struct UnitRegs {
  bool active;
  int fid[6];
  int nm;          // faces that are unknowns with this element alone (bit f)
  T d[4];
  T a[6];
  T b[6];
  T c[3];
  T lam;
  uint32_t off[6];
};

// Element record of the lane's element in unit `unit`.
template <typename T, int NP, int EPB>
__device__ inline void unit_info(const UnitIO<T>& io, const UnitLane& L, int unit, UnitRegs<T>& R) {
  const int e = unit * EPB + L.slot;
  R.active = L.slot < EPB && e < io.n_elem;
  R.nm = 0;
  if (R.active) {
    const ElemInfo* ei = io.info + e;
    R.d[0] = (T)(ei->d[0] * io.lam[e]);
    R.d[1] = (T)ei->d[1];
    R.d[2] = (T)ei->d[2];
    R.d[3] = (T)ei->d[3];
#pragma unroll
    for (int f = 0; f < 6; ++f) R.fid[f] = ei->fid[f];
    R.nm = ei->nmask;
  }
}

// Issues the face loads of a unit (MODES 0 and 1); no arithmetic on them,
// so that they can stay in flight while another unit computes.
template <typename T, int NP, int MODE>
__device__ inline void unit_data(const UnitIO<T>& io, const UnitLane& L, UnitRegs<T>& R) {
  static_assert(MODE == 0 || MODE == 1, "MODE 3 loads through unit_data_ranged");
  constexpr int NF = NP * NP;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    R.a[f] = 0;
    R.b[f] = 0;
    if (R.active && L.colok) {
      if (R.fid[f] < io.nff) {
        const int64_t g = (int64_t)R.fid[f] * NF + L.col;
        if constexpr (MODE == 0) {
          R.a[f] = io.x_free[g];
        } else {
          R.a[f] = io.z[g];
          R.b[f] = io.p_in[g];
        }
      } else if (MODE == 0 && io.x_bdry != nullptr) {
        R.a[f] = io.x_bdry[(int64_t)(R.fid[f] - io.nff) * NF + L.col];
      }
    }
  }
}

// Output stores.  The fused CG apply (MODE 1) writes its results with the
// non-temporal hint: nothing reads them again in the same launch, and
// measured on MI355X its CG iteration is 2 to 10 % faster for it; the other
// kernels measured as fast or faster with plain stores.
template <int MODE, typename T>
__device__ inline void put(T* p, T v) {
  if constexpr (MODE == 1) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// ---- range-checked trace access (MODE 3, FP64) -------------------------------
// A raw buffer resource spans one trace vector of the problem (under 2 GiB,
// which the batch set-up checks).  The memory unit checks every access
// against that range: one at kOutOfRange reads zero and writes nothing.
// Masked lanes take that offset instead of a branch, so every path through a
// unit issues the same loads and stores, and the compiler's wait for a unit's
// face data counts exactly the memory operations issued after them: the loads
// of the next unit stay in flight through the arithmetic of this one (with
// branches around them the count differs between paths and the wait falls
// back to all of them).
constexpr uint32_t kOutOfRange = 0x80000000u;
struct UnitBufs {
  __amdgpu_buffer_rsrc_t z, p_in, x, qa, qb, p_out;
};
__device__ inline __amdgpu_buffer_rsrc_t trace_rsrc(const void* p, uint32_t bytes) {
  // word 3: 32-bit data format, which untyped buffer accesses need on gfx9
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}
template <int NP>
__device__ inline UnitBufs unit_bufs(const UnitIO<double>& io) {
  const uint32_t n = (uint32_t)io.nff * (uint32_t)(NP * NP) * 8u;
  return {trace_rsrc(io.z, n),  trace_rsrc(io.p_in, n), trace_rsrc(io.x, n),
          trace_rsrc(io.qa, n), trace_rsrc(io.qb, n),   trace_rsrc(io.p_out, n)};
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ inline double buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
// non-temporal (cache policy bit 1): nothing reads these in the same phase
__device__ inline void buf_store_nt(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 2);
}

// Element record of unit `unit` (valid: the unit is one to compute) loaded
// without a branch: a lane without an element reads element 0's record and
// is marked inactive.  Nothing is computed from the loads here.
template <int NP, int EPB>
__device__ inline void unit_info_ranged(const UnitIO<double>& io, const UnitLane& L, int unit,
                                        bool valid, UnitRegs<double>& R) {
  // global address space: generic (flat) loads would make every later wait
  // for memory a wait for all of it
  typedef const __attribute__((address_space(1))) ElemInfo GInfo;
  typedef const __attribute__((address_space(1))) double GDouble;
  const int e = unit * EPB + L.slot;
  R.active = valid && L.slot < EPB && e < io.n_elem;
  const int ec = R.active ? e : 0;
  GInfo* ei = (GInfo*)io.info + ec;
#pragma unroll
  for (int k = 0; k < 4; ++k) R.d[k] = ei->d[k];
  R.lam = ((GDouble*)io.lam)[ec];
#pragma unroll
  for (int f = 0; f < 6; ++f) R.fid[f] = ei->fid[f];
  R.nm = 0;
}

// Face loads of a unit in MODE 3: z and p_old on every face, x on the three
// faces the unit owns (its high faces: batched problems have no Neumann side).
template <int NP>
__device__ inline void unit_data_ranged(const UnitBufs& B, const UnitIO<double>& io,
                                        const UnitLane& L, UnitRegs<double>& R) {
  constexpr int NF = NP * NP;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const bool on = R.active && L.colok && R.fid[f] < io.nff;
    R.off[f] = on ? ((uint32_t)R.fid[f] * NF + (uint32_t)L.col) * 8u : kOutOfRange;
    R.a[f] = buf_load(B.z, R.off[f]);
    R.b[f] = buf_load(B.p_in, R.off[f]);
    if (f & 1) R.c[f >> 1] = buf_load(B.x, R.off[f]);
  }
}

// The 1D table entries a lane needs at its face-node column (q1, q2).  A
// caller that runs many units can load them once: in the batched kernel the
// tables are device memory, and loads issued inside a unit would wait behind
// the next unit's face loads.
template <typename T>
struct LaneTab {
  T bs0q1, bs1q1, bs0q2, bs1q2, lamq1, lamq2;
};
template <typename T, typename Tab>
__device__ inline LaneTab<T> lane_tab(const Tab& tab, const UnitLane& L) {
  // a lane past the last column (q2 >= n_p) reads entry 0
  const int q1 = L.colok ? L.q1 : 0, q2 = L.colok ? L.q2 : 0;
  return {(T)tab.bs0[q1], (T)tab.bs1[q1], (T)tab.bs0[q2],
          (T)tab.bs1[q2], (T)tab.lam[q1], (T)tab.lam[q2]};
}

// Element arithmetic of one unit given its input face values xf (already in
// registers, faces 0..3 also staged in LDS by the caller before the first
// barrier): expansion into the element eigenspace, reductions back to the
// faces, stores of qa / qb, and the quadratic form xf.out into *dot.  A face
// in nm (on a Neumann side of the box) has no second element: its other
// slot is written with zero, so that qa + qb is the face's sum.  MODE 3
// takes the lane's table entries (lt) and its face offsets into the ranged
// trace vectors (bufs, off) from the caller.
template <typename T, int NP, int EPB, int MODE, typename Tab>
__device__ inline void unit_core(const UnitIO<T>& io, const Tab& tab, UnitSmem<T, NP, EPB>& sm,
                                 const UnitLane& L, bool active, const int* fid, int nm,
                                 const T* d, const T* xf, double* dot,
                                 const UnitBufs* bufs = nullptr, const uint32_t* off = nullptr,
                                 const LaneTab<T>* lt = nullptr) {
  constexpr int NF = NP * NP;
  constexpr int P = upitch<NP>();
  const int sl = L.sl, q1 = L.q1, q2 = L.q2, col = L.col;
  if constexpr (!TabTraits<Tab>::neumann) nm = 0;
  const T h01 = TabTraits<Tab>::exact_mass ? (T)tab.H01 : (T)0;
  __syncthreads();

  // expansion into the element eigenspace, division, axis-2 reduction
  T r2lo = 0, r2hi = 0;
  if (active && L.colok) {
    const T* f0lo = sm.face[sl][0];
    const T* f0hi = sm.face[sl][1];
    const T* f1lo = sm.face[sl][2];
    const T* f1hi = sm.face[sl][3];
    LaneTab<T> t;
    if constexpr (MODE == 3) t = *lt;
    else t = {tab.bs0[q1], tab.bs1[q1], tab.bs0[q2], tab.bs1[q2], tab.lam[q1], tab.lam[q2]};
    const T c0 = d[1] * t.bs0q1, c1 = d[1] * t.bs1q1;
    const T c2 = d[2] * t.bs0q2, c3 = d[2] * t.bs1q2;
    const T x2lo = d[3] * xf[4], x2hi = d[3] * xf[5];
    const T dij = d[0] + d[1] * t.lamq1 + d[2] * t.lamq2;
#pragma unroll
    for (int q3 = 0; q3 < NP; ++q3) {
      T F = c0 * f0lo[q2 + NP * q3];
      F += c1 * f0hi[q2 + NP * q3];
      F += c2 * f1lo[q1 + NP * q3];
      F += c3 * f1hi[q1 + NP * q3];
      F += tab.bs0[q3] * x2lo;
      F += tab.bs1[q3] * x2hi;
      const T u = div_fast(F, dij + d[3] * tab.lam[q3]);
      sm.u[sl][q1 + P * (q2 + NP * q3)] = u;
      r2lo += tab.bs0[q3] * u;
      r2hi += tab.bs1[q3] * u;
    }
  }
  __syncthreads();

  // reductions back to the faces and the face-diagonal term
  T out[6];
  if constexpr (MODE == 3)
    for (int f = 0; f < 6; ++f) out[f] = 0;
  if (active && L.colok) {
    {
      // axis 0: face node (q2,q3) = col
      const T* u = sm.u[sl] + P * col;
      T lo = 0, hi = 0;
#pragma unroll
      for (int a = 0; a < NP; ++a) {
        lo += tab.bs0[a] * u[a];
        hi += tab.bs1[a] * u[a];
      }
      out[0] = d[1] * (tab.H * xf[0] - lo);
      out[1] = d[1] * (tab.H11 * xf[1] - hi);
      if constexpr (TabTraits<Tab>::exact_mass) {
        out[0] += d[1] * h01 * xf[1];
        out[1] += d[1] * h01 * xf[0];
      }
    }
    {
      // axis 1: face node (q1,q3) = col
      const T* u = sm.u[sl] + q1 + P * NP * q2;
      T lo = 0, hi = 0;
#pragma unroll
      for (int b = 0; b < NP; ++b) {
        lo += tab.bs0[b] * u[P * b];
        hi += tab.bs1[b] * u[P * b];
      }
      out[2] = d[2] * (tab.H * xf[2] - lo);
      out[3] = d[2] * (tab.H11 * xf[3] - hi);
      if constexpr (TabTraits<Tab>::exact_mass) {
        out[2] += d[2] * h01 * xf[3];
        out[3] += d[2] * h01 * xf[2];
      }
    }
    out[4] = d[3] * (tab.H * xf[4] - r2lo);
    out[5] = d[3] * (tab.H11 * xf[5] - r2hi);
    if constexpr (TabTraits<Tab>::exact_mass) {
      out[4] += d[3] * h01 * xf[5];
      out[5] += d[3] * h01 * xf[4];
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      if (fid[f] >= io.nff) continue;
      if constexpr (MODE != 3) {
        const int64_t g = (int64_t)fid[f] * NF + col;
        put<MODE>((f & 1) ? io.qa + g : io.qb + g, out[f]);
        if ((nm >> f) & 1) put<MODE>((f & 1) ? io.qb + g : io.qa + g, (T)0);
      }
      if constexpr (MODE != 0) *dot += (double)(xf[f] * out[f]);
    }
  }
  if constexpr (MODE == 3) {
    // every lane stores; off is out of range where the lane has no face
#pragma unroll
    for (int f = 0; f < 6; ++f) buf_store_nt((f & 1) ? bufs->qa : bufs->qb, off[f], out[f]);
  }
  __syncthreads();                          // LDS is reused by the next unit
}

// MODES 0 and 1 from loaded registers: forms the input (MODE 1:
// p = z + beta p_old, written by the element below each face), stages it and
// runs the element arithmetic.
template <typename T, int NP, int EPB, int MODE, typename Tab>
__device__ inline void unit_compute(const UnitIO<T>& io, const Tab& tab, UnitSmem<T, NP, EPB>& sm,
                                    const UnitLane& L, const UnitRegs<T>& R, double* acc) {
  constexpr int NF = NP * NP;
  T xf[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    T v = R.a[f];
    if constexpr (MODE == 1) {
      v = R.a[f] + io.beta * R.b[f];
      // the element below owns the face; on a Neumann side the only element
      const bool own_lo = TabTraits<Tab>::neumann && ((R.nm >> f) & 1);
      if (((f & 1) || own_lo) && R.active && L.colok && R.fid[f] < io.nff)
        put<MODE>(io.p_out + (int64_t)R.fid[f] * NF + L.col, v);
    }
    xf[f] = v;
    if (f < 4 && R.active && L.colok) sm.face[L.sl][f][L.col] = v;
  }
  double dot = 0.0;
  unit_core<T, NP, EPB, MODE>(io, tab, sm, L, R.active, R.fid, R.nm, R.d, xf, &dot);
  acc[0] += dot;
}

// One-kernel CG iteration (MODE 2), split into its loads and its arithmetic
// so that the loads of a unit can be issued before the launch's scalar
// prologue.  Every load of the unit is issued before its first store, so
// that all of them are in flight together (a store in between would order
// them).  In the first launch only D^-1 and z are read.
template <typename T>
struct CgLoads {
  bool on[6];
  T dv[6], zo[6], wa[6], wb[6], so[6], pi[3], xo[3];
};

template <typename T, int NP>
__device__ inline void cg2_loads(const UnitIO<T>& io, const UnitLane& L, const UnitRegs<T>& R,
                                 CgLoads<T>& C) {
  constexpr int NF = NP * NP;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    C.on[f] = R.active && L.colok && R.fid[f] < io.nff;
    C.dv[f] = 1;
    C.zo[f] = C.wa[f] = C.wb[f] = C.so[f] = 0;
    if (f & 1) C.pi[f >> 1] = C.xo[f >> 1] = 0;
    if (C.on[f]) {
      const int64_t g = (int64_t)R.fid[f] * NF + L.col;
      C.dv[f] = io.dinv[g];
      C.zo[f] = io.z_old[g];
      if (!io.first) {
        C.wa[f] = io.w_a[g];
        C.wb[f] = io.w_b[g];
        C.so[f] = io.s_old[g];
        if (f & 1) {
          C.pi[f >> 1] = io.p_in[g];
          C.xo[f >> 1] = io.x[g];
        }
      }
    }
  }
}

// Per face: s = D^-1 w + beta s_old, z = z_old - alpha s, and on the faces
// the unit owns p = z_old + beta p_old, x += alpha p and the r.z, r.r
// shares; then the operator applied to z.  A unit owns the high face of each
// axis and, on a Neumann side at the low end of the box, the low face too;
// the loads of the latter are issued here (rare: boundary elements only).
template <typename T, int NP, int EPB, typename Tab>
__device__ inline void cg2_compute(const UnitIO<T>& io, const Tab& tab, UnitSmem<T, NP, EPB>& sm,
                                   const UnitLane& L, const UnitRegs<T>& R, const CgLoads<T>& C,
                                   double* acc) {
  constexpr int NF = NP * NP;
  T xf[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    T v = 0;
    if (C.on[f]) {
      const int64_t g = (int64_t)R.fid[f] * NF + L.col;
      const T d = C.dv[f];
      const bool own_lo = TabTraits<Tab>::neumann && !(f & 1) && ((R.nm >> f) & 1);
      if (io.first) {
        v = C.zo[f];
      } else {
        const T sn = d * (C.wa[f] + C.wb[f]) + io.beta * C.so[f];
        v = C.zo[f] - io.alpha * sn;
        if (f & 1) {                          // the element below owns the face
          const T pn = C.zo[f] + io.beta * C.pi[f >> 1];
          io.s_new[g] = sn;
          io.p_out[g] = pn;
          io.z_new[g] = v;
          io.x[g] = C.xo[f >> 1] + io.alpha * pn;
        } else if (own_lo) {
          const T pn = C.zo[f] + io.beta * io.p_in[g];
          const T xo = io.x[g];
          io.s_new[g] = sn;
          io.p_out[g] = pn;
          io.z_new[g] = v;
          io.x[g] = xo + io.alpha * pn;
        }
      }
      if ((f & 1) || own_lo) {
        const double r = (double)div_fast(v, d);
        acc[1] += (double)v * r;
        acc[2] += r * r;
      }
    }
    xf[f] = v;
    if (f < 4 && R.active && L.colok) sm.face[L.sl][f][L.col] = v;
  }
  double dot = 0.0;
  unit_core<T, NP, EPB, 2>(io, tab, sm, L, R.active, R.fid, R.nm, R.d, xf, &dot);
  acc[0] += dot;
}

// Processes elements [unit EPB, unit EPB + EPB).  Every thread of the block
// calls it (tid = its index in the block); threads beyond EPB * tpe idle.
// Adds to acc the thread's share of the element-local quadratic forms
// v_e^T K_e v_e of the input v (MODES 1, 2) and, in MODE 2, of r.z and r.r
// over the faces the unit owns (acc[1], acc[2]).
template <typename T, int NP, int EPB, int MODE, typename Tab>
__device__ inline void apply_unit(const UnitIO<T>& io, const Tab& tab, UnitSmem<T, NP, EPB>& sm,
                                  int unit, double* acc, int tid = (int)threadIdx.x) {
  constexpr int NF = NP * NP;
  const UnitLane L = unit_lane<NP, EPB>(tid);
  UnitRegs<T> R;
  unit_info<T, NP, EPB>(io, L, unit, R);
  if constexpr (MODE != 2) {
    unit_data<T, NP, MODE>(io, L, R);
    unit_compute<T, NP, EPB, MODE>(io, tab, sm, L, R, acc);
  } else {
    CgLoads<T> C;
    cg2_loads<T, NP>(io, L, R, C);
    cg2_compute<T, NP, EPB>(io, tab, sm, L, R, C, acc);
  }
}

// Units [u0, u1) with the loads of unit u + 1 (and the element records of
// unit u + 2) issued before the arithmetic of unit u, so that a block always
// has memory traffic in flight (MODES 0 and 1).  `between` runs once, after
// the first unit's loads are issued and before any arithmetic; when it
// returns false nothing is computed and the function returns false.
struct NoStep {
  __device__ bool operator()() const { return true; }
};
template <typename T, int NP, int EPB, int MODE, typename Tab, typename Between = NoStep>
__device__ inline bool run_units_pipelined(const UnitIO<T>& io, const Tab& tab,
                                           UnitSmem<T, NP, EPB>& sm, int u0, int u1, double* acc,
                                           int tid = (int)threadIdx.x, Between between = {}) {
  static_assert(MODE == 0 || MODE == 1, "MODE 3 runs through run_units_ranged");
  if (u0 >= u1) return between();
  const UnitLane L = unit_lane<NP, EPB>(tid);
  UnitRegs<T> cur, nxt;
  unit_info<T, NP, EPB>(io, L, u0, cur);
  unit_data<T, NP, MODE>(io, L, cur);
  if (u0 + 1 < u1) unit_info<T, NP, EPB>(io, L, u0 + 1, nxt);
  if (!between()) return false;
  for (int u = u0; u < u1; ++u) {
    const UnitRegs<T> c = cur;
    if (u + 1 < u1) {
      unit_data<T, NP, MODE>(io, L, nxt);
      cur = nxt;
      if (u + 2 < u1) unit_info<T, NP, EPB>(io, L, u + 2, nxt);
    }
    unit_compute<T, NP, EPB, MODE>(io, tab, sm, L, c, acc);
  }
  return true;
}

// MODE 3 from loaded registers: p = z + beta p_old on every face; on the
// faces the unit owns (its high faces) p and the previous iteration's x step
// x + alpha p_old are stored; then the element arithmetic.
template <int NP, int EPB, typename Tab>
__device__ inline void unit_compute_ranged(const UnitBufs& B, const UnitIO<double>& io,
                                           const Tab& tab, const LaneTab<double>& lt,
                                           UnitSmem<double, NP, EPB>& sm,
                                           const UnitLane& L, const UnitRegs<double>& R,
                                           double* acc) {
  static_assert(!TabTraits<Tab>::neumann, "MODE 3 is for meshes without Neumann sides");
  double xf[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const double v = R.a[f] + io.beta * R.b[f];
    if (f & 1) {
      buf_store_nt(B.p_out, R.off[f], v);
      buf_store_nt(B.x, R.off[f], R.c[f >> 1] + io.alpha * R.b[f]);
    }
    xf[f] = v;
    if (f < 4 && R.active && L.colok) sm.face[L.sl][f][L.col] = v;
  }
  const double d[4] = {R.d[0] * R.lam, R.d[1], R.d[2], R.d[3]};
  double dot = 0.0;
  unit_core<double, NP, EPB, 3>(io, tab, sm, L, R.active, R.fid, 0, d, xf, &dot, &B, R.off, &lt);
  acc[0] += dot;
}

// Units [u0, u1) in MODE 3 with the face loads of unit u + 1 and the element
// record of unit u + 2 in flight during the arithmetic of unit u.  Every load
// and store is issued unconditionally (a unit beyond u1 is inactive: its
// record is element 0's and its face accesses are out of range), so that no
// path through the loop changes the count of memory operations in flight.
template <int NP, int EPB, typename Tab>
__device__ inline void run_units_ranged(const UnitIO<double>& io, const Tab& tab,
                                        UnitSmem<double, NP, EPB>& sm, int u0, int u1,
                                        double* acc, int tid) {
  if (u0 >= u1) return;
  const UnitLane L = unit_lane<NP, EPB>(tid);
  const UnitBufs B = unit_bufs<NP>(io);
  const LaneTab<double> lt = lane_tab<double>(tab, L);
  UnitRegs<double> cur, nxt;
  unit_info_ranged<NP, EPB>(io, L, u0, true, cur);
  unit_data_ranged<NP>(B, io, L, cur);
  unit_info_ranged<NP, EPB>(io, L, u0 + 1, u0 + 1 < u1, nxt);
  for (int u = u0; u < u1; ++u) {
    const UnitRegs<double> c = cur;
    unit_data_ranged<NP>(B, io, L, nxt);
    cur = nxt;
    unit_info_ranged<NP, EPB>(io, L, u + 2, u + 2 < u1, nxt);
    unit_compute_ranged<NP, EPB>(B, io, tab, lt, sm, L, c, acc);
  }
}

}  // namespace hdg
