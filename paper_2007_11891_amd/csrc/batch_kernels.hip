// Batched Jacobi-PCG for many independent condensed-HDG problems of uneven
// sizes and degrees in one persistent launch.
//
// Each CG iteration of a problem is one or two phases over its segments:
//   apply  : element segments (a problem and a range of its element work
//            units); per segment the previous update's partials (r.z, r.r)
//            of that problem are re-summed in a fixed order, convergence is
//            decided, p = z + beta p_old is formed on the units' faces
//            (z = D^-1 r) and x takes the previous iteration's step on the
//            faces they own, the transformed operator is applied (the work
//            unit of the single-problem kernels, selected by degree and tile
//            shape) and one p.q partial is written per segment;
//   update : vector segments (a problem and a range of its free trace); per
//            segment the problem's apply partials are re-summed, alpha is
//            formed, z is updated and one r.z and one r.r partial are
//            written per segment.
// The one-phase form fuses both into one element pass per iteration, and the
// pencil form marches element columns (see below).  Converged problems drop
// out; the kernel returns when every problem is done.  Per-problem state
// lives in two slots (A: read by apply, written by update; B: the reverse),
// written by the block that owns the problem's first segment of the phase.
// Every reduction is a fixed-order sum over per-segment partials, so the
// result depends neither on timing nor on which block ran which segment.
//
// Grid barrier: each block publishes an arrival epoch in its own cache line;
// block 0 waits for all of them and then releases every block through its
// own line.  Every wait is bounded: on a time-out the kernel raises an error
// flag and every block returns, so the grid always drains.
#include "batch.hpp"
#include "elem_unit.hpp"
#include "pencil_unit.hpp"

namespace hdg {

constexpr int kBT = 256;                 // threads per block
constexpr unsigned kSpinLimit = 1u << 22;
constexpr int kMaxBlocksPerThread = 8;   // grid of at most kBT * 8 blocks

template <int NP>
__host__ __device__ constexpr int unit_lds_words() { return epb_max<NP>() * lds_elem_words<NP>(); }
__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kBatchLdsWords =
    cmax(cmax(cmax(unit_lds_words<2>(), unit_lds_words<3>()), cmax(unit_lds_words<4>(), unit_lds_words<5>())),
         cmax(cmax(cmax(unit_lds_words<6>(), unit_lds_words<7>()), cmax(unit_lds_words<8>(), unit_lds_words<9>())),
              cmax(unit_lds_words<10>(), unit_lds_words<11>())));
static_assert(kBatchLdsWords * 8 <= 40000, "batched LDS budget");
template <int NP>
__host__ __device__ constexpr int pencil_lds_words() {
  return (int)((sizeof(PencilSmem<double, NP, epb_max<NP>()>) + 7) / 8);
}
constexpr int kBatchPencilLdsWords =
    cmax(cmax(cmax(pencil_lds_words<2>(), pencil_lds_words<3>()),
              cmax(pencil_lds_words<4>(), pencil_lds_words<5>())),
         cmax(cmax(cmax(pencil_lds_words<6>(), pencil_lds_words<7>()),
                   cmax(pencil_lds_words<8>(), pencil_lds_words<9>())),
              cmax(pencil_lds_words<10>(), pencil_lds_words<11>())));
static_assert(kBatchPencilLdsWords * 8 <= 40000, "batched pencil LDS budget");

// Grid barrier.  Block i (> 0) publishes its arrival epoch in line i of
// `arrive`; block 0 polls all arrival lines (its threads in parallel), then
// publishes the epoch in line i of `release` for every block, which polls
// only its own line: no word is polled by more than one block.  Ordering:
// every wave waits for its stores, the block synchronises, one thread makes
// them visible to the device (release fence) before the arrival store; after
// the wait one thread invalidates stale cached data (acquire fence) before
// the block synchronises again.  Returns false when a wait timed out (then
// every block must return).
__device__ inline bool grid_sync(const BatchArgs& a, unsigned epoch) {
  __shared__ int s_ok;
  GridBar* gb = a.bar;
  unsigned* arrive = a.flags;
  unsigned* release = a.flags + (size_t)gridDim.x * kFlagStride;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (blockIdx.x == 0) {
    // each thread watches blocks tid + 1 + j kBT (j < kMaxBlocksPerThread),
    // all its loads in flight together
    bool ok = true;
    unsigned spins = 0;
    for (;;) {
      unsigned v[kMaxBlocksPerThread];
#pragma unroll
      for (int j = 0; j < kMaxBlocksPerThread; ++j) {
        const unsigned i = threadIdx.x + 1 + j * kBT;
        v[j] = i < gridDim.x ? __hip_atomic_load(arrive + (size_t)i * kFlagStride, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)
                             : epoch;
      }
      bool all = true;
#pragma unroll
      for (int j = 0; j < kMaxBlocksPerThread; ++j) all = all && v[j] >= epoch;
      if (all) break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        ok = false;
        break;
      }
    }
    if (!ok) __hip_atomic_store(&gb->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
    __syncthreads();
    for (unsigned i = threadIdx.x + 1; i < gridDim.x; i += kBT)
      __hip_atomic_store(release + (size_t)i * kFlagStride, epoch, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  } else if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(arrive + (size_t)blockIdx.x * kFlagStride, epoch, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (__hip_atomic_load(release + (size_t)blockIdx.x * kFlagStride, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT) < epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        __hip_atomic_store(&gb->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  if (threadIdx.x == 0)
    s_ok = __hip_atomic_load(&gb->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
  __syncthreads();
  return s_ok != 0;
}

// Wave-uniform copies (scalar registers) of values every lane holds equal.
template <typename T>
__device__ inline T* uni_ptr(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}
__device__ inline double uni_f64(double x) {
  const uint64_t v = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ inline int uni_int(int x) { return __builtin_amdgcn_readfirstlane(x); }

typedef const __attribute__((address_space(4))) double cdouble;
struct ConstTab {   // lumped mass: the face term is H on both faces, no coupling
  cdouble* bs0;
  cdouble* bs1;
  cdouble* lam;
  double H;
  double H11;
  static constexpr double H01 = 0.0;
};
// batched problems are all-Dirichlet with the lumped mass
template <>
struct TabTraits<ConstTab> {
  static constexpr bool neumann = false;
  static constexpr bool exact_mass = false;
};

// Units [u0, u1) of one problem at degree NP - 1 and tile EPB.  The
// per-degree tables (a device buffer the kernel never writes) are read as
// constant memory, i.e. with scalar loads.  The empty asm hides the
// pointer's origin so that the compiler cannot hoist the table loads of
// every degree to the kernel entry, which would keep all of them live in
// scalar registers.  (The pointer must be a plain device address: never the
// address of a kernel argument, which would force a private copy.)
template <int NP, int EPB>
__device__ inline double run_units(const UnitIO<double>& io, const double* tabs, double* smem,
                                   int u0, int u1) {
  constexpr int o = batch_tab_off(NP);
  const double* tp = tabs;
  asm volatile("" : "+s"(tp));
  cdouble* ct = (cdouble*)tp;
  const ConstTab tab{ct + o, ct + o + NP, ct + o + 2 * NP, ct[o + 3 * NP], ct[o + 3 * NP]};
  auto& sm = *reinterpret_cast<UnitSmem<double, NP, EPB>*>(smem);
  // the thread index through an empty asm: otherwise the compiler hoists every
  // degree's per-lane index arithmetic (loop-invariant) to the kernel entry
  // and keeps all of it live, which more than doubles the vector registers
  int tid = (int)threadIdx.x;
  asm volatile("" : "+v"(tid));
  double acc[3] = {0.0, 0.0, 0.0};
  run_units_ranged<NP, EPB>(io, tab, sm, u0, u1, acc, tid);
  return acc[0];
}

// The last x step of a finished solve, x += alpha p_old on the faces the
// units [u0, u1) own (their high faces; batched problems have no Neumann
// side).
template <int NP, int EPB>
__device__ inline void final_x_units(const UnitIO<double>& io, int u0, int u1, int tid) {
  constexpr int NF = NP * NP;
  const UnitLane L = unit_lane<NP, EPB>(tid);
  for (int u = u0; u < u1; ++u) {
    UnitRegs<double> R;
    unit_info<double, NP, EPB>(io, L, u, R);
    if (!R.active || !L.colok) continue;
#pragma unroll
    for (int f = 1; f < 6; f += 2)
      if (R.fid[f] < io.nff) {
        const int64_t g = (int64_t)R.fid[f] * NF + L.col;
        io.x[g] += io.alpha * io.p_in[g];
      }
  }
}

__device__ inline void dispatch_final_x(int np, int variant, const UnitIO<double>& io, int u0,
                                        int u1) {
  int tid = (int)threadIdx.x;
  asm volatile("" : "+v"(tid));
  switch (np * 4 + variant) {
#define HDG_FCASE(N)                                                           \
  case N * 4 + 0: final_x_units<N, epb_var<N, 0>()>(io, u0, u1, tid); return; \
  case N * 4 + 1: final_x_units<N, epb_var<N, 1>()>(io, u0, u1, tid); return; \
  case N * 4 + 2: final_x_units<N, epb_var<N, 2>()>(io, u0, u1, tid); return;
    HDG_FCASE(2) HDG_FCASE(3) HDG_FCASE(4) HDG_FCASE(5) HDG_FCASE(6) HDG_FCASE(7)
    HDG_FCASE(8) HDG_FCASE(9) HDG_FCASE(10) HDG_FCASE(11)
#undef HDG_FCASE
    default: return;
  }
}

// The one-phase form: units [u0, u1) of one problem through the one-kernel
// CG iteration of the single-problem kernels (MODE 2); acc gets the unit's
// shares of z.Az, r.z and r.r.
template <int NP, int EPB>
__device__ inline void run_units_cgcg(const UnitIO<double>& io, const double* tabs, double* smem,
                                      int u0, int u1, double* acc) {
  constexpr int o = batch_tab_off(NP);
  const double* tp = tabs;
  asm volatile("" : "+s"(tp));
  cdouble* ct = (cdouble*)tp;
  const ConstTab tab{ct + o, ct + o + NP, ct + o + 2 * NP, ct[o + 3 * NP], ct[o + 3 * NP]};
  auto& sm = *reinterpret_cast<UnitSmem<double, NP, EPB>*>(smem);
  int tid = (int)threadIdx.x;
  asm volatile("" : "+v"(tid));
  for (int u = u0; u < u1; ++u) apply_unit<double, NP, EPB, 2>(io, tab, sm, u, acc, tid);
}

__device__ inline void dispatch_units_cgcg(int np, int variant, const UnitIO<double>& io,
                                           const double* tabs, double* smem, int u0, int u1,
                                           double* acc) {
  switch (np * 4 + variant) {
#define HDG_UCASE(N)                                                                              \
  case N * 4 + 0: run_units_cgcg<N, epb_var<N, 0>()>(io, tabs, smem, u0, u1, acc); return;      \
  case N * 4 + 1: run_units_cgcg<N, epb_var<N, 1>()>(io, tabs, smem, u0, u1, acc); return;      \
  case N * 4 + 2: run_units_cgcg<N, epb_var<N, 2>()>(io, tabs, smem, u0, u1, acc); return;
    HDG_UCASE(2) HDG_UCASE(3) HDG_UCASE(4) HDG_UCASE(5) HDG_UCASE(6) HDG_UCASE(7)
    HDG_UCASE(8) HDG_UCASE(9) HDG_UCASE(10) HDG_UCASE(11)
#undef HDG_UCASE
    default: return;
  }
}

__device__ inline double dispatch_units(int np, int variant, const UnitIO<double>& io,
                                        const double* tabs, double* smem, int u0, int u1) {
  switch (np * 4 + variant) {
#define HDG_UCASE(N)                                                                 \
  case N * 4 + 0: return run_units<N, epb_var<N, 0>()>(io, tabs, smem, u0, u1);   \
  case N * 4 + 1: return run_units<N, epb_var<N, 1>()>(io, tabs, smem, u0, u1);   \
  case N * 4 + 2: return run_units<N, epb_var<N, 2>()>(io, tabs, smem, u0, u1);
    HDG_UCASE(2) HDG_UCASE(3) HDG_UCASE(4) HDG_UCASE(5) HDG_UCASE(6) HDG_UCASE(7)
    HDG_UCASE(8) HDG_UCASE(9) HDG_UCASE(10) HDG_UCASE(11)
#undef HDG_UCASE
    default: return 0.0;
  }
}

// Pencil form: columns [pen0, pen1) of one problem (column pen = ig + n_ig j,
// whole columns along x3) through the pencil march of pencil_unit.hpp at
// degree NP - 1 and EPB slots; with final_x only the last x update of a
// finished solve.  Tables from the batch table buffer into LDS (after a
// barrier: the previous run, possibly of another degree, shares the LDS).
template <int NP, int EPB>
__device__ inline double run_pencils(const BatchArgs& a, const MeshDev& m, double* smem, int tid,
                                     int64_t off, int it, int pen0, int pen1, double alpha,
                                     double beta, bool final_x) {
  constexpr int o = batch_tab_off(NP);
  const double* tp = a.tabs;
  asm volatile("" : "+s"(tp));
  cdouble* ct = (cdouble*)tp;
  auto& sm = *reinterpret_cast<PencilSmem<double, NP, EPB>*>(smem);
  __syncthreads();
  if (tid < NP) {
    sm.bs[tid] = PencilPair<double>{ct[o + tid], ct[o + NP + tid]};
    sm.lam[tid] = ct[o + 2 * NP + tid];
  }
  const double H = ct[o + 3 * NP];
  const UnitLane Ln = unit_lane<NP, EPB>(tid);
  const int n_ig = (m.n1 + EPB - 1) / EPB;
  const double* __restrict__ z = a.z + off;
  const double* __restrict__ pin = ((it & 1) ? a.p0 : a.p1) + off;   // p_{k-1}
  double* __restrict__ pout = ((it & 1) ? a.p1 : a.p0) + off;        // p_k
  double* __restrict__ x = a.x + off;
  double* __restrict__ qa = a.qa + off;
  double* __restrict__ qb = a.qb + off;
  const int plane = m.n1 * m.n2;
  double dot = 0.0;
  for (int pen = pen0; pen < pen1; ++pen) {
    const int ig = pen % n_ig, j = pen / n_ig;
    const int i = ig * EPB + Ln.slot;
    const bool act = Ln.slot < EPB && i < m.n1 && Ln.colok;
    const int ic = min(i, m.n1 - 1);
    PencilRow row;
    pencil_row(m, ic, j, row);
    if (final_x) {
      pencil_final_x<double, NP>(m, row, act, Ln.col, 0, m.n3, alpha, pin, x);
      continue;
    }
    const int rowe = m.n1 * j + ic;
    PencilLoads<double> L;
    pencil_load<double, NP>(m, z, pin, x, row, 0, act, Ln.col, rowe, true, L);
    double carry_p = 0, carry_w = 0;
    for (int k = 0; k < m.n3; ++k) {
      const int kn = min(k + 1, m.n3 - 1);
      pencil_step<double, NP, EPB>(z, pin, pout, x, qa, qb, sm, Ln, act, m, row, k, kn,
                                   rowe + plane * kn, L, k == 0, k + 1 == m.n3, alpha, beta, H, H,
                                   0.0, carry_p, carry_w, &dot);
    }
  }
  return dot;
}

__device__ inline double dispatch_pencils(int np, int variant, const BatchArgs& a,
                                          const MeshDev& m, double* smem, int64_t off, int it,
                                          int pen0, int pen1, double alpha, double beta,
                                          bool final_x) {
  // the thread index through an empty asm (see run_units)
  int tid = (int)threadIdx.x;
  asm volatile("" : "+v"(tid));
  switch (np * 4 + variant) {
#define HDG_PCASE(N)                                                                           \
  case N * 4 + 0:                                                                              \
    return run_pencils<N, epb_var<N, 0>()>(a, m, smem, tid, off, it, pen0, pen1, alpha, beta,  \
                                           final_x);                                           \
  case N * 4 + 1:                                                                              \
    return run_pencils<N, epb_var<N, 1>()>(a, m, smem, tid, off, it, pen0, pen1, alpha, beta,  \
                                           final_x);                                           \
  case N * 4 + 2:                                                                              \
    return run_pencils<N, epb_var<N, 2>()>(a, m, smem, tid, off, it, pen0, pen1, alpha, beta,  \
                                           final_x);
    HDG_PCASE(2) HDG_PCASE(3) HDG_PCASE(4) HDG_PCASE(5) HDG_PCASE(6) HDG_PCASE(7)
    HDG_PCASE(8) HDG_PCASE(9) HDG_PCASE(10) HDG_PCASE(11)
#undef HDG_PCASE
    default: return 0.0;
  }
}

// ---- the work of one segment in each phase ----------------------------------
// Every function below handles one segment of one phase of CG iteration `it`.

// Two-phase forms, start: z = D^-1 b, x = 0, p_{-1} = 0 on vector segment s,
// and the segment's partials of r.z and r.r for iteration 0.
__device__ __forceinline__ void init_seg_two_phase(const BatchArgs& a, int s, double* s_red) {
  const BatchSeg sg = a.vseg[s];
  const int64_t off = a.probs[sg.prob].off;
  double rz = 0.0, rr = 0.0;
  for (int64_t g = off + sg.begin + threadIdx.x; g < off + sg.end; g += kBT) {
    const double v = a.b[g];
    const double zv = a.dinv[g] * v;
    a.z[g] = zv;
    a.x[g] = 0.0;
    a.p1[g] = 0.0;
    rz += v * zv;
    rr += v * v;
  }
  const double brz = block_sum<kBT>(rz, s_red);
  const double brr = block_sum<kBT>(rr, s_red);
  if (threadIdx.x == 0) {
    a.prz[s] = brz;
    a.prr[s] = brr;
  }
}

// One-phase form, start: z_0 = D^-1 b in slot 0, x = 0, p_{-1} = s_{-1} = 0
// (slot 1) on vector segment s.
__device__ __forceinline__ void init_seg_one_phase(const BatchArgs& a, int s) {
  const BatchSeg sg = a.vseg[s];
  const int64_t off = a.probs[sg.prob].off;
  for (int64_t g = off + sg.begin + threadIdx.x; g < off + sg.end; g += kBT) {
    a.z[g] = a.dinv[g] * a.b[g];
    a.x[g] = 0.0;
    a.p1[g] = 0.0;
    a.s1[g] = 0.0;
  }
}

// Two-phase form, apply phase: re-sum the problem's r.z and r.r partials of
// the previous update in a fixed order, decide convergence (the owner of the
// problem's first segment records it in slot B), form p = z + beta p_old on
// the segment's units, make the previous iteration's x step x += alpha p_old
// on the faces they own, and apply the operator; one p.q partial per
// segment.  The apply that detects the stop only makes that last x step.
__device__ __forceinline__ void apply_seg(const BatchArgs& a, int s, int it, double* smem, double* s_red) {
  const BatchSeg sg = a.useg[s];
  const int pb = uni_int(sg.prob);
  const BatchProbDev* P = a.probs + pb;
  if (a.A[pb].done != 0) return;
  const double rho_prev = a.A[pb].rho;
  double rr_stop = a.A[pb].rr_stop;
  double rho, rr;
  sum_partials2<kBT>(a.prz + P->vseg_begin, a.prr + P->vseg_begin, P->n_vsegs, s_red, &rho, &rr);
  if (it == 0) rr_stop = P->rtol2 * rr;
  const double bb = (it == 0) ? 0.0 : rho / rho_prev;
  int done = 0;
  if (!isfinite(rr) || !isfinite(bb)) done = 3;
  else if (rr <= rr_stop) done = 1;
  else if (it >= P->maxit) done = 2;
  if (s == P->useg_begin && threadIdx.x == 0) {
    a.B[pb].rho = rho;
    a.B[pb].rr = rr;
    a.B[pb].rr_stop = rr_stop;
    a.B[pb].iter = it;
    a.B[pb].done = done;
  }
  const int64_t off = P->off;
  UnitIO<double> io{};
  io.info = uni_ptr(P->info);
  io.lam = uni_ptr(P->lam);
  io.n_elem = uni_int(P->n_elem);
  io.nff = uni_int(P->nff);
  io.p_in = uni_ptr(((it & 1) ? a.p0 : a.p1) + off);   // p_{k-1}
  io.x = uni_ptr(a.x + off);
  io.alpha = uni_f64(a.A[pb].alpha);                     // alpha_{k-1}, 0 before the first update
  if (done) {                             // the last x step, then the solve is complete
    dispatch_final_x(uni_int(P->np), uni_int(P->variant), io, sg.begin, sg.end);
    return;
  }
  io.qa = uni_ptr(a.qa + off);
  io.qb = uni_ptr(a.qb + off);
  io.z = uni_ptr(a.z + off);
  io.p_out = uni_ptr(((it & 1) ? a.p1 : a.p0) + off);
  io.beta = uni_f64(bb);
  const double dot =
      dispatch_units(uni_int(P->np), uni_int(P->variant), io, a.tabs, smem, sg.begin, sg.end);
  const double bs = block_sum<kBT>(dot, s_red);
  if (threadIdx.x == 0) a.ppq[s] = bs;
}

// Update-phase bookkeeping shared by the two-phase forms: decisions read slot
// B (slot A is written in this phase).  Returns false when the segment has
// nothing to update (problem finished or broken down), else true with alpha.
__device__ __forceinline__ bool update_alpha(const BatchArgs& a, int s, int it, double* s_red,
                                             double* alpha_out) {
  const BatchSeg sg = a.vseg[s];
  const int pb = uni_int(sg.prob);
  const BatchProbDev* P = a.probs + pb;
  const int bdone = a.B[pb].done;
  const bool owner = (s == P->vseg_begin) && threadIdx.x == 0;
  if (bdone == 0 && a.A[pb].done != 0) return false;   // broke down in an earlier update
  if (bdone) {
    if (owner && a.A[pb].done == 0) {                 // finished in this iteration's apply
      a.A[pb].done = bdone;
      a.A[pb].iter = a.B[pb].iter;
      a.A[pb].rr = a.B[pb].rr;
      a.A[pb].rr_stop = a.B[pb].rr_stop;
      atomicAdd(&a.bar->done_count, 1u);
    }
    return false;
  }
  const double pq = sum_partials<kBT>(a.ppq + P->useg_begin, P->n_usegs, 1, 0, s_red);
  const double rho = a.B[pb].rho;
  const double alpha = rho / pq;
  if (!(pq > 0.0) || !isfinite(alpha)) {
    if (owner) {
      a.A[pb].done = 3;
      a.A[pb].iter = it;
      atomicAdd(&a.bar->done_count, 1u);
    }
    return false;
  }
  if (owner) {
    a.A[pb].rho = rho;
    a.A[pb].alpha = alpha;
    a.A[pb].rr_stop = a.B[pb].rr_stop;
    a.A[pb].rr = a.B[pb].rr;
    a.A[pb].iter = it + 1;
  }
  *alpha_out = alpha;
  return true;
}

// Two-phase form, update phase: alpha from the problem's p.q partials, then
// z -= alpha D^-1 (qa + qb) and the segment's r.z, r.r partials (x takes its
// step alpha p in the next apply phase).
__device__ __forceinline__ void update_seg(const BatchArgs& a, int s, int it, double* s_red) {
  double alpha;
  if (!update_alpha(a, s, it, s_red, &alpha)) return;
  const BatchSeg sg = a.vseg[s];
  const BatchProbDev* P = a.probs + uni_int(sg.prob);
  const int64_t lo = P->off + sg.begin, hi = P->off + sg.end;
  double rz = 0.0, rr = 0.0;
  int64_t g = lo + threadIdx.x;
  constexpr int U = 8;
  for (; g + (U - 1) * kBT < hi; g += U * kBT) {
    double zv[U], q[U], d[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      zv[k] = a.z[g + k * kBT];
      q[k] = a.qa[g + k * kBT] + a.qb[g + k * kBT];
      d[k] = a.dinv[g + k * kBT];
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const double zn = zv[k] - alpha * (d[k] * q[k]);
      a.z[g + k * kBT] = zn;
      const double rn = div_fast(zn, d[k]);
      rz += zn * rn;
      rr += rn * rn;
    }
  }
  for (; g < hi; g += kBT) {
    const double d = a.dinv[g];
    const double zn = a.z[g] - alpha * (d * (a.qa[g] + a.qb[g]));
    a.z[g] = zn;
    const double rn = div_fast(zn, d);
    rz += zn * rn;
    rr += rn * rn;
  }
  const double brz = block_sum<kBT>(rz, s_red);
  const double brr = block_sum<kBT>(rr, s_red);
  if (threadIdx.x == 0) {
    a.prz[s] = brz;
    a.prr[s] = brr;
  }
}

// One-phase form: every iteration is one pass over the element segments, as
// the single-problem one-kernel CG (Chronopoulos-Gear recurrences): per
// segment the problem's partials of the previous pass (z.Az, r.z, r.r of
// iterate k - 1, parity slot (k - 1) & 1) are re-summed in a fixed order,
// convergence is decided and alpha_{k-1}, beta_{k-1} formed; then each unit
// updates s, z and, on the faces it owns, p and x, and applies the operator
// to the new z.  Slots alternate with the parity rd = k & 1 exactly as the
// single-problem launches do; the state slot read is A for even k, B for odd.
__device__ __forceinline__ void pass_seg(const BatchArgs& a, int s, int it, double* smem, double* s_red) {
  const int rd = it & 1;
  double* const zs[2] = {a.z, a.z1};
  double* const ps_[2] = {a.p0, a.p1};
  double* const ss[2] = {a.s0, a.s1};
  double* const qas[2] = {a.qa, a.qa1};
  double* const qbs[2] = {a.qb, a.qb1};
  const double* prev = a.pcg + (size_t)(rd ^ 1) * 3 * a.max_segs;
  double* cur = a.pcg + (size_t)rd * 3 * a.max_segs;
  const BatchSeg sg = a.useg[s];
  const int pb = uni_int(sg.prob);
  const BatchProbDev* P = a.probs + pb;
  BatchState* R = rd ? a.B + pb : a.A + pb;
  BatchState* W = rd ? a.A + pb : a.B + pb;
  const bool owner = (s == P->useg_begin) && threadIdx.x == 0;
  const int rdone = R->done;
  if (rdone) {                              // finished earlier: keep both slots equal
    if (owner && W->done == 0) *W = *R;
    return;
  }
  const int k = R->iter;
  double alpha = 0.0, beta = 0.0;
  if (k == 0) {
    if (owner) {
      W->iter = 1;
      W->done = 0;
    }
  } else {
    double del = 0.0, gam = 0.0, rr = 0.0;
    sum_partials2<kBT>(prev + P->useg_begin, prev + a.max_segs + P->useg_begin, P->n_usegs, s_red,
                       &del, &gam);
    rr = sum_partials<kBT>(prev + 2 * a.max_segs + P->useg_begin, P->n_usegs, 1, 0, s_red);
    const double rr_stop = (k == 1) ? P->rtol2 * rr : R->rr_stop;
    int done = 0;
    if (!isfinite(rr) || !isfinite(gam)) done = 3;
    else if (rr <= rr_stop) done = 1;
    else if (k - 1 >= P->maxit) done = 2;
    else {
      beta = (k == 1) ? 0.0 : gam / R->rho;
      alpha = (k == 1) ? gam / del : gam / (del - beta * gam / R->alpha);
      if (!(alpha > 0.0) || !isfinite(alpha) || !isfinite(beta)) done = 3;
    }
    if (owner) {
      W->rr = rr;
      W->rr_stop = rr_stop;
      W->done = done;
      if (done) {
        W->iter = k - 1;                    // x_{k-1} is the result
        atomicAdd(&a.bar->done_count, 1u);
      } else {
        W->rho = gam;
        W->alpha = alpha;
        W->iter = k + 1;
      }
    }
    if (done) return;
  }
  const int64_t off = P->off;
  UnitIO<double> io{};
  io.info = uni_ptr(P->info);
  io.lam = uni_ptr(P->lam);
  io.n_elem = uni_int(P->n_elem);
  io.nff = uni_int(P->nff);
  io.first = k == 0;
  io.z_old = uni_ptr((k == 0 ? zs[rd] : zs[rd ^ 1]) + off);
  io.z_new = uni_ptr(zs[rd] + off);
  io.p_in = uni_ptr(ps_[rd] + off);
  io.p_out = uni_ptr(ps_[rd ^ 1] + off);
  io.s_old = uni_ptr(ss[rd] + off);
  io.s_new = uni_ptr(ss[rd ^ 1] + off);
  io.w_a = uni_ptr(qas[rd ^ 1] + off);
  io.w_b = uni_ptr(qbs[rd ^ 1] + off);
  io.qa = uni_ptr(qas[rd] + off);
  io.qb = uni_ptr(qbs[rd] + off);
  io.dinv = uni_ptr(a.dinv + off);
  io.x = uni_ptr(a.x + off);
  io.alpha = uni_f64(alpha);
  io.beta = uni_f64(beta);
  double acc[3] = {0.0, 0.0, 0.0};
  dispatch_units_cgcg(uni_int(P->np), uni_int(P->variant), io, a.tabs, smem, sg.begin, sg.end,
                      acc);
  block_sums<kBT, 3>(acc);
  if (threadIdx.x == 0) {
    cur[s] = acc[0];
    cur[a.max_segs + s] = acc[1];
    cur[2 * a.max_segs + s] = acc[2];
  }
}

// One-phase form, after the last pass: a problem decided in an odd pass wrote
// slot A, in an even pass slot B; the host reads A.
__device__ __forceinline__ void pass_result(const BatchArgs& a, int s) {
  const BatchSeg sg = a.useg[s];
  const BatchProbDev* P = a.probs + sg.prob;
  if (s == P->useg_begin && threadIdx.x == 0 && a.A[sg.prob].done == 0 && a.B[sg.prob].done != 0)
    a.A[sg.prob] = a.B[sg.prob];
}

// Two-phase form on the pencil march (form 2), apply phase: as apply_seg,
// but the segment is a range of whole columns along x3; p and x (x +=
// alpha_{k-1} p_{k-1}) are updated on the faces the columns own and the x3
// faces of a column are summed in registers.  The apply that detects the
// stop still makes the last x update.
__device__ __forceinline__ void pencil_apply_seg(const BatchArgs& a, int s, int it, double* smem,
                                        double* s_red) {
  const BatchSeg sg = a.useg[s];
  const int pb = uni_int(sg.prob);
  const BatchProbDev* P = a.probs + pb;
  if (a.A[pb].done != 0) return;
  const double rho_prev = a.A[pb].rho;
  const double alpha = uni_f64(a.A[pb].alpha);   // alpha_{k-1}, 0 before the first update
  double rr_stop = a.A[pb].rr_stop;
  double rho, rr;
  sum_partials2<kBT>(a.prz + P->vseg_begin, a.prr + P->vseg_begin, P->n_vsegs, s_red, &rho, &rr);
  if (it == 0) rr_stop = P->rtol2 * rr;
  const double bb = (it == 0) ? 0.0 : rho / rho_prev;
  int done = 0;
  if (!isfinite(rr) || !isfinite(bb)) done = 3;
  else if (rr <= rr_stop) done = 1;
  else if (it >= P->maxit) done = 2;
  if (s == P->useg_begin && threadIdx.x == 0) {
    a.B[pb].rho = rho;
    a.B[pb].rr = rr;
    a.B[pb].rr_stop = rr_stop;
    a.B[pb].iter = it;
    a.B[pb].done = done;
  }
  const double dot = dispatch_pencils(uni_int(P->np), uni_int(P->variant), a, a.meshes[pb], smem,
                                      P->off, it, sg.begin, sg.end, alpha, uni_f64(bb), done != 0);
  if (done) return;                         // the last x update is in
  const double bs = block_sum<kBT>(dot, s_red);
  if (threadIdx.x == 0) a.ppq[s] = bs;
}

// Pencil form, update phase: z -= alpha D^-1 w with w = qa + qb, except on
// the problem's free x3 faces, whose qa holds the sum.
__device__ __forceinline__ void pencil_update_seg(const BatchArgs& a, int s, int it, double* s_red) {
  double alpha;
  if (!update_alpha(a, s, it, s_red, &alpha)) return;
  const BatchSeg sg = a.vseg[s];
  const BatchProbDev* P = a.probs + uni_int(sg.prob);
  const int64_t off = P->off;
  const int x3_lo = P->x3_lo, x3_hi = P->x3_hi;
  double rz = 0.0, rr = 0.0;
  // eight entries per thread with all their loads in flight together
  // (entries past the segment read its first entry and are dropped)
  constexpr int U = 8;
  for (int r0 = sg.begin + (int)threadIdx.x; r0 < sg.end; r0 += U * kBT) {
    double d[U], w[U], zv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = r0 + u * kBT;
      const int64_t g = off + (r < sg.end ? r : sg.begin);
      d[u] = a.dinv[g];
      zv[u] = a.z[g];
      w[u] = a.qa[g];
      if (r < x3_lo || r >= x3_hi) w[u] += a.qb[g];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = r0 + u * kBT;
      if (r >= sg.end) continue;
      const double zn = zv[u] - alpha * (d[u] * w[u]);
      a.z[off + r] = zn;
      const double rn = div_fast(zn, d[u]);
      rz += zn * rn;
      rr += rn * rn;
    }
  }
  const double brz = block_sum<kBT>(rz, s_red);
  const double brr = block_sum<kBT>(rr, s_red);
  if (threadIdx.x == 0) {
    a.prz[s] = brz;
    a.prr[s] = brr;
  }
}

template <int FORM>
struct FormTraits {
  static constexpr int phases = FORM == 1 ? 1 : 2;
  static constexpr int lds_words = FORM == 2 ? kBatchPencilLdsWords : kBatchLdsWords;
};

template <int FORM>
__device__ __forceinline__ void init_seg(const BatchArgs& a, int s, double* s_red) {
  if constexpr (FORM == 1) init_seg_one_phase(a, s);
  else init_seg_two_phase(a, s, s_red);
}

// Phase 0: the element segments; phase 1 (two-phase forms): the vector segments.
template <int FORM>
__device__ __forceinline__ void run_seg(const BatchArgs& a, int phase, int s, int it, double* smem,
                               double* s_red) {
  if constexpr (FORM == 0) {
    if (phase == 0) apply_seg(a, s, it, smem, s_red);
    else update_seg(a, s, it, s_red);
  } else if constexpr (FORM == 1) {
    pass_seg(a, s, it, smem, s_red);
  } else {
    if (phase == 0) pencil_apply_seg(a, s, it, smem, s_red);
    else pencil_update_seg(a, s, it, s_red);
  }
}

// ---- the persistent kernel ----------------------------------------------------
// Every block owns one contiguous range of segments per phase; all problems
// iterate in lockstep phases separated by grid barriers; converged problems
// drop out and the kernel returns when every problem is done.  The one-phase
// form numbers its blocks so that consecutive ranges sit on one XCD
// (neighbouring elements of a problem, whose shared faces both read, meet in
// the same L2).
// Blocks per CU: two for the two-phase form (201 registers, no spill; with
// its element pass keeping the next unit's loads in flight it measured 470
// against 490 us per iteration of the 256-problem batch at three, where it
// spilled 84 bytes per lane), three for the others: four fit the one-phase
// form's paths in 128 registers (a 100-byte spill) but measured slower (630
// against 583 us), and the pencil form measured slower at two (615 against
// 578 us).
template <int FORM>
__global__ void __launch_bounds__(kBT, FORM == 0 ? 2 : 3) batch_cg_kernel(BatchArgs a) {
  __shared__ double smem[FormTraits<FORM>::lds_words];
  __shared__ double s_red[kBT / 64];
  const int bid = FORM == 1 ? xcd_remap((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  unsigned epoch = 0;
  for (int s = a.vseg_range[bid]; s < a.vseg_range[bid + 1]; ++s) init_seg<FORM>(a, s, s_red);
  if (!grid_sync(a, ++epoch)) return;
  for (int it = 0; it < a.max_iters; ++it) {
    for (int s = a.useg_range[bid]; s < a.useg_range[bid + 1]; ++s)
      run_seg<FORM>(a, 0, s, it, smem, s_red);
    if (!grid_sync(a, ++epoch)) return;
    if constexpr (FormTraits<FORM>::phases == 2) {
      for (int s = a.vseg_range[bid]; s < a.vseg_range[bid + 1]; ++s)
        run_seg<FORM>(a, 1, s, it, smem, s_red);
      if (!grid_sync(a, ++epoch)) return;
    }
    if (__hip_atomic_load(&a.bar->done_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
        (unsigned)a.n_probs)
      break;
  }
  if constexpr (FORM == 1)
    for (int s = a.useg_range[bid]; s < a.useg_range[bid + 1]; ++s) pass_result(a, s);
}

// State reset before every batched solve (a kernel, so that it can sit in the
// captured graph next to the solver).
__global__ void batch_reset_kernel(BatchState* A, BatchState* B, GridBar* bar, unsigned* flags,
                                   int n_probs, int n_flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_probs) {
    BatchState s{};
    s.rho = 1.0;
    A[i] = s;
    B[i] = s;
  }
  if (i < n_flags) {
    flags[(size_t)i * kFlagStride] = 0u;                                // arrival
    flags[((size_t)n_flags + i) * kFlagStride] = 0u;                    // release
  }
  if (i == 0) {
    bar->pad0 = 0;
    bar->done_count = 0;
    bar->err = 0;
  }
}

namespace {
const void* batch_kernel_fn(int form) {
  return form == 1   ? reinterpret_cast<const void*>(batch_cg_kernel<1>)
         : form == 2 ? reinterpret_cast<const void*>(batch_cg_kernel<2>)
                     : reinterpret_cast<const void*>(batch_cg_kernel<0>);
}
}  // namespace

hipError_t batch_occupancy(int form, int* blocks_per_cu) {
  // the grid must be co-resident
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batch_kernel_fn(form), kBT,
                                                      0);
}

hipError_t launch_batch_reset(BatchState* A, BatchState* B, GridBar* bar, unsigned* flags,
                              int n_probs, int nblocks, hipStream_t s) {
  const int n = n_probs > nblocks ? n_probs : nblocks;
  const int nb = (n + 255) / 256 > 0 ? (n + 255) / 256 : 1;
  hipLaunchKernelGGL(batch_reset_kernel, dim3(nb), dim3(256), 0, s, A, B, bar, flags, n_probs,
                     nblocks);
  return hipGetLastError();
}

hipError_t launch_batch_cg(const BatchArgs& args, int nblocks, hipStream_t s) {
  if (nblocks < 1 || nblocks > kBT * kMaxBlocksPerThread) return hipErrorInvalidValue;
  if (args.form < 0 || args.form > 2) return hipErrorInvalidValue;
  BatchArgs a = args;
  void* params[] = {&a};
  return hipLaunchCooperativeKernel(batch_kernel_fn(a.form), dim3(nblocks), dim3(kBT), params, 0,
                                    s);
}

}  // namespace hdg
