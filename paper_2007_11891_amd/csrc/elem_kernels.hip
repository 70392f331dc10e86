// Single-problem element kernels: the plain operator application (MODE 0)
// and the fused CG application (MODE 1), both looping over work units of
// `apply_unit` (elem_unit.hpp).  The tile shape (elements per unit) is a
// template parameter; the context selects one of three variants per degree.
//
// Fused CG apply (paper: section "Summary of solution method", solver
// HDG-trans): forms p = z + beta p_old on the fly (the CG carries
// z = D^-1 r, see vec_kernels.hip), writes p on the faces it owns, and
// reduces p.q from element-local quadratic forms into one partial per block.
// Everything that needs no face gather (the x and residual updates) is left
// to the streaming update kernel.
#include "cg_state.hpp"
#include "elem_unit.hpp"

namespace hdg {

template <typename T>
struct ApplyIO {
  const T* x_free;   // plain mode: input on free faces
  const T* x_bdry;   // plain mode: input on boundary faces (tail), may be null
  T* qa;
  T* qb;
  // fused CG mode
  const T* z;
  T* p0;
  T* p1;
  double* partials;  // pq[2][pmax] | rz[2][pmax] | rr[2][pmax]
  int pmax;
  int n_upd;         // number of update-kernel partials
  CgScalars* sc;
  // one-kernel CG (MODE 2): the ping-pong buffers of slot rd (read) and
  // slot rd ^ 1 (written), resolved by the host for this launch's parity
  T* z_rd;
  T* z_wr;
  T* p_rd;
  T* p_wr;
  T* s_rd;
  T* s_wr;
  T* qa_rd;
  T* qb_rd;
  T* qa_wr;
  T* qb_wr;
  T* x;
  const T* dinv;
  int rd;            // this launch reads state slot rd and writes slot rd ^ 1
  int n_parts;       // partials per slot written by the previous launch
};

// Prologue of the one-kernel CG iteration (Chronopoulos-Gear form of the
// preconditioned CG, one global reduction per iteration), in two parts so
// that the first unit's face loads can be issued in between.  Launch k reads
// slot rd = k & 1 and writes slot rd ^ 1 (block 0).
//
// cgcg_head: a finished solve skips the launch (block 0 carries the final
// state over to the other slot); otherwise returns k.
template <typename T>
__device__ inline bool cgcg_head(const ApplyIO<T>& io, int* k) {
  CgState* R = io.rd ? &io.sc->B : &io.sc->A;
  CgState* W = io.rd ? &io.sc->A : &io.sc->B;
  const int rdone = R->done;
  *k = R->iter;
  if (rdone) {                              // uniform over the grid
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      W->done = rdone;
      W->iter = R->iter;
      W->rr = R->rr;
      W->rr_stop = R->rr_stop;
    }
    return true;
  }
  return false;
}

// cgcg_scalars: for k >= 1, sums the previous launch's partials of
// delta = z.Az, gamma = r.z and r.r (all of iterate k - 1; their loads were
// issued into ps at the start of the launch), tests
// convergence of x_{k-1}, and forms
//   beta_{k-1} = gamma_{k-1} / gamma_{k-2}            (0 for k = 1)
//   alpha_{k-1} = gamma_{k-1} / (delta_{k-1} - beta_{k-1} gamma_{k-1} / alpha_{k-2})
// (alpha_0 = gamma_0 / delta_0).  Slot fields: rho = gamma of the previous
// iterate, alpha = its alpha, iter = k.  *skip when the solve ends here.
template <typename T, int NT>
__device__ inline void cgcg_scalars(const ApplyIO<T>& io, int k, PartialSums<NT, 3>& ps,
                                    const double* const* pp, T* alpha, T* beta, bool* skip) {
  CgState* R = io.rd ? &io.sc->B : &io.sc->A;
  CgState* W = io.rd ? &io.sc->A : &io.sc->B;
  const bool leader = blockIdx.x == 0 && threadIdx.x == 0;
  const double rtol2 = R->rtol2;
  const int maxit = R->maxit;
  if (k == 0) {
    *skip = false;
    *alpha = 0;
    *beta = 0;
    if (leader) {
      W->iter = 1;
      W->rtol2 = rtol2;
      W->maxit = maxit;
      W->done = 0;
    }
    return;
  }
  double sums[3];
  ps.reduce(pp, io.n_parts, sums);
  const double del = sums[0], gam = sums[1], rr = sums[2];
  const double rr_stop = (k == 1) ? rtol2 * rr : R->rr_stop;
  int done = 0;
  double a = 0.0, b = 0.0;
  if (!isfinite(rr) || !isfinite(gam)) done = 3;
  else if (rr <= rr_stop) done = 1;
  else if (k - 1 >= maxit) done = 2;
  else {
    b = (k == 1) ? 0.0 : gam / R->rho;
    a = (k == 1) ? gam / del : gam / (del - b * gam / R->alpha);
    if (!(a > 0.0) || !isfinite(a) || !isfinite(b)) done = 3;
  }
  if (leader) {
    W->rr = rr;
    W->rr_stop = rr_stop;
    W->rtol2 = rtol2;
    W->maxit = maxit;
    W->pq = del;
    W->done = done;
    if (done) {
      W->iter = k - 1;                      // iterations completed: x_{k-1} is the result
    } else {
      W->rho = gam;
      W->alpha = a;
      W->iter = k + 1;
    }
  }
  *skip = done != 0;
  *alpha = (T)a;
  *beta = (T)b;
}

// MODE 0: plain apply, 1: fused CG apply (two-kernel CG), 2: one-kernel CG iteration.
// PIPE: the block's units run software-pipelined (chosen when a block has
// more than one unit; it costs registers).
template <typename T, int NP, int EPB, int MODE, int PIPE>
__global__ void __launch_bounds__((unit_threads<NP, EPB>()))
elem_apply_kernel(const MeshDev mesh, const ElemTab<T> tab, ApplyIO<T> io, int units_per_block) {
  constexpr int NT = unit_threads<NP, EPB>();
  __shared__ UnitSmem<T, NP, EPB> sm;
  __shared__ double s_red[NT / 64];

  UnitIO<T> u{};
  u.info = mesh.info;
  u.lam = mesh.lam;
  u.n_elem = (int)mesh.n_elem;
  u.nff = (int)mesh.n_free_faces;
  u.qa = io.qa;
  u.qb = io.qb;
  if constexpr (MODE == 0) {
    if (io.sc && io.sc->B.done) return;      // inside a finished nodal-basis CG
    u.x_free = io.x_free;
    u.x_bdry = io.x_bdry;
  } else if constexpr (MODE == 2) {
    // the first unit's element records load together with the state slot
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const UnitLane L = unit_lane<NP, EPB>((int)threadIdx.x);
    UnitRegs<T> R0;
    unit_info<T, NP, EPB>(u, L, bid * units_per_block, R0);
    // the previous launch's partials (slot rd ^ 1): delta, gamma, r.r
    const int ks = io.rd ^ 1;
    const double* pp[3] = {io.partials + (size_t)ks * io.pmax,
                           io.partials + (size_t)(2 + ks) * io.pmax,
                           io.partials + (size_t)(4 + ks) * io.pmax};
    PartialSums<NT, 3> ps;
    ps.issue(pp, io.n_parts);
    int k;
    if (cgcg_head(io, &k)) return;
    const bool first = k == 0;
    u.first = first;
    u.z_old = first ? io.z_rd : io.z_wr;       // z_k lives in slot k & 1
    u.z_new = io.z_rd;
    u.p_in = io.p_rd;                          // p_{k-2}
    u.p_out = io.p_wr;                         // p_{k-1}
    u.s_old = io.s_rd;
    u.s_new = io.s_wr;
    u.w_a = io.qa_wr;                          // A z_{k-1}, from the previous launch
    u.w_b = io.qb_wr;
    u.qa = io.qa_rd;
    u.qb = io.qb_rd;
    u.dinv = io.dinv;
    u.x = io.x;
    // the first unit's face loads go out before the scalar prologue's
    CgLoads<T> C0;
    cg2_loads<T, NP>(u, L, R0, C0);
    bool skip;
    T alpha, beta;
    cgcg_scalars<T, NT>(io, k, ps, pp, &alpha, &beta, &skip);
    if (skip) return;
    u.alpha = alpha;
    u.beta = beta;
    double acc[3] = {0.0, 0.0, 0.0};
    cg2_compute<T, NP, EPB>(u, tab, sm, L, R0, C0, acc);
    for (int un = 1; un < units_per_block; ++un)
      apply_unit<T, NP, EPB, MODE>(u, tab, sm, bid * units_per_block + un, acc);
    // z.Az, r.z, r.r of this launch's iterate, one partial each per block
    block_sums<NT, 3>(acc);
    if (threadIdx.x == 0) {
      io.partials[(size_t)io.rd * io.pmax + blockIdx.x] = acc[0];
      io.partials[(size_t)(2 + io.rd) * io.pmax + blockIdx.x] = acc[1];
      io.partials[(size_t)(4 + io.rd) * io.pmax + blockIdx.x] = acc[2];
    }
    return;
  } else {
    // MODE 1: the state slot, then the first unit's loads, then the partial
    // sums and beta
    int iter;
    if (cg_head(io.sc, &iter)) return;
    u.z = io.z;
    u.p_in = (iter & 1) ? io.p0 : io.p1;     // iteration k reads p_{k-1}, writes p_k
    u.p_out = (iter & 1) ? io.p1 : io.p0;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int k2 = iter & 1;
    const double* pp[2] = {io.partials + (size_t)(2 + k2) * io.pmax,
                           io.partials + (size_t)(4 + k2) * io.pmax};
    PartialSums<NT, 2> ps;
    ps.issue(pp, io.n_upd);
    auto scalars = [&]() -> bool {
      bool skip;
      T beta;
      cg_scalars<T, NT>(io.sc, io.n_upd, iter, ps, pp, &beta, &skip);
      u.beta = beta;
      return !skip;
    };
    double acc[3] = {0.0, 0.0, 0.0};
    if constexpr (PIPE == 0) {
      const UnitLane L = unit_lane<NP, EPB>((int)threadIdx.x);
      UnitRegs<T> R0;
      unit_info<T, NP, EPB>(u, L, bid * units_per_block, R0);
      unit_data<T, NP, 1>(u, L, R0);
      if (!scalars()) return;
      unit_compute<T, NP, EPB, 1>(u, tab, sm, L, R0, acc);
      for (int un = 1; un < units_per_block; ++un)
        apply_unit<T, NP, EPB, 1>(u, tab, sm, bid * units_per_block + un, acc);
    } else {
      if (!run_units_pipelined<T, NP, EPB, 1>(u, tab, sm, bid * units_per_block,
                                              (bid + 1) * units_per_block, acc,
                                              (int)threadIdx.x, scalars))
        return;
    }
    // one partial per block, summed by every block of the update kernel
    const double bs = block_sum<NT>(acc[0], s_red);
    if (threadIdx.x == 0) io.partials[(size_t)(iter & 1) * io.pmax + blockIdx.x] = bs;
    return;
  }
  if constexpr (MODE == 0) {
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    double acc[3] = {0.0, 0.0, 0.0};
    if constexpr (PIPE == 0) {
      for (int un = 0; un < units_per_block; ++un)
        apply_unit<T, NP, EPB, MODE>(u, tab, sm, bid * units_per_block + un, acc);
    } else {
      run_units_pipelined<T, NP, EPB, MODE>(u, tab, sm, bid * units_per_block,
                                            (bid + 1) * units_per_block, acc);
    }
  }
}

// ================================ launch ====================================
constexpr int kApplyGridMax = 2048;

// work units and the block grid for EPB elements per unit
static void grid_for(int64_t n_elem, int epb, int* nblocks, int* units_per_block) {
  const int64_t units = (n_elem + epb - 1) / epb;
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

template <int NP>
static int epb_of_variant(int v) {
  switch (v) {
    case 1: return epb_var<NP, 1>();
    case 2: return epb_var<NP, 2>();
    default: return epb_var<NP, 0>();
  }
}

template <typename T, int NP, int EPB, int MODE>
static hipError_t launch_variant(const hdg_ctx* c, const ElemTab<T>& tab, const ApplyIO<T>& io,
                                 hipStream_t s) {
  int nb, upb;
  grid_for(c->n_elem, EPB, &nb, &upb);
  if (nb == 0) return hipSuccess;
  if (MODE != 2 && upb > 1)
    hipLaunchKernelGGL((elem_apply_kernel<T, NP, EPB, MODE, (MODE != 2 ? 1 : 0)>), dim3(nb),
                       dim3(unit_threads<NP, EPB>()), 0, s, c->mesh, tab, io, upb);
  else
    hipLaunchKernelGGL((elem_apply_kernel<T, NP, EPB, MODE, 0>), dim3(nb),
                       dim3(unit_threads<NP, EPB>()), 0, s, c->mesh, tab, io, upb);
  return hipGetLastError();
}

template <typename T, int NP, int MODE>
static hipError_t launch_apply_np(const hdg_ctx* c, const ElemTab<T>& tab, const ApplyIO<T>& io,
                                  hipStream_t s) {
  switch (c->tile_variant) {
    case 1: return launch_variant<T, NP, epb_var<NP, 1>(), MODE>(c, tab, io, s);
    case 2: return launch_variant<T, NP, epb_var<NP, 2>(), MODE>(c, tab, io, s);
    default: return launch_variant<T, NP, epb_var<NP, 0>(), MODE>(c, tab, io, s);
  }
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

int tile_epb(int np, int variant) {
  switch (np) {
#define HDG_CASE(N) \
  case N: return epb_of_variant<N>(variant);
    HDG_CASE(2) HDG_CASE(3) HDG_CASE(4) HDG_CASE(5) HDG_CASE(6) HDG_CASE(7) HDG_CASE(8)
    HDG_CASE(9) HDG_CASE(10) HDG_CASE(11) HDG_CASE(12) HDG_CASE(13) HDG_CASE(14)
    HDG_CASE(15) HDG_CASE(16) HDG_CASE(17)
#undef HDG_CASE
    default: return 1;
  }
}

template <int NP>
static int threads_of_variant(int v) {
  switch (v) {
    case 1: return unit_threads<NP, epb_var<NP, 1>()>();
    case 2: return unit_threads<NP, epb_var<NP, 2>()>();
    default: return unit_threads<NP, epb_var<NP, 0>()>();
  }
}

int tile_threads(int np, int variant) {
  switch (np) {
#define HDG_CASE(N) \
  case N: return threads_of_variant<N>(variant);
    HDG_CASE(2) HDG_CASE(3) HDG_CASE(4) HDG_CASE(5) HDG_CASE(6) HDG_CASE(7) HDG_CASE(8)
    HDG_CASE(9) HDG_CASE(10) HDG_CASE(11) HDG_CASE(12) HDG_CASE(13) HDG_CASE(14)
    HDG_CASE(15) HDG_CASE(16) HDG_CASE(17)
#undef HDG_CASE
    default: return 64;
  }
}

int elem_apply_blocks(int np, int64_t n_elem, int variant) {
  int nb = 0, upb = 0;
  grid_for(n_elem, tile_epb(np, variant), &nb, &upb);
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
                             hipStream_t s, CgScalars* skip_if_done) {
  ApplyIO<T> io{};
  io.x_free = x_free;
  io.x_bdry = x_bdry;
  io.qa = qa;
  io.qb = qb;
  io.sc = skip_if_done;
  return launch_apply_dispatch<T, 0>(c, tab_of<T>(c), io, s);
}

template <typename T>
hipError_t launch_cg_apply(const hdg_ctx* c, CgWork<T>& w, hipStream_t s) {
  ApplyIO<T> io{};
  io.qa = w.qa;
  io.qb = w.qb;
  io.z = w.z;
  io.p0 = w.p[0];
  io.p1 = w.p[1];
  io.partials = w.partials;
  io.pmax = w.pmax;
  io.n_upd = w.update_blocks;
  io.sc = w.sc;
  return launch_apply_dispatch<T, 1>(c, tab_of<T>(c), io, s);
}

template <typename T>
hipError_t launch_cgcg_iter(const hdg_ctx* c, CgWork<T>& w, int rd, hipStream_t s) {
  ApplyIO<T> io{};
  const int wr = rd ^ 1;
  io.z_rd = w.zz[rd];
  io.z_wr = w.zz[wr];
  io.p_rd = w.p[rd];
  io.p_wr = w.p[wr];
  io.s_rd = w.s[rd];
  io.s_wr = w.s[wr];
  io.qa_rd = w.qq[rd][0];
  io.qb_rd = w.qq[rd][1];
  io.qa_wr = w.qq[wr][0];
  io.qb_wr = w.qq[wr][1];
  io.x = w.x;
  io.dinv = w.dinv;
  io.partials = w.partials;
  io.pmax = w.pmax;
  io.sc = w.sc;
  io.rd = rd;
  io.n_parts = w.apply_blocks;
  return launch_apply_dispatch<T, 2>(c, tab_of<T>(c), io, s);
}

template hipError_t launch_cgcg_iter<double>(const hdg_ctx*, CgWork<double>&, int, hipStream_t);
template hipError_t launch_cgcg_iter<float>(const hdg_ctx*, CgWork<float>&, int, hipStream_t);
template hipError_t launch_elem_apply<double>(const hdg_ctx*, const double*, const double*,
                                              double*, double*, hipStream_t, CgScalars*);
template hipError_t launch_elem_apply<float>(const hdg_ctx*, const float*, const float*, float*,
                                             float*, hipStream_t, CgScalars*);
template hipError_t launch_cg_apply<double>(const hdg_ctx*, CgWork<double>&, hipStream_t);
template hipError_t launch_cg_apply<float>(const hdg_ctx*, CgWork<float>&, hipStream_t);

}  // namespace hdg
