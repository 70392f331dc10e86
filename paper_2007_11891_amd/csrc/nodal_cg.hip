// Nodal-basis CG solvers of the paper's solver comparison (section "Summary
// of solution method"): HDG-unprec (no preconditioner), HDG-diag (the main
// diagonal of the inverse face blocks) and HDG-block (the inverse face
// blocks, algorithm "Block_Preconditioner"), beside HDG-trans, the
// transformed solver of elem_kernels.hip / vec_kernels.hip.
//
// The operator is applied in the nodal trace basis, as the paper's untransformed
// solvers do: the face transform of p into the eigen-face basis
// (S^T M x S^T M), the transformed element operator, and the transform of the
// residual back (M S x M S).  The preconditioners (section "Preconditioners"):
// the transformed face block of K is diagonal (entries y), so the inverse
// face block is (S x S) diag(1 / y) (S^T x S^T) -- transform with S^T, scale,
// transform with S -- and its main diagonal is ((S o S) x (S o S)) (1 / y)
// per face (o: entrywise square), computed once per solve.  1 / y is the
// eigen-basis Jacobi diagonal of HDG-trans.
//
// One iteration is four launches: ncg_in (state slot A -> B, beta,
// p = z + beta p, p^ = (S^T M x S^T M) p), the element apply of p^, ncg_out
// (q = (M S x M S)(qa + qb), p.q partials) and the update (alpha,
// x += alpha p, r -= alpha q, z = P^-1 r; slot B -> A), a vector kernel for
// HDG-unprec / HDG-diag and a face kernel for HDG-block.  Reductions are
// fixed-order sums of block partials, as in the transformed CG; partial slot
// k & 1 holds iteration k's r.z, r.r and p.q.
#include "device_common.hpp"

namespace hdg {

// Face kernels: FPB whole faces per block, one thread per face node, and a
// grid of at most kNcgFaceGridMax blocks looping over face groups.
constexpr int kNcgFaceGridMax = 2048;
template <int NP>
struct NcgFace {
  static constexpr int NF = NP * NP;
  static constexpr int FPB = (256 / NF) > 0 ? 256 / NF : 1;
  static constexpr int NT = (FPB * NF + 63) / 64 * 64;
};
constexpr int kNcgVecThreads = 256;
constexpr int kNcgUnroll = 4;

struct NcgArgs {
  int64_t n;             // free trace length
  int64_t n_faces;       // free faces
  const double* m_in;    // S^T M  (n_p x n_p, row-major)
  const double* m_out;   // M S
  const double* m_st;    // S^T
  const double* m_s;     // S
  double* x;
  double* r;
  double* z;
  double* p;
  double* phat;
  double* q;
  const double* qa;
  const double* qb;
  const double* b;       // right-hand side (init)
  const double* pd;      // HDG-diag: nodal diagonal of the inverse face blocks
  const double* dinv;    // HDG-block: 1 / y, eigen-face basis
  double* partials;      // pq[2][pmax] | rz[2][pmax] | rr[2][pmax]
  int pmax;
  int n_face_blocks;     // partials written by a face kernel
  int n_vec_blocks;      // partials written by a vector kernel
  int precond;           // 0 none, 2 diagonal, 3 block
  CgScalars* sc;
};

// The two rows of a 1D matrix A (n_p x n_p, row-major) a thread needs for
// (A x A) on its face node (qa, qb) = (lt % n_p, lt / n_p).
template <int NP>
struct Rows {
  double a[NP], b[NP];
  __device__ inline void load(const double* __restrict__ A, int lt, bool active) {
    const int qa = active ? lt % NP : 0, qb = active ? lt / NP : 0;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      a[k] = A[qa * NP + k];
      b[k] = A[qb * NP + k];
    }
  }
};

// (A x A) applied to the face held in s_in (n_p x n_p, lower index fastest):
// t[a, c] = sum_b A[a, b] in[b, c], then out[a, c] = sum_d A[c, d] t[a, d].
// Every thread of the block calls it (two barriers).
template <int NP>
__device__ inline double face_tt(const Rows<NP>& A, const double* s_in, double* s_t, int lt,
                                 bool active) {
  const int qa = lt % NP, qb = lt / NP;
  if (active) {
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < NP; ++b) acc += A.a[b] * s_in[b + NP * qb];
    s_t[lt] = acc;
  }
  __syncthreads();
  double out = 0.0;
  if (active) {
#pragma unroll
    for (int d = 0; d < NP; ++d) out += A.b[d] * s_t[qa + NP * d];
  }
  __syncthreads();
  return out;
}

// First kernel of iteration k: reads slot A, sums the r.z and r.r partials of
// iteration k, decides convergence, publishes slot B (block 0), then
// p = z + beta p and p^ = (S^T M x S^T M) p on every free face.
template <int NP>
__global__ void __launch_bounds__(NcgFace<NP>::NT) ncg_in_kernel(NcgArgs a) {
  using F = NcgFace<NP>;
  constexpr int NF = F::NF, FPB = F::FPB, NT = F::NT;
  __shared__ double s_in[FPB][NF];
  __shared__ double s_t[FPB][NF];
  if (a.sc->A.done) return;                  // uniform over the grid
  const int it = a.sc->A.iter;
  const int k2 = it & 1;
  // issued together: the partials, the first face group's z and p, A's rows
  // partials of HDG-block come from the face-structured update
  const int nparts = a.precond == 3 ? a.n_face_blocks : a.n_vec_blocks;
  const double* pp[2] = {a.partials + (size_t)(2 + k2) * a.pmax,
                         a.partials + (size_t)(4 + k2) * a.pmax};
  PartialSums<NT, 2> sums;
  sums.issue(pp, nparts);
  const int slot = threadIdx.x / NF;
  const int lt = threadIdx.x - slot * NF;
  const int sl = slot < FPB ? slot : 0;
  const int64_t groups = (a.n_faces + FPB - 1) / FPB;
  int64_t g = blockIdx.x;
  double zv = 0.0, pv = 0.0;
  {
    const int64_t f = g * FPB + slot;
    if (g < groups && slot < FPB && f < a.n_faces) {
      zv = a.z[f * NF + lt];
      pv = a.p[f * NF + lt];
    }
  }
  Rows<NP> A;
  A.load(a.m_in, lt, slot < FPB);
  const double rho_prev = a.sc->A.rho;
  const double rtol2 = a.sc->A.rtol2;
  const int maxit = a.sc->A.maxit;
  double rr_stop = a.sc->A.rr_stop;
  double red[2];
  sums.reduce(pp, nparts, red);
  const double rho = red[0], rr = red[1];
  if (it == 0) rr_stop = rtol2 * rr;
  const double beta = (it == 0) ? 0.0 : rho / rho_prev;
  int done = 0;
  if (!isfinite(rr) || !isfinite(beta)) done = 3;
  else if (rr <= rr_stop) done = 1;
  else if (it >= maxit) done = 2;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.sc->B.rho = rho;
    a.sc->B.rr = rr;
    a.sc->B.rr_stop = rr_stop;
    a.sc->B.iter = it;
    a.sc->B.maxit = maxit;
    a.sc->B.rtol2 = rtol2;
    a.sc->B.done = done;
  }
  if (done) return;
  for (; g < groups; g += gridDim.x) {
    const int64_t f = g * FPB + slot;
    const bool active = slot < FPB && f < a.n_faces;
    const int64_t i = f * NF + lt;
    if (g != (int64_t)blockIdx.x && active) {   // later groups: load here
      zv = a.z[i];
      pv = a.p[i];
    }
    if (active) {
      const double v = zv + beta * pv;
      a.p[i] = v;
      s_in[slot][lt] = v;
    }
    __syncthreads();
    const double o = face_tt<NP>(A, s_in[sl], s_t[sl], lt, active);
    if (active) a.phat[i] = o;
  }
}

// q = (M S x M S)(qa + qb) on every free face; partials of p.q.
template <int NP>
__global__ void __launch_bounds__(NcgFace<NP>::NT) ncg_out_kernel(NcgArgs a) {
  using F = NcgFace<NP>;
  constexpr int NF = F::NF, FPB = F::FPB, NT = F::NT;
  __shared__ double s_in[FPB][NF];
  __shared__ double s_t[FPB][NF];
  if (a.sc->B.done || a.sc->A.done) return;  // uniform over the grid
  const int k2 = a.sc->B.iter & 1;
  const int slot = threadIdx.x / NF;
  const int lt = threadIdx.x - slot * NF;
  const int64_t groups = (a.n_faces + FPB - 1) / FPB;
  Rows<NP> A;
  A.load(a.m_out, lt, slot < FPB);
  double pq[1] = {0.0};
  for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
    const int64_t f = g * FPB + slot;
    const bool active = slot < FPB && f < a.n_faces;
    const int64_t i = f * NF + lt;
    double pv = 0.0;
    if (active) {
      s_in[slot][lt] = a.qa[i] + a.qb[i];
      pv = a.p[i];
    }
    __syncthreads();
    const double o = face_tt<NP>(A, s_in[slot < FPB ? slot : 0], s_t[slot < FPB ? slot : 0], lt,
                                 active);
    if (active) {
      a.q[i] = o;
      pq[0] += pv * o;
    }
  }
  block_sums<NT, 1>(pq);
  if (threadIdx.x == 0) a.partials[(size_t)k2 * a.pmax + blockIdx.x] = pq[0];
}

// HDG-block at the start of the solve: z = P^-1 r with
// P^-1 = (S x S) diag(1 / y) (S^T x S^T) per free face, and the partials of
// r.z and r.r of iteration 0.
template <int NP>
__global__ void __launch_bounds__(NcgFace<NP>::NT) ncg_block_init_kernel(NcgArgs a) {
  using F = NcgFace<NP>;
  constexpr int NF = F::NF, FPB = F::FPB, NT = F::NT;
  __shared__ double s_in[FPB][NF];
  __shared__ double s_t[FPB][NF];
  const int slot = threadIdx.x / NF;
  const int lt = threadIdx.x - slot * NF;
  const int sl = slot < FPB ? slot : 0;
  const int64_t groups = (a.n_faces + FPB - 1) / FPB;
  Rows<NP> At, As;
  At.load(a.m_st, lt, slot < FPB);
  As.load(a.m_s, lt, slot < FPB);
  double sums[2] = {0.0, 0.0};
  for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
    const int64_t f = g * FPB + slot;
    const bool active = slot < FPB && f < a.n_faces;
    const int64_t i = f * NF + lt;
    double rv = 0.0, dv = 0.0;
    if (active) {
      rv = a.r[i];
      dv = a.dinv[i];
      s_in[slot][lt] = rv;
    }
    __syncthreads();
    const double e = face_tt<NP>(At, s_in[sl], s_t[sl], lt, active);
    if (active) s_in[slot][lt] = dv * e;
    __syncthreads();
    const double zv = face_tt<NP>(As, s_in[sl], s_t[sl], lt, active);
    if (active) {
      a.z[i] = zv;
      sums[0] += rv * zv;
      sums[1] += rv * rv;
    }
  }
  block_sums<NT, 2>(sums);
  if (threadIdx.x == 0) {
    a.partials[(size_t)2 * a.pmax + blockIdx.x] = sums[0];
    a.partials[(size_t)4 * a.pmax + blockIdx.x] = sums[1];
  }
}

// HDG-block's update of iteration k, one face group at a time (reads slot B,
// writes slot A from block 0): alpha = rho / p.q, x += alpha p,
// r -= alpha q, z = (S x S) diag(1 / y) (S^T x S^T) r, partials of r.z and
// r.r for iteration k + 1.
template <int NP>
__global__ void __launch_bounds__(NcgFace<NP>::NT) ncg_update_block_kernel(NcgArgs a) {
  using F = NcgFace<NP>;
  constexpr int NF = F::NF, FPB = F::FPB, NT = F::NT;
  __shared__ double s_in[FPB][NF];
  __shared__ double s_t[FPB][NF];
  if (a.sc->A.done) return;                  // broke down in an earlier update
  const int done = a.sc->B.done;
  if (done) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.sc->A.done = done;
      a.sc->A.rr = a.sc->B.rr;
      a.sc->A.iter = a.sc->B.iter;
    }
    return;
  }
  const int k = a.sc->B.iter;
  const double rho = a.sc->B.rho;
  // issued together: the p.q partials, the first face group's vectors, the rows
  const double* ppq[1] = {a.partials + (size_t)(k & 1) * a.pmax};
  PartialSums<NT, 1> spq;
  spq.issue(ppq, a.n_face_blocks);
  const int slot = threadIdx.x / NF;
  const int lt = threadIdx.x - slot * NF;
  const int sl = slot < FPB ? slot : 0;
  const int64_t groups = (a.n_faces + FPB - 1) / FPB;
  int64_t g = blockIdx.x;
  double xv = 0.0, pv = 0.0, rv = 0.0, qv = 0.0, dv = 0.0;
  {
    const int64_t f = g * FPB + slot;
    if (g < groups && slot < FPB && f < a.n_faces) {
      const int64_t i = f * NF + lt;
      xv = a.x[i];
      pv = a.p[i];
      rv = a.r[i];
      qv = a.q[i];
      dv = a.dinv[i];
    }
  }
  Rows<NP> At, As;
  At.load(a.m_st, lt, slot < FPB);
  As.load(a.m_s, lt, slot < FPB);
  double pq;
  spq.reduce(ppq, a.n_face_blocks, &pq);
  const double alpha = rho / pq;
  if (!(pq > 0.0) || !isfinite(alpha)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.sc->A.done = 3;
      a.sc->A.iter = k;
      a.sc->A.pq = pq;
    }
    return;
  }
  double sums[2] = {0.0, 0.0};
  for (; g < groups; g += gridDim.x) {
    const int64_t f = g * FPB + slot;
    const bool active = slot < FPB && f < a.n_faces;
    const int64_t i = f * NF + lt;
    if (g != (int64_t)blockIdx.x && active) {   // later groups: load here
      xv = a.x[i];
      pv = a.p[i];
      rv = a.r[i];
      qv = a.q[i];
      dv = a.dinv[i];
    }
    double rn = 0.0;
    if (active) {
      rn = rv - alpha * qv;
      a.x[i] = xv + alpha * pv;
      a.r[i] = rn;
      s_in[slot][lt] = rn;
    }
    __syncthreads();
    const double e = face_tt<NP>(At, s_in[sl], s_t[sl], lt, active);
    if (active) s_in[slot][lt] = dv * e;
    __syncthreads();
    const double zv = face_tt<NP>(As, s_in[sl], s_t[sl], lt, active);
    if (active) {
      a.z[i] = zv;
      sums[0] += rn * zv;
      sums[1] += rn * rn;
    }
  }
  block_sums<NT, 2>(sums);
  const int k1 = (k + 1) & 1;
  if (threadIdx.x == 0) {
    a.partials[(size_t)(2 + k1) * a.pmax + blockIdx.x] = sums[0];
    a.partials[(size_t)(4 + k1) * a.pmax + blockIdx.x] = sums[1];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.sc->A.rho = rho;
    a.sc->A.alpha = alpha;
    a.sc->A.pq = pq;
    a.sc->A.rr_stop = a.sc->B.rr_stop;
    a.sc->A.rr = a.sc->B.rr;
    a.sc->A.iter = k + 1;
    a.sc->A.done = 0;
  }
}

// Update of iteration k for HDG-unprec and HDG-diag (reads slot B, writes
// slot A from block 0): alpha = rho / p.q, x += alpha p, r -= alpha q,
// z = r or d r, partials of r.z and r.r for iteration k + 1.
__global__ void __launch_bounds__(kNcgVecThreads) ncg_update_kernel(NcgArgs a) {
  if (a.sc->A.done) return;                  // broke down in an earlier update
  const int done = a.sc->B.done;
  if (done) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.sc->A.done = done;
      a.sc->A.rr = a.sc->B.rr;
      a.sc->A.iter = a.sc->B.iter;
    }
    return;
  }
  const int k = a.sc->B.iter;
  const double rho = a.sc->B.rho;
  const double* ppq[1] = {a.partials + (size_t)(k & 1) * a.pmax};
  PartialSums<kNcgVecThreads, 1> spq;
  spq.issue(ppq, a.n_face_blocks);
  double pq;
  spq.reduce(ppq, a.n_face_blocks, &pq);
  const double alpha = rho / pq;
  if (!(pq > 0.0) || !isfinite(alpha)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.sc->A.done = 3;
      a.sc->A.iter = k;
      a.sc->A.pq = pq;
    }
    return;
  }
  const int pc = a.precond;
  double sums[2] = {0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * kNcgVecThreads;
  for (int64_t g0 = (int64_t)blockIdx.x * kNcgVecThreads + threadIdx.x; g0 < a.n;
       g0 += kNcgUnroll * stride) {
    double xv[kNcgUnroll], pv[kNcgUnroll], rv[kNcgUnroll], qv[kNcgUnroll], dv[kNcgUnroll];
#pragma unroll
    for (int u = 0; u < kNcgUnroll; ++u) {
      const int64_t g = g0 + u * stride;
      if (g < a.n) {
        xv[u] = a.x[g];
        pv[u] = a.p[g];
        rv[u] = a.r[g];
        qv[u] = a.q[g];
        dv[u] = pc == 2 ? a.pd[g] : 1.0;
      }
    }
#pragma unroll
    for (int u = 0; u < kNcgUnroll; ++u) {
      const int64_t g = g0 + u * stride;
      if (g < a.n) {
        const double rn = rv[u] - alpha * qv[u];
        a.x[g] = xv[u] + alpha * pv[u];
        a.r[g] = rn;
        const double zn = dv[u] * rn;
        a.z[g] = zn;
        sums[0] += rn * zn;
        sums[1] += rn * rn;
      }
    }
  }
  block_sums<kNcgVecThreads, 2>(sums);
  const int k1 = (k + 1) & 1;
  if (threadIdx.x == 0) {
    a.partials[(size_t)(2 + k1) * a.pmax + blockIdx.x] = sums[0];
    a.partials[(size_t)(4 + k1) * a.pmax + blockIdx.x] = sums[1];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.sc->A.rho = rho;
    a.sc->A.alpha = alpha;
    a.sc->A.pq = pq;
    a.sc->A.rr_stop = a.sc->B.rr_stop;
    a.sc->A.rr = a.sc->B.rr;
    a.sc->A.iter = k + 1;
    a.sc->A.done = 0;
  }
}

// Start of the solve: x = 0, r = b, p = 0, and for HDG-unprec / HDG-diag
// z = b or d b with the partials of r.z and r.r of iteration 0 (HDG-block's
// come from ncg_block_init_kernel).
__global__ void __launch_bounds__(kNcgVecThreads) ncg_init_kernel(NcgArgs a) {
  const int pc = a.precond;
  double sums[2] = {0.0, 0.0};
  for (int64_t g = (int64_t)blockIdx.x * kNcgVecThreads + threadIdx.x; g < a.n;
       g += (int64_t)gridDim.x * kNcgVecThreads) {
    const double bv = a.b[g];
    a.x[g] = 0.0;
    a.r[g] = bv;
    a.p[g] = 0.0;
    if (pc != 3) {
      const double zv = (pc == 2 ? a.pd[g] : 1.0) * bv;
      a.z[g] = zv;
      sums[0] += bv * zv;
    }
    sums[1] += bv * bv;
  }
  block_sums<kNcgVecThreads, 2>(sums);
  if (threadIdx.x == 0 && pc != 3) {
    a.partials[(size_t)2 * a.pmax + blockIdx.x] = sums[0];
    a.partials[(size_t)4 * a.pmax + blockIdx.x] = sums[1];
  }
}

// ================================ launch ====================================
template <int NP>
static int ncg_face_blocks_np(int64_t n_faces) {
  constexpr int FPB = NcgFace<NP>::FPB;
  const int64_t g = (n_faces + FPB - 1) / FPB;
  return (int)(g < kNcgFaceGridMax ? (g > 0 ? g : 1) : kNcgFaceGridMax);
}

int ncg_face_blocks(int np, int64_t n_faces) {
  switch (np) {
#define HDG_CASE(N) \
  case N: return ncg_face_blocks_np<N>(n_faces);
    HDG_CASE(2) HDG_CASE(3) HDG_CASE(4) HDG_CASE(5) HDG_CASE(6) HDG_CASE(7) HDG_CASE(8)
    HDG_CASE(9) HDG_CASE(10) HDG_CASE(11) HDG_CASE(12) HDG_CASE(13) HDG_CASE(14)
    HDG_CASE(15) HDG_CASE(16) HDG_CASE(17)
#undef HDG_CASE
    default: return 1;
  }
}

static int ncg_vec_blocks(int64_t n) {
  int64_t nb = (n + kNcgVecThreads * kNcgUnroll - 1) / (kNcgVecThreads * kNcgUnroll);
  return (int)(nb < 1 ? 1 : (nb > 512 ? 512 : nb));
}

static NcgArgs ncg_args(const hdg_ctx* c, CgWork<double>& w, int precond, const double* b) {
  const int npf = c->np * c->np;
  NcgArgs a{};
  a.n = c->n_free;
  a.n_faces = c->n_free_faces;
  a.m_st = c->d_mats64;
  a.m_in = c->d_mats64 + npf;
  a.m_s = c->d_mats64 + 2 * npf;
  a.m_out = c->d_mats64 + 3 * npf;
  a.x = w.x;
  a.r = w.s[0];
  a.z = w.z;
  a.p = w.p[0];
  a.phat = w.p[1];
  a.q = w.s[1];
  a.qa = w.qa;
  a.qb = w.qb;
  a.b = b;
  a.pd = w.zz[1];
  a.dinv = w.dinv;
  a.partials = w.partials;
  a.pmax = w.pmax;
  a.n_face_blocks = ncg_face_blocks(c->np, c->n_free_faces);
  a.n_vec_blocks = ncg_vec_blocks(c->n_free);
  a.precond = precond;
  a.sc = w.sc;
  return a;
}

template <int NP>
static hipError_t ncg_face_launch(int which, const NcgArgs& a, int nb, hipStream_t s) {
  constexpr int NT = NcgFace<NP>::NT;
  if (which == 0) hipLaunchKernelGGL(ncg_in_kernel<NP>, dim3(nb), dim3(NT), 0, s, a);
  else if (which == 1) hipLaunchKernelGGL(ncg_out_kernel<NP>, dim3(nb), dim3(NT), 0, s, a);
  else if (which == 2) hipLaunchKernelGGL(ncg_update_block_kernel<NP>, dim3(nb), dim3(NT), 0, s, a);
  else hipLaunchKernelGGL(ncg_block_init_kernel<NP>, dim3(nb), dim3(NT), 0, s, a);
  return hipGetLastError();
}

// which: 0 in, 1 out, 2 HDG-block update, 3 HDG-block start
static hipError_t ncg_face(const hdg_ctx* c, int which, const NcgArgs& a, hipStream_t s) {
  const int nb = a.n_face_blocks;
  switch (c->np) {
#define HDG_CASE(N) \
  case N: return ncg_face_launch<N>(which, a, nb, s);
    HDG_CASE(2) HDG_CASE(3) HDG_CASE(4) HDG_CASE(5) HDG_CASE(6) HDG_CASE(7) HDG_CASE(8)
    HDG_CASE(9) HDG_CASE(10) HDG_CASE(11) HDG_CASE(12) HDG_CASE(13) HDG_CASE(14)
    HDG_CASE(15) HDG_CASE(16) HDG_CASE(17)
#undef HDG_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ncg_init(const hdg_ctx* c, CgWork<double>& w, int precond, const double* b,
                           hipStream_t s) {
  const NcgArgs a = ncg_args(c, w, precond, b);
  hipLaunchKernelGGL(ncg_init_kernel, dim3(a.n_vec_blocks), dim3(kNcgVecThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && precond == 3) e = ncg_face(c, 3, a, s);
  return e;
}

hipError_t launch_ncg_iter(const hdg_ctx* c, CgWork<double>& w, int precond, hipStream_t s) {
  const NcgArgs a = ncg_args(c, w, precond, nullptr);
  hipError_t e = ncg_face(c, 0, a, s);
  if (e == hipSuccess) e = launch_elem_apply<double>(c, a.phat, nullptr, w.qa, w.qb, s, w.sc);
  if (e == hipSuccess) e = ncg_face(c, 1, a, s);
  if (e != hipSuccess) return e;
  if (precond == 3) return ncg_face(c, 2, a, s);
  hipLaunchKernelGGL(ncg_update_kernel, dim3(a.n_vec_blocks), dim3(kNcgVecThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace hdg
