// Batched Jacobi-PCG for many independent condensed-HDG problems of uneven
// sizes and degrees in one persistent launch.
//
// All problems iterate in lockstep phases separated by grid-wide barriers:
//   apply  : every block takes its contiguous range of element work units
//            (problem, unit); per problem it re-sums the previous update's
//            partials (r.z, r.r) in a fixed order, decides convergence, forms
//            p = D^-1 r + beta p_old on the unit's faces, applies the
//            transformed operator (the same `apply_unit` as the single-problem
//            kernels, selected by degree and tile shape) and writes one p.q
//            partial per unit;
//   update : every block takes its contiguous range of vector chunks; per
//            problem it re-sums the apply partials, forms alpha and updates
//            r, writing r.z and r.r partials per chunk.
// Converged problems drop out; the kernel returns when every problem is done.
// Per-problem state lives in two slots (A: read by apply, written by update;
// B: the reverse), written by the block that owns the problem's first unit or
// chunk.  Reductions are deterministic (fixed order, identical in every block).
//
// The grid barrier spins with a bounded count: if it is ever exceeded the
// kernel raises an error flag and every block returns, so the grid always
// drains.
#include "batch.hpp"
#include "elem_unit.hpp"

namespace hdg {

constexpr int kBT = 256;                 // threads per block
constexpr int kChunk = kBT * 4;          // DOFs per update chunk
constexpr unsigned kSpinLimit = 1u << 22;

template <int NP>
__host__ __device__ constexpr int unit_lds_words() { return epb_max<NP>() * lds_elem_words<NP>(); }
__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kBatchLdsWords =
    cmax(cmax(cmax(unit_lds_words<2>(), unit_lds_words<3>()), cmax(unit_lds_words<4>(), unit_lds_words<5>())),
         cmax(cmax(cmax(unit_lds_words<6>(), unit_lds_words<7>()), cmax(unit_lds_words<8>(), unit_lds_words<9>())),
              cmax(unit_lds_words<10>(), unit_lds_words<11>())));
static_assert(kBatchLdsWords * 8 <= 60000, "batched LDS budget");

// Returns false when the barrier timed out (then every block must return).
__device__ inline bool grid_sync(GridBar* gb, unsigned nblocks) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned gen = __hip_atomic_load(&gb->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();   // release this block's writes
    const unsigned arrived =
        __hip_atomic_fetch_add(&gb->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&gb->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&gb->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(&gb->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > kSpinLimit) {
          __hip_atomic_store(&gb->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    __threadfence();   // acquire the other blocks' writes
    if (__hip_atomic_load(&gb->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

template <int NP, int EPB>
__device__ inline double unit_np(const UnitIO<double>& io, const BatchTabs& tabs, double* smem,
                                 int unit) {
  constexpr int o = batch_tab_off(NP);
  const TabRef<double> tab{tabs.v + o, tabs.v + o + NP, tabs.v + o + 2 * NP, tabs.v[o + 3 * NP]};
  return apply_unit<double, NP, EPB, 1>(io, tab, *reinterpret_cast<UnitSmem<double, NP, EPB>*>(smem),
                                       unit);
}

__device__ inline double dispatch_unit(int np, int variant, const UnitIO<double>& io,
                                       const BatchTabs& tabs, double* smem, int unit) {
  switch (np * 4 + variant) {
#define HDG_UCASE(N)                                                          \
  case N * 4 + 0: return unit_np<N, epb_var<N, 0>()>(io, tabs, smem, unit); \
  case N * 4 + 1: return unit_np<N, epb_var<N, 1>()>(io, tabs, smem, unit); \
  case N * 4 + 2: return unit_np<N, epb_var<N, 2>()>(io, tabs, smem, unit);
    HDG_UCASE(2) HDG_UCASE(3) HDG_UCASE(4) HDG_UCASE(5) HDG_UCASE(6) HDG_UCASE(7)
    HDG_UCASE(8) HDG_UCASE(9) HDG_UCASE(10) HDG_UCASE(11)
#undef HDG_UCASE
    default: return 0.0;
  }
}

__global__ void __launch_bounds__(kBT, 2) batch_cg_kernel(BatchArgs a) {
  __shared__ double smem[kBatchLdsWords];
  __shared__ double s_red[kBT / 64];
  const int bid = blockIdx.x;
  const unsigned nb = gridDim.x;
  const int NU = a.n_units_total, NC = a.n_chunks_total;

  // ---- init: r = b, x = 0, p_{-1} = 0, partials of iteration 0 -----------
  for (int c = a.chunk_range[bid]; c < a.chunk_range[bid + 1]; ++c) {
    const BatchProbDev* P = a.probs + a.chunk_prob[c];
    const int64_t lo = P->off + (int64_t)(c - P->chunk_begin) * kChunk;
    const int64_t hi = (lo + kChunk < P->off + P->n) ? lo + kChunk : P->off + P->n;
    double rz = 0.0, rr = 0.0;
    for (int64_t g = lo + threadIdx.x; g < hi; g += kBT) {
      const double v = a.b[g];
      a.r[g] = v;
      a.x[g] = 0.0;
      a.p1[g] = 0.0;
      rz += v * (a.dinv[g] * v);
      rr += v * v;
    }
    const double brz = block_sum<kBT>(rz, s_red);
    const double brr = block_sum<kBT>(rr, s_red);
    if (threadIdx.x == 0) {
      a.prz[c] = brz;
      a.prr[c] = brr;
    }
  }
  if (!grid_sync(a.bar, nb)) return;

  for (int it = 0; it < a.max_iters; ++it) {
    const int k2 = it & 1;
    // ------------------------------ apply -----------------------------------
    {
      int cur = -1;
      bool skip = true;
      UnitIO<double> io{};
      for (int u = a.unit_range[bid]; u < a.unit_range[bid + 1]; ++u) {
        const int pb = a.unit_prob[u];
        const BatchProbDev* P = a.probs + pb;
        if (pb != cur) {
          cur = pb;
          skip = a.A[pb].done != 0;
          if (!skip) {
            const double rho_prev = a.A[pb].rho;
            const double alpha_prev = a.A[pb].alpha;
            double rr_stop = a.A[pb].rr_stop;
            double rho, rr;
            sum_partials2<kBT>(a.prz + (size_t)k2 * NC + P->chunk_begin,
                               a.prr + (size_t)k2 * NC + P->chunk_begin, P->n_chunks, s_red, &rho,
                               &rr);
            if (it == 0) rr_stop = P->rtol2 * rr;
            const double bb = (it == 0) ? 0.0 : rho / rho_prev;
            int done = 0;
            if (!isfinite(rr) || !isfinite(bb)) done = 3;
            else if (rr <= rr_stop) done = 1;
            else if (it >= P->maxit) done = 2;
            io.info = P->info;
            io.lam = P->lam;
            io.n_elem = P->n_elem;
            io.nff = P->nff;
            io.qa = a.qa + P->off;
            io.qb = a.qb + P->off;
            io.r = a.r + P->off;
            io.dinv = a.dinv + P->off;
            io.p_in = ((it & 1) ? a.p0 : a.p1) + P->off;
            io.p_out = ((it & 1) ? a.p1 : a.p0) + P->off;
            io.x = a.x + P->off;
            io.beta = bb;
            io.alpha_x = alpha_prev;
            io.finish = done != 0;
            if (u == P->unit_begin && threadIdx.x == 0) {
              a.B[pb].rho = rho;
              a.B[pb].rr = rr;
              a.B[pb].rr_stop = rr_stop;
              a.B[pb].iter = it;
              a.B[pb].done = done;
            }
          }
        }
        if (skip) continue;
        const double dot = dispatch_unit(P->np, P->variant, io, a.tabs, smem, u - P->unit_begin);
        if (!io.finish) {
          const double bs = block_sum<kBT>(dot, s_red);
          if (threadIdx.x == 0) a.ppq[(size_t)k2 * NU + u] = bs;
        }
      }
    }
    if (!grid_sync(a.bar, nb)) return;
    // ------------------------------ update ----------------------------------
    {
      int cur = -1;
      bool skip = true;
      double alpha = 0.0;
      for (int c = a.chunk_range[bid]; c < a.chunk_range[bid + 1]; ++c) {
        const int pb = a.chunk_prob[c];
        const BatchProbDev* P = a.probs + pb;
        if (pb != cur) {
          cur = pb;
          // decisions read slot B only (slot A is written in this phase)
          const int bdone = a.B[pb].done;
          const bool owner = (c == P->chunk_begin) && threadIdx.x == 0;
          if (bdone == 0 && a.A[pb].done != 0) {
            skip = true;                        // broke down in an earlier update
          } else if (bdone) {
            skip = true;
            if (owner && a.A[pb].done == 0) {   // finished in this iteration's apply
              a.A[pb].done = bdone;
              a.A[pb].iter = a.B[pb].iter;
              a.A[pb].rr = a.B[pb].rr;
              a.A[pb].rr_stop = a.B[pb].rr_stop;
              atomicAdd(&a.bar->done_count, 1u);
            }
          } else {
            const double pq = sum_partials<kBT>(a.ppq + (size_t)k2 * NU + P->unit_begin,
                                                P->n_units, 1, 0, s_red);
            const double rho = a.B[pb].rho;
            alpha = rho / pq;
            if (!(pq > 0.0) || !isfinite(alpha)) {
              skip = true;
              if (owner) {
                a.A[pb].done = 3;
                a.A[pb].iter = it;
                atomicAdd(&a.bar->done_count, 1u);
              }
            } else {
              skip = false;
              if (owner) {
                a.A[pb].rho = rho;
                a.A[pb].alpha = alpha;
                a.A[pb].rr_stop = a.B[pb].rr_stop;
                a.A[pb].rr = a.B[pb].rr;
                a.A[pb].iter = it + 1;
              }
            }
          }
        }
        if (skip) continue;
        const int64_t lo = P->off + (int64_t)(c - P->chunk_begin) * kChunk;
        const int64_t hi = (lo + kChunk < P->off + P->n) ? lo + kChunk : P->off + P->n;
        double rz = 0.0, rr = 0.0;
        for (int64_t g = lo + threadIdx.x; g < hi; g += kBT) {
          const double rn = a.r[g] - alpha * (a.qa[g] + a.qb[g]);
          a.r[g] = rn;
          rz += rn * (a.dinv[g] * rn);
          rr += rn * rn;
        }
        const double brz = block_sum<kBT>(rz, s_red);
        const double brr = block_sum<kBT>(rr, s_red);
        if (threadIdx.x == 0) {
          a.prz[(size_t)(k2 ^ 1) * NC + c] = brz;
          a.prr[(size_t)(k2 ^ 1) * NC + c] = brr;
        }
      }
    }
    if (!grid_sync(a.bar, nb)) return;
    if (__hip_atomic_load(&a.bar->done_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
        (unsigned)a.n_probs)
      break;
  }
}

// State reset before every batched solve (a kernel, so that it can sit in the
// captured graph next to the solver).
__global__ void batch_reset_kernel(BatchState* A, BatchState* B, GridBar* bar, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    BatchState s{};
    s.rho = 1.0;
    A[i] = s;
    B[i] = s;
  }
  if (i == 0) {
    bar->count = 0;
    bar->gen = 0;
    bar->done_count = 0;
    bar->err = 0;
  }
}

hipError_t batch_occupancy(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batch_cg_kernel, kBT, 0);
}

hipError_t launch_batch_reset(BatchState* A, BatchState* B, GridBar* bar, int n, hipStream_t s) {
  const int nb = (n + 255) / 256 > 0 ? (n + 255) / 256 : 1;
  hipLaunchKernelGGL(batch_reset_kernel, dim3(nb), dim3(256), 0, s, A, B, bar, n);
  return hipGetLastError();
}

hipError_t launch_batch_cg(const BatchArgs& args, int nblocks, hipStream_t s) {
  BatchArgs a = args;
  void* params[] = {&a};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(batch_cg_kernel), dim3(nblocks),
                                    dim3(kBT), params, 0, s);
}

int batch_chunk() { return kChunk; }

}  // namespace hdg
