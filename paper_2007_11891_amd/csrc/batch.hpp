// Device-side description of a batch of independent problems.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hdg_internal.hpp"

namespace hdg {

// 1D tables (B_S columns, Lambda, H) of the degrees n_p = 2..11 at one
// tau_hat, packed: for each n_p, bs0[n_p] bs1[n_p] lam[n_p] H.
__host__ __device__ constexpr int batch_tab_off(int np) {
  return np <= 2 ? 0 : batch_tab_off(np - 1) + 3 * (np - 1) + 1;
}
constexpr int kBatchMaxNP = 11;
constexpr int kBatchTabWords = batch_tab_off(kBatchMaxNP + 1);
struct BatchTabs {
  double v[kBatchTabWords];
};

struct BatchProbDev {
  const ElemInfo* info;
  const double* lam;
  int n_elem;
  int nff;              // free faces
  int np;               // p + 1
  int variant;          // tile variant of the element work units
  int64_t off;          // offset of the free trace in the concatenated vectors
  int64_t n;            // free trace length
  int unit_begin, n_units;
  int chunk_begin, n_chunks;
  int maxit;
  int pad;
  double rtol2;
};

struct BatchState {
  double rho;       // A: rho_{k-1};  B: rho_k
  double alpha;     // A: alpha_{k-1}
  double rr_stop;
  double rr;
  int iter;
  int done;         // 0 running, 1 converged, 2 cap, 3 breakdown
  int pad0, pad1;
};

struct GridBar {
  unsigned count;
  unsigned gen;
  unsigned done_count;
  unsigned err;
};

struct BatchArgs {
  const BatchProbDev* probs;
  int n_probs;
  int max_iters;
  const int* unit_prob;
  const int* chunk_prob;
  const int* unit_range;    // [nblocks + 1]
  const int* chunk_range;   // [nblocks + 1]
  int n_units_total;
  int n_chunks_total;
  double* x;
  double* r;
  double* p0;
  double* p1;
  double* qa;
  double* qb;
  const double* dinv;
  const double* b;
  double* ppq;              // [2][n_units_total]
  double* prz;              // [2][n_chunks_total]
  double* prr;              // [2][n_chunks_total]
  BatchState* A;
  BatchState* B;
  GridBar* bar;
  BatchTabs tabs;
};

hipError_t batch_occupancy(int* blocks_per_cu);
hipError_t launch_batch_reset(BatchState* A, BatchState* B, GridBar* bar, int n, hipStream_t s);
hipError_t launch_batch_cg(const BatchArgs& args, int nblocks, hipStream_t s);
int batch_chunk();

}  // namespace hdg
