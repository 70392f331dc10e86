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

// A contiguous piece of one problem's work owned by one block: element work
// units [begin, end) in the apply phase, free-trace entries [begin, end) in
// the vector phases (both relative to the problem).
struct BatchSeg {
  int prob;
  int begin;
  int end;
  int pad;
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
  int useg_begin, n_usegs;   // apply segments (consecutive in the global list)
  int vseg_begin, n_vsegs;   // vector segments (consecutive in the global list)
  int maxit;
  int pad;
  double rtol2;
  // pencil form: the problem's free x3 faces as a DOF range of its trace
  // (relative to off); their contributions arrive summed in qa alone
  int x3_lo, x3_hi;
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
  unsigned pad0;
  unsigned done_count;  // problems finished
  unsigned err;         // a barrier wait timed out
  unsigned pad;
};

constexpr int kFlagStride = 32;   // one 128-byte line per block arrival flag

struct BatchArgs {
  const BatchProbDev* probs;
  int n_probs;
  int max_iters;
  const BatchSeg* useg;
  const int* useg_range;    // [nblocks + 1]
  const BatchSeg* vseg;
  const int* vseg_range;    // [nblocks + 1]
  double* x;
  double* z;                // D^-1 r
  double* p0;
  double* p1;
  double* qa;
  double* qb;
  const double* dinv;
  const double* b;
  double* ppq;              // [n_useg]
  double* prz;              // [n_vseg]
  double* prr;              // [n_vseg]
  BatchState* A;
  BatchState* B;
  GridBar* bar;
  unsigned* flags;          // [2][nblocks * kFlagStride]: arrival, release lines
  const double* tabs;       // [kBatchTabWords], written by the host before the launch
  // one-phase form (Chronopoulos-Gear recurrences, one element pass per
  // iteration): second slots of z and of A z (qa, qb), the two slots of
  // s = D^-1 A p, and the per-segment partials of z.Az, r.z, r.r of both
  // parities: pcg[(slot * 3 + j) * max_segs + segment]
  int form;                 // 0 two phases (apply, update), 1 one phase, 2 two phases on
                            // the pencil march (x updated in the apply phase)
  int max_segs;
  double* z1;
  double* s0;
  double* s1;
  double* qa1;
  double* qb1;
  double* pcg;
  const MeshDev* meshes;    // pencil form: per-problem mesh records
};

// co-resident blocks per CU of the persistent kernel of a form
hipError_t batch_occupancy(int form, int* blocks_per_cu);
hipError_t launch_batch_reset(BatchState* A, BatchState* B, GridBar* bar, unsigned* flags,
                              int n_probs, int nblocks, hipStream_t s);
hipError_t launch_batch_cg(const BatchArgs& args, int nblocks, hipStream_t s);

}  // namespace hdg
