// State machine of the two-kernel CG forms (textbook preconditioned CG with
// z = D^-1 r carried instead of r; paper: section "Summary of solution
// method", solver HDG-trans): the prologue of the element launch of
// iteration k, shared by the element kernels of every two-kernel form.  The
// element launch reads state slot A and its block 0 writes slot B; the
// update launch reads B and writes A (include/hdg_internal.hpp, CgState).
#pragma once
#include "device_common.hpp"

namespace hdg {

// A finished solve skips the whole launch; otherwise returns the iteration k.
__device__ inline bool cg_head(const CgScalars* sc, int* iter) {
  *iter = sc->A.iter;
  return sc->A.done != 0;                   // uniform over the grid
}

// Reads slot A, sums the update partials (r.z and r.r of iterate k; their
// loads already issued into ps), decides convergence, publishes slot B from
// block 0 and forms beta_k = rho_k / rho_{k-1} (0 at k = 0).  *skip when the
// solve ends here: 1 converged, 2 iteration cap, 3 breakdown.
template <typename T, int NT>
__device__ inline void cg_scalars(CgScalars* sc, int n_upd, int it, PartialSums<NT, 2>& ps,
                                  const double* const* pp, T* beta, bool* skip) {
  const double rho_prev = sc->A.rho;
  const double rtol2 = sc->A.rtol2;
  const int maxit = sc->A.maxit;
  double rr_stop = sc->A.rr_stop;
  double sums[2];
  ps.reduce(pp, n_upd, sums);
  const double rho = sums[0], rr = sums[1];
  if (it == 0) rr_stop = rtol2 * rr;
  const double b = (it == 0) ? 0.0 : rho / rho_prev;
  int done = 0;
  if (!isfinite(rr) || !isfinite(b)) done = 3;
  else if (rr <= rr_stop) done = 1;
  else if (it >= maxit) done = 2;
  *skip = done != 0;
  *beta = (T)b;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->B.rho = rho;
    sc->B.rr = rr;
    sc->B.rr_stop = rr_stop;
    sc->B.iter = it;
    sc->B.maxit = maxit;
    sc->B.rtol2 = rtol2;
    sc->B.done = done;
  }
}

}  // namespace hdg
