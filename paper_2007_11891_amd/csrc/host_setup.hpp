// Host-only parts of the C ABI that touch no GPU: error reporting, the trace
// layout of a mesh and the validation of creation arguments.  Plain C++ (no
// HIP header), so that it also builds and runs under host sanitizers.
#pragma once
#include <cstdint>

#include "../../include/hdg.h"

namespace hdg {

// Records a printf-style message for hdg_last_error and returns st.
hdg_status fail(hdg_status st, const char* fmt, ...);

// Face counts of the trace layout: interior faces, then the Neumann sides
// (free), then the Dirichlet sides, each side in the order (0,0), (0,1),
// (1,0), ... (2,1).  side_off[k] is the first face id of side k.
struct FaceCounts {
  int64_t n_int, n_free_faces, n_faces, n_neu;
  int64_t side_off[6];
};
FaceCounts face_counts(const int n[3], int neumann_sides);

// The checks of hdg_create_ex on its host arguments (HDG_OK or HDG_EINVAL
// with the message recorded).
hdg_status validate_create(const int n_elem[3], const double* h1, const double* h2,
                           const double* h3, int p, double tau_hat, const double* lambda_host,
                           double lambda_const, int neumann_sides, int exact_mass);

// The checks of hdg_batch_create on its host arguments.
hdg_status validate_batch_create(int count, const int* n_elem3, const int* p,
                                 const double* lambda, double tau_hat);

}  // namespace hdg
