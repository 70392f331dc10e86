// One-time 1D tables (host, FP64).
#pragma once
#include <vector>

namespace hdg {

struct Tables1D {
  int p = 0, np = 0;
  double tau = 0.0;
  bool exact_mass = false;     // M exact (Gauss quadrature) instead of lumped diag(w)
  std::vector<double> x, w;    // GLL points, weights
  std::vector<double> M;       // mass matrix (row-major)
  std::vector<double> D;       // D_ij = int phi_i phi_j'     (row-major)
  std::vector<double> S;       // S^T M S = I, S^T L S = Lambda (columns = eigvecs)
  std::vector<double> Lam;     // ascending eigenvalues
  std::vector<double> BS;      // B_S[k*2+s]
  double H = 0.0;              // G + C^T M^-1 C = [[H, H01], [H01, H11]] (low, high end)
  double H11 = 0.0;
  double H01 = 0.0;            // zero for the lumped mass
  std::vector<double> St;      // S^T        (row-major, out[a] = sum_i A[a*n+i] in[i])
  std::vector<double> StM;     // S^T M
  std::vector<double> MS;      // M S
};

Tables1D make_tables(int p, double tau, bool exact_mass = false);

}  // namespace hdg
