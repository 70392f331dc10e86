// One-time 1D setup on the host, FP64 (paper: equation (element_matrices),
// equation (generalized_eigenvalue_decomposition), equation (hdgbs)).
//
// GLL points by Newton iteration on P_p', weights 2 / (p (p+1) P_p(x)^2);
// Lagrange differentiation by barycentric weights; the generalized symmetric
// eigenproblem L s = Lambda M s with the lumped (diagonal) GLL mass M is
// reduced to the ordinary one M^-1/2 L M^-1/2 v = Lambda v and solved by the
// cyclic Jacobi rotation method; S = M^-1/2 V.
#include "setup1d.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace hdg {

// Legendre P_n and its derivative at x by the three-term recurrence.
static void legendre(int n, long double x, long double* P, long double* dP) {
  long double p0 = 1.0L, p1 = x;
  if (n == 0) { *P = 1.0L; *dP = 0.0L; return; }
  for (int k = 2; k <= n; ++k) {
    long double pk = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  *P = p1;
  // P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1) for |x| < 1
  *dP = (std::fabs(x) < 1.0L) ? n * (x * p1 - p0) / (x * x - 1.0L)
                              : 0.5L * n * (n + 1) * (x > 0 ? 1.0L : ((n % 2) ? 1.0L : -1.0L));
}

static void gll(int p, std::vector<double>& x, std::vector<double>& w) {
  const int n = p + 1;
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  x[0] = -1.0;
  x[p] = 1.0;
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 1; i < p; ++i) {
    long double xi = -std::cos(pi * i / p);
    for (int it = 0; it < 100; ++it) {
      long double P, dP;
      legendre(p, xi, &P, &dP);
      // P_p'' from the Legendre equation: (1-x^2) P'' = 2x P' - p(p+1) P
      long double d2P = (2.0L * xi * dP - p * (p + 1.0L) * P) / (1.0L - xi * xi);
      long double dx = dP / d2P;
      xi -= dx;
      if (std::fabs(dx) < 1e-19L) break;
    }
    x[i] = (double)xi;
  }
  // symmetrise against round-off
  for (int i = 0; i < n / 2; ++i) {
    double a = 0.5 * (x[n - 1 - i] - x[i]);
    x[i] = -a;
    x[n - 1 - i] = a;
  }
  if (n % 2) x[n / 2] = 0.0;
  for (int i = 0; i < n; ++i) {
    long double P, dP;
    legendre(p, (long double)x[i], &P, &dP);
    w[i] = (double)(2.0L / (p * (p + 1.0L) * P * P));
  }
}

// Cyclic Jacobi eigenvalue method for a symmetric n x n matrix A (row-major,
// overwritten).  Returns eigenvectors in the columns of V.
static void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& V,
                         std::vector<double>& lam) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i * n + j] * A[i * n + j];
        if (i != j) off += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-34 * tot) break;
    for (int pp = 0; pp < n - 1; ++pp)
      for (int q = pp + 1; q < n; ++q) {
        const double apq = A[pp * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = A[pp * n + pp], aqq = A[q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) /
                         (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns pp, q: A <- A J
          const double akp = A[k * n + pp], akq = A[k * n + q];
          A[k * n + pp] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows pp, q: A <- J^T A
          const double apk = A[pp * n + k], aqk = A[q * n + k];
          A[pp * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        A[pp * n + q] = A[q * n + pp] = 0.0;
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + pp], vkq = V[k * n + q];
          V[k * n + pp] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  lam.resize(n);
  for (int i = 0; i < n; ++i) lam[i] = A[i * n + i];
}

Tables1D make_tables(int p, double tau) {
  Tables1D t;
  t.p = p;
  t.np = p + 1;
  t.tau = tau;
  const int n = t.np;
  gll(p, t.x, t.w);
  // barycentric weights and the nodal derivative matrix Dh_ij = phi_j'(x_i)
  std::vector<long double> bw(n, 1.0L);
  for (int j = 0; j < n; ++j)
    for (int m = 0; m < n; ++m)
      if (m != j) bw[j] /= ((long double)t.x[j] - (long double)t.x[m]);
  std::vector<double> Dh(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    long double diag = 0.0L;
    for (int j = 0; j < n; ++j) {
      if (i == j) continue;
      long double v = (bw[j] / bw[i]) / ((long double)t.x[i] - (long double)t.x[j]);
      Dh[i * n + j] = (double)v;
      diag -= v;
    }
    Dh[i * n + i] = (double)diag;
  }
  // D_ij = int phi_i phi_j' = w_i phi_j'(x_i) (GLL exact to degree 2p-1)
  t.D.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) t.D[i * n + j] = t.w[i] * Dh[i * n + j];
  // L = E + D M^-1 D^T, E = tau (e0 e0^T + ep ep^T)
  std::vector<double> L(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      long double s = 0.0L;
      for (int k = 0; k < n; ++k) s += (long double)t.D[i * n + k] * t.D[j * n + k] / t.w[k];
      L[i * n + j] = (double)s;
    }
  L[0] += tau;
  L[n * n - 1] += tau;
  // A = M^-1/2 L M^-1/2, A v = Lambda v, S = M^-1/2 V
  std::vector<double> A(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) A[i * n + j] = L[i * n + j] / std::sqrt(t.w[i] * t.w[j]);
  std::vector<double> V, lam;
  jacobi_eigen(n, A, V, lam);
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return lam[a] < lam[b]; });
  t.S.assign(n * n, 0.0);
  t.Lam.assign(n, 0.0);
  for (int c = 0; c < n; ++c) {
    const int src = order[c];
    t.Lam[c] = lam[src];
    // sign: first entry of clearly nonzero magnitude is positive
    double sgn = 1.0;
    for (int i = 0; i < n; ++i) {
      const double v = V[i * n + src];
      if (std::fabs(v) > 1e-8) { sgn = v > 0 ? 1.0 : -1.0; break; }
    }
    for (int i = 0; i < n; ++i) t.S[i * n + c] = sgn * V[i * n + src] / std::sqrt(t.w[i]);
  }
  // B_S = S^T B - S^T D M^-1 C with B = -tau [e0, ep], C = [-e0, ep]
  t.BS.assign(n * 2, 0.0);
  for (int k = 0; k < n; ++k) {
    long double s0 = -(long double)tau * t.S[0 * n + k];
    long double s1 = -(long double)tau * t.S[(n - 1) * n + k];
    for (int i = 0; i < n; ++i) {
      s0 += (long double)t.S[i * n + k] * t.D[i * n + 0] / t.w[0];
      s1 -= (long double)t.S[i * n + k] * t.D[i * n + (n - 1)] / t.w[n - 1];
    }
    t.BS[k * 2 + 0] = (double)s0;
    t.BS[k * 2 + 1] = (double)s1;
  }
  // H = G + C^T M^-1 C = (tau + 1/w_0) I_2 for GLL end points
  t.H = tau + 1.0 / t.w[0];
  // derived per-face / per-axis transform matrices (row-major, out = A in)
  t.StM.assign(n * n, 0.0);
  t.St.assign(n * n, 0.0);
  t.MS.assign(n * n, 0.0);
  for (int a = 0; a < n; ++a)
    for (int i = 0; i < n; ++i) {
      t.St[a * n + i] = t.S[i * n + a];
      t.StM[a * n + i] = t.S[i * n + a] * t.w[i];
      t.MS[a * n + i] = t.w[a] * t.S[a * n + i];
    }
  return t;
}

}  // namespace hdg
