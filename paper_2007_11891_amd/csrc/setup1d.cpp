// One-time 1D setup on the host, FP64 (paper: equation (element_matrices),
// equation (generalized_eigenvalue_decomposition), equation (hdgbs)).
//
// GLL points by Newton iteration on P_p', weights 2 / (p (p+1) P_p(x)^2);
// Lagrange differentiation by barycentric weights.  The mass matrix is the
// lumped GLL one, diag(w), or the exact one, M_ij = int phi_i phi_j by
// Gauss-Legendre quadrature with p + 2 points (exact to degree 2p + 3).  The
// generalized symmetric eigenproblem L s = Lambda M s is reduced to the
// ordinary one R^-1 L R^-T v = Lambda v with M = R R^T (R = diag(sqrt(w))
// for the lumped mass, the Cholesky factor otherwise) and solved by the
// cyclic Jacobi rotation method; S = R^-T V.
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

// Gauss-Legendre points (roots of P_n by Newton from Chebyshev guesses) and
// weights 2 / ((1 - x^2) P_n'(x)^2).
static void gauss(int n, std::vector<long double>& x, std::vector<long double>& w) {
  x.assign(n, 0.0L);
  w.assign(n, 0.0L);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    long double xi = -std::cos(pi * (i + 0.75L) / (n + 0.5L));
    long double P = 0.0L, dP = 1.0L;
    for (int it = 0; it < 100; ++it) {
      legendre(n, xi, &P, &dP);
      const long double dx = P / dP;
      xi -= dx;
      if (std::fabs(dx) < 1e-19L) break;
    }
    legendre(n, xi, &P, &dP);
    x[i] = xi;
    w[i] = 2.0L / ((1.0L - xi * xi) * dP * dP);
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

Tables1D make_tables(int p, double tau, bool exact_mass) {
  Tables1D t;
  t.p = p;
  t.np = p + 1;
  t.tau = tau;
  t.exact_mass = exact_mass;
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
  // mass matrix, its inverse and the factor R (M = R R^T, lower triangular)
  std::vector<long double> Mi(n * n, 0.0L), Rf(n * n, 0.0L);
  t.M.assign(n * n, 0.0);
  if (!exact_mass) {
    for (int i = 0; i < n; ++i) {
      t.M[i * n + i] = t.w[i];
      Mi[i * n + i] = 1.0L / t.w[i];
      Rf[i * n + i] = std::sqrt((long double)t.w[i]);
    }
  } else {
    std::vector<long double> gx, gw;
    gauss(p + 2, gx, gw);
    std::vector<long double> Ml(n * n, 0.0L);
    for (int g = 0; g < p + 2; ++g) {
      // phi_j(gx) by the barycentric formula (no Gauss point is a GLL point)
      std::vector<long double> phi(n);
      long double den = 0.0L;
      for (int j = 0; j < n; ++j) {
        phi[j] = bw[j] / (gx[g] - (long double)t.x[j]);
        den += phi[j];
      }
      for (int j = 0; j < n; ++j) phi[j] /= den;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ml[i * n + j] += gw[g] * phi[i] * phi[j];
    }
    for (int i = 0; i < n * n; ++i) t.M[i] = (double)Ml[i];
    // Cholesky M = R R^T
    for (int j = 0; j < n; ++j) {
      long double d = Ml[j * n + j];
      for (int k = 0; k < j; ++k) d -= Rf[j * n + k] * Rf[j * n + k];
      Rf[j * n + j] = std::sqrt(d);
      for (int i = j + 1; i < n; ++i) {
        long double v = Ml[i * n + j];
        for (int k = 0; k < j; ++k) v -= Rf[i * n + k] * Rf[j * n + k];
        Rf[i * n + j] = v / Rf[j * n + j];
      }
    }
    // M^-1 = R^-T R^-1 from the columns of R^-1 (forward substitution)
    std::vector<long double> Ri(n * n, 0.0L);
    for (int c = 0; c < n; ++c)
      for (int i = c; i < n; ++i) {
        long double v = (i == c) ? 1.0L : 0.0L;
        for (int k = c; k < i; ++k) v -= Rf[i * n + k] * Ri[k * n + c];
        Ri[i * n + c] = v / Rf[i * n + i];
      }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        long double s = 0.0L;
        for (int k = 0; k < n; ++k) s += Ri[k * n + i] * Ri[k * n + j];
        Mi[i * n + j] = s;
      }
  }
  // L = E + D M^-1 D^T, E = tau (e0 e0^T + ep ep^T)
  std::vector<double> L(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      long double s = 0.0L;
      for (int k = 0; k < n; ++k)
        for (int l = 0; l < n; ++l)
          if (Mi[k * n + l] != 0.0L) s += (long double)t.D[i * n + k] * Mi[k * n + l] * t.D[j * n + l];
      L[i * n + j] = (double)s;
    }
  L[0] += tau;
  L[n * n - 1] += tau;
  // A = R^-1 L R^-T (R lower triangular): solve R Y = L, then R A^T = Y^T
  std::vector<long double> Y(n * n, 0.0L);
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      long double v = L[i * n + c];
      for (int k = 0; k < i; ++k) v -= Rf[i * n + k] * Y[k * n + c];
      Y[i * n + c] = v / Rf[i * n + i];
    }
  std::vector<double> A(n * n);
  {
    std::vector<long double> Z(n * n, 0.0L);   // Z = R^-1 Y^T = (Y R^-T)^T = A^T = A
    for (int c = 0; c < n; ++c)
      for (int i = 0; i < n; ++i) {
        long double v = Y[c * n + i];
        for (int k = 0; k < i; ++k) v -= Rf[i * n + k] * Z[k * n + c];
        Z[i * n + c] = v / Rf[i * n + i];
      }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) A[i * n + j] = (double)(0.5L * (Z[i * n + j] + Z[j * n + i]));
  }
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
    // S column = R^-T v by back substitution
    std::vector<long double> col(n, 0.0L);
    for (int i = n - 1; i >= 0; --i) {
      long double v = V[i * n + src];
      for (int k = i + 1; k < n; ++k) v -= Rf[k * n + i] * col[k];
      col[i] = v / Rf[i * n + i];
    }
    // sign: first entry of clearly nonzero magnitude is positive
    double sgn = 1.0;
    for (int i = 0; i < n; ++i)
      if (std::fabs((double)col[i]) > 1e-8) { sgn = col[i] > 0 ? 1.0 : -1.0; break; }
    for (int i = 0; i < n; ++i) t.S[i * n + c] = sgn * (double)col[i];
  }
  // B_S = S^T B - S^T D M^-1 C with B = -tau [e0, ep], C = [-e0, ep]:
  // (M^-1 C)_{:,0} = -M^-1 e0, (M^-1 C)_{:,1} = M^-1 ep
  t.BS.assign(n * 2, 0.0);
  std::vector<long double> DMc0(n, 0.0L), DMc1(n, 0.0L);   // (D M^-1 C) columns
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      DMc0[i] -= (long double)t.D[i * n + k] * Mi[k * n + 0];
      DMc1[i] += (long double)t.D[i * n + k] * Mi[k * n + (n - 1)];
    }
  for (int k = 0; k < n; ++k) {
    long double s0 = -(long double)tau * t.S[0 * n + k];
    long double s1 = -(long double)tau * t.S[(n - 1) * n + k];
    for (int i = 0; i < n; ++i) {
      s0 -= (long double)t.S[i * n + k] * DMc0[i];
      s1 -= (long double)t.S[i * n + k] * DMc1[i];
    }
    t.BS[k * 2 + 0] = (double)s0;
    t.BS[k * 2 + 1] = (double)s1;
  }
  // H = G + C^T M^-1 C: (tau + 1/w_0) I_2 for the lumped mass
  t.H = (double)((long double)tau + Mi[0]);
  t.H11 = (double)((long double)tau + Mi[n * n - 1]);
  t.H01 = (double)(-Mi[n - 1]);
  // derived per-face / per-axis transform matrices (row-major, out = A in)
  t.StM.assign(n * n, 0.0);
  t.St.assign(n * n, 0.0);
  t.MS.assign(n * n, 0.0);
  for (int a = 0; a < n; ++a)
    for (int i = 0; i < n; ++i) {
      t.St[a * n + i] = t.S[i * n + a];
      long double sm = 0.0L, ms = 0.0L;
      for (int k = 0; k < n; ++k) {
        sm += (long double)t.S[k * n + a] * t.M[k * n + i];   // (S^T M)_ai
        ms += (long double)t.M[a * n + k] * t.S[k * n + i];   // (M S)_ai
      }
      t.StM[a * n + i] = (double)sm;
      t.MS[a * n + i] = (double)ms;
    }
  return t;
}

}  // namespace hdg
