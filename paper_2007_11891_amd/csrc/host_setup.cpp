// Host-only parts of the C ABI (include/hdg.h): error reporting, solver
// option defaults, the 1D tables of the paper's one-time setup (equations
// (element_matrices), (generalized_eigenvalue_decomposition), (hdgbs)), the
// trace layout and the validation of creation arguments.  No HIP: this unit
// is also built with host sanitizers by the test suite.
#include "host_setup.hpp"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "setup1d.hpp"

namespace hdg {

thread_local std::string g_err;

hdg_status fail(hdg_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

FaceCounts face_counts(const int n[3], int neumann_sides) {
  FaceCounts fc{};
  const int64_t n1 = n[0], n2 = n[1], n3 = n[2];
  const int64_t tb[3] = {n2 * n3, n1 * n3, n1 * n2};
  fc.n_int = (n1 - 1) * n2 * n3 + n1 * (n2 - 1) * n3 + n1 * n2 * (n3 - 1);
  int64_t off = fc.n_int;
  for (int pass = 1; pass >= 0; --pass) {
    for (int k = 0; k < 6; ++k)
      if (((neumann_sides >> k) & 1) == pass) {
        fc.side_off[k] = off;
        off += tb[k >> 1];
      }
    if (pass == 1) fc.n_free_faces = off;
  }
  fc.n_faces = off;
  fc.n_neu = fc.n_free_faces - fc.n_int;
  return fc;
}

hdg_status validate_create(const int n_elem[3], const double* h1, const double* h2,
                           const double* h3, int p, double tau_hat, const double* lambda_host,
                           double lambda_const, int neumann_sides, int exact_mass) {
  if (!n_elem) return fail(HDG_EINVAL, "n_elem is NULL");
  const double* hs[3] = {h1, h2, h3};
  for (int a = 0; a < 3; ++a) {
    if (n_elem[a] < 1 || n_elem[a] > (1 << 20))
      return fail(HDG_EINVAL, "n_elem[%d] = %d out of range", a, n_elem[a]);
    if (!hs[a]) return fail(HDG_EINVAL, "width array %d is NULL", a);
    for (int i = 0; i < n_elem[a]; ++i)
      if (!(hs[a][i] > 0.0) || !std::isfinite(hs[a][i]))
        return fail(HDG_EINVAL, "width h%d[%d] must be finite and > 0", a + 1, i);
  }
  if (p < 1 || p > 16) return fail(HDG_EINVAL, "p must be in [1, 16], got %d", p);
  if (!(tau_hat > 0.0) || !std::isfinite(tau_hat)) return fail(HDG_EINVAL, "tau_hat must be > 0");
  const int64_t ne = (int64_t)n_elem[0] * n_elem[1] * n_elem[2];
  if (ne > (int64_t)1 << 28) return fail(HDG_EINVAL, "more than 2^28 elements");
  if (lambda_host) {
    for (int64_t e = 0; e < ne; ++e)
      if (!(lambda_host[e] >= 0.0) || !std::isfinite(lambda_host[e]))
        return fail(HDG_EINVAL, "lambda[%lld] must be finite and >= 0", (long long)e);
  } else if (!(lambda_const >= 0.0) || !std::isfinite(lambda_const)) {
    return fail(HDG_EINVAL, "lambda_const must be finite and >= 0");
  }
  if (exact_mass != 0 && exact_mass != 1)
    return fail(HDG_EINVAL, "exact_mass must be 0 or 1, got %d", exact_mass);
  if (neumann_sides < 0 || neumann_sides > 63)
    return fail(HDG_EINVAL, "neumann_sides must be a mask of bits 0..5, got %d", neumann_sides);
  if (neumann_sides == 63) {
    bool any = false;
    if (lambda_host) {
      for (int64_t e = 0; e < ne && !any; ++e) any = lambda_host[e] > 0.0;
    } else {
      any = lambda_const > 0.0;
    }
    if (!any)
      return fail(HDG_EINVAL, "every side Neumann with lambda = 0: the condensed operator is "
                              "singular (constants are in its kernel)");
  }
  return HDG_OK;
}

hdg_status validate_batch_create(int count, const int* n_elem3, const int* p,
                                 const double* lambda, double tau_hat) {
  if (count < 1 || count > (1 << 16)) return fail(HDG_EINVAL, "count must be in [1, 65536]");
  if (!n_elem3 || !p || !lambda) return fail(HDG_EINVAL, "NULL argument");
  if (!(tau_hat > 0.0) || !std::isfinite(tau_hat)) return fail(HDG_EINVAL, "tau_hat must be > 0");
  for (int i = 0; i < count; ++i) {
    for (int a = 0; a < 3; ++a)
      if (n_elem3[3 * i + a] < 1 || n_elem3[3 * i + a] > 4096)
        return fail(HDG_EINVAL, "problem %d: n_elem[%d] = %d out of [1, 4096]", i, a,
                    n_elem3[3 * i + a]);
    if (p[i] < 1 || p[i] > 10)
      return fail(HDG_EINVAL, "problem %d: batched degrees must be in [1, 10], got %d", i, p[i]);
    if (!(lambda[i] >= 0.0) || !std::isfinite(lambda[i]))
      return fail(HDG_EINVAL, "problem %d: lambda must be finite and >= 0", i);
  }
  return HDG_OK;
}

}  // namespace hdg

using namespace hdg;

extern "C" {

void hdg_default_opts(hdg_solve_opts* o) {
  if (!o) return;
  o->rtol = 1e-10;
  o->maxit = 20000;
  o->precond = 1;
  o->mixed = 0;
  o->inner_rtol = 1e-2;
  o->max_outer = 12;
  o->check_every = 25;
  o->variant = -1;
  o->guess = 0;
}

const char* hdg_last_error(void) { return g_err.c_str(); }

hdg_status hdg_tables(int p, double tau_hat, double* x, double* w, double* D, double* S,
                      double* Lam, double* BS, double* H) {
  if (p < 1 || p > 16) return fail(HDG_EINVAL, "p must be in [1, 16], got %d", p);
  if (!(tau_hat > 0.0) || !std::isfinite(tau_hat)) return fail(HDG_EINVAL, "tau_hat must be > 0");
  Tables1D t = make_tables(p, tau_hat);
  const int n = t.np;
  if (x) std::memcpy(x, t.x.data(), sizeof(double) * n);
  if (w) std::memcpy(w, t.w.data(), sizeof(double) * n);
  if (D) std::memcpy(D, t.D.data(), sizeof(double) * n * n);
  if (S) std::memcpy(S, t.S.data(), sizeof(double) * n * n);
  if (Lam) std::memcpy(Lam, t.Lam.data(), sizeof(double) * n);
  if (BS) std::memcpy(BS, t.BS.data(), sizeof(double) * n * 2);
  if (H) *H = t.H;
  return HDG_OK;
}

hdg_status hdg_layout(const int n_elem[3], int p, int neumann_sides, int64_t* n_free,
                      int64_t* n_all, int64_t* n_vol) {
  if (!n_elem) return fail(HDG_EINVAL, "n_elem is NULL");
  for (int a = 0; a < 3; ++a)
    if (n_elem[a] < 1 || n_elem[a] > (1 << 20))
      return fail(HDG_EINVAL, "n_elem[%d] = %d out of range", a, n_elem[a]);
  if (p < 1 || p > 16) return fail(HDG_EINVAL, "p must be in [1, 16], got %d", p);
  if (neumann_sides < 0 || neumann_sides > 63)
    return fail(HDG_EINVAL, "neumann_sides must be a mask of bits 0..5, got %d", neumann_sides);
  const FaceCounts fc = face_counts(n_elem, neumann_sides);
  const int64_t npf = (int64_t)(p + 1) * (p + 1);
  if (n_free) *n_free = fc.n_free_faces * npf;
  if (n_all) *n_all = (fc.n_faces + fc.n_neu) * npf;
  if (n_vol) *n_vol = (int64_t)n_elem[0] * n_elem[1] * n_elem[2] * npf * (p + 1);
  return HDG_OK;
}

}  // extern "C"
