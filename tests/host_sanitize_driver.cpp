// Host-only checks of the library's setup, layout and argument validation,
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// test_host_sanitizers.py (no GPU, no HIP).  Prints "host checks OK" and
// returns 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "hdg.h"
#include "host_setup.hpp"
#include "setup1d.hpp"

static int g_failures = 0;
#define CHECK(cond, ...)                                  \
  do {                                                    \
    if (!(cond)) {                                        \
      ++g_failures;                                       \
      std::printf("FAILED %s:%d: ", __FILE__, __LINE__);  \
      std::printf(__VA_ARGS__);                           \
      std::printf("\n");                                  \
    }                                                     \
  } while (0)

static const double kNaN = std::numeric_limits<double>::quiet_NaN();
static const double kInf = std::numeric_limits<double>::infinity();

static void expect_einval(hdg_status st, const char* what) {
  CHECK(st == HDG_EINVAL, "%s: status %d", what, (int)st);
  CHECK(std::strlen(hdg_last_error()) > 0, "%s: no message", what);
}

// ||S^T M S - I||_max for row-major S (columns = eigenvectors) and M
static double orth_defect(int n, const std::vector<double>& S, const std::vector<double>& M) {
  double worst = 0.0;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      double acc = 0.0;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) acc += S[i * n + a] * M[i * n + j] * S[j * n + b];
      worst = std::fmax(worst, std::fabs(acc - (a == b ? 1.0 : 0.0)));
    }
  return worst;
}

static void check_tables() {
  hdg_default_opts(nullptr);
  hdg_solve_opts o;
  hdg_default_opts(&o);
  CHECK(o.rtol > 0.0 && o.maxit > 0, "default options");
  for (int p = 1; p <= 16; ++p)
    for (double tau : {0.05, 1.0, 20.0}) {
      const int n = p + 1;
      std::vector<double> x(n), w(n), D(n * n), S(n * n), Lam(n), BS(2 * n);
      double H = 0.0;
      CHECK(hdg_tables(p, tau, x.data(), w.data(), D.data(), S.data(), Lam.data(), BS.data(),
                       &H) == HDG_OK, "tables p=%d", p);
      double ws = 0.0;
      for (int i = 0; i < n; ++i) ws += w[i];
      CHECK(std::fabs(ws - 2.0) < 1e-13, "GLL weights sum p=%d: %.17g", p, ws);
      CHECK(x[0] == -1.0 && x[n - 1] == 1.0, "GLL end points p=%d", p);
      for (int i = 1; i < n; ++i) CHECK(x[i] > x[i - 1], "GLL points ascending p=%d", p);
      for (int i = 1; i < n; ++i) CHECK(Lam[i] >= Lam[i - 1], "eigenvalues ascending p=%d", p);
      CHECK(Lam[0] > -1e-12, "eigenvalues nonnegative p=%d", p);
      std::vector<double> M(n * n, 0.0);
      for (int i = 0; i < n; ++i) M[i * n + i] = w[i];
      CHECK(orth_defect(n, S, M) < 1e-11, "S^T M S = I (lumped) p=%d", p);
      CHECK(std::isfinite(H) && H > 0.0, "H p=%d", p);
      // NULL outputs are skipped
      CHECK(hdg_tables(p, tau, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
            HDG_OK, "tables with NULL outputs p=%d", p);
    }
  for (int p = 1; p <= 16; ++p) {
    const hdg::Tables1D t = hdg::make_tables(p, 1.0, true);
    CHECK(orth_defect(t.np, t.S, t.M) < 1e-10, "S^T M S = I (exact mass) p=%d", p);
  }
  for (int p : {0, -3, 17, 1000}) expect_einval(hdg_tables(p, 1.0, 0, 0, 0, 0, 0, 0, 0), "tables p");
  for (double tau : {0.0, -1.0, kNaN, kInf})
    expect_einval(hdg_tables(3, tau, 0, 0, 0, 0, 0, 0, 0), "tables tau");
}

static void check_layout() {
  for (int n1 = 1; n1 <= 4; ++n1)
    for (int n2 = 1; n2 <= 4; ++n2)
      for (int n3 = 1; n3 <= 4; ++n3)
        for (int p : {1, 2, 7, 16})
          for (int mask = 0; mask < 64; ++mask) {
            const int n[3] = {n1, n2, n3};
            int64_t nf = -1, na = -1, nv = -1;
            CHECK(hdg_layout(n, p, mask, &nf, &na, &nv) == HDG_OK, "layout");
            const int64_t npf = (int64_t)(p + 1) * (p + 1);
            const int64_t inter = (int64_t)(n1 - 1) * n2 * n3 + (int64_t)n1 * (n2 - 1) * n3 +
                                  (int64_t)n1 * n2 * (n3 - 1);
            const int64_t side[6] = {(int64_t)n2 * n3, (int64_t)n2 * n3, (int64_t)n1 * n3,
                                     (int64_t)n1 * n3, (int64_t)n1 * n2, (int64_t)n1 * n2};
            int64_t neu = 0, all = inter;
            for (int k = 0; k < 6; ++k) {
              all += side[k];
              if ((mask >> k) & 1) neu += side[k];
            }
            CHECK(nf == (inter + neu) * npf, "n_free n=%d,%d,%d mask=%d", n1, n2, n3, mask);
            CHECK(na == (all + neu) * npf, "n_all n=%d,%d,%d mask=%d", n1, n2, n3, mask);
            CHECK(nv == (int64_t)n1 * n2 * n3 * npf * (p + 1), "n_vol");
            const hdg::FaceCounts fc = hdg::face_counts(n, mask);
            for (int k = 0; k < 6; ++k)
              CHECK(fc.side_off[k] >= fc.n_int && fc.side_off[k] + side[k] <= fc.n_faces,
                    "side offsets inside the face range");
          }
  const int ok[3] = {2, 2, 2};
  int64_t v = 0;
  CHECK(hdg_layout(ok, 3, 0, nullptr, nullptr, nullptr) == HDG_OK, "layout NULL outputs");
  expect_einval(hdg_layout(nullptr, 3, 0, &v, &v, &v), "layout NULL n");
  const int bad_n[][3] = {{0, 2, 2}, {2, -1, 2}, {2, 2, (1 << 20) + 1}};
  for (const auto& b : bad_n) expect_einval(hdg_layout(b, 3, 0, &v, &v, &v), "layout n");
  for (int p : {0, 17}) expect_einval(hdg_layout(ok, p, 0, &v, &v, &v), "layout p");
  for (int m : {-1, 64}) expect_einval(hdg_layout(ok, 3, m, &v, &v, &v), "layout mask");
}

static void check_create_validation() {
  const int n[3] = {3, 2, 4};
  std::vector<double> h1(3, 1.0 / 3), h2(2, 0.5), h3(4, 0.25), lam(24, 1.0);
  using hdg::validate_create;
  CHECK(validate_create(n, h1.data(), h2.data(), h3.data(), 4, 1.0, lam.data(), 0.0, 0, 0) ==
        HDG_OK, "valid create");
  CHECK(validate_create(n, h1.data(), h2.data(), h3.data(), 4, 1.0, nullptr, 2.0, 63, 1) == HDG_OK,
        "valid create, all Neumann, lambda > 0");
  expect_einval(validate_create(nullptr, h1.data(), h2.data(), h3.data(), 4, 1, 0, 1, 0, 0), "n NULL");
  expect_einval(validate_create(n, nullptr, h2.data(), h3.data(), 4, 1, 0, 1, 0, 0), "h1 NULL");
  for (double bad : {0.0, -0.1, kNaN, kInf}) {
    std::vector<double> hb = h2;
    hb[1] = bad;
    expect_einval(validate_create(n, h1.data(), hb.data(), h3.data(), 4, 1, 0, 1, 0, 0), "width");
  }
  for (int p : {0, 17}) expect_einval(validate_create(n, h1.data(), h2.data(), h3.data(), p, 1, 0, 1, 0, 0), "p");
  for (double tau : {0.0, kNaN, kInf})
    expect_einval(validate_create(n, h1.data(), h2.data(), h3.data(), 4, tau, 0, 1, 0, 0), "tau");
  for (double bad : {-1.0, kNaN, kInf}) {
    std::vector<double> lb = lam;
    lb[23] = bad;
    expect_einval(validate_create(n, h1.data(), h2.data(), h3.data(), 4, 1, lb.data(), 0, 0, 0), "lambda");
    expect_einval(validate_create(n, h1.data(), h2.data(), h3.data(), 4, 1, nullptr, bad, 0, 0), "lambda const");
  }
  expect_einval(validate_create(n, h1.data(), h2.data(), h3.data(), 4, 1, 0, 1, 0, 2), "exact_mass");
  for (int m : {-1, 64}) expect_einval(validate_create(n, h1.data(), h2.data(), h3.data(), 4, 1, 0, 1, m, 0), "mask");
  std::vector<double> zero(24, 0.0);
  expect_einval(validate_create(n, h1.data(), h2.data(), h3.data(), 4, 1, zero.data(), 0, 63, 0), "singular");
  expect_einval(validate_create(n, h1.data(), h2.data(), h3.data(), 4, 1, nullptr, 0.0, 63, 0), "singular const");
  const int big[3] = {1024, 1024, 1024};
  std::vector<double> hb(1024, 1.0 / 1024);
  expect_einval(validate_create(big, hb.data(), hb.data(), hb.data(), 2, 1, nullptr, 1, 0, 0), "too many elements");
}

static void check_batch_validation() {
  using hdg::validate_batch_create;
  const int n3[6] = {4, 5, 6, 12, 4, 7};
  const int p[2] = {2, 10};
  const double lam[2] = {0.01, 100.0};
  CHECK(validate_batch_create(2, n3, p, lam, 1.0) == HDG_OK, "valid batch");
  for (int c : {0, -1, (1 << 16) + 1}) expect_einval(validate_batch_create(c, n3, p, lam, 1.0), "count");
  expect_einval(validate_batch_create(2, nullptr, p, lam, 1.0), "n NULL");
  expect_einval(validate_batch_create(2, n3, nullptr, lam, 1.0), "p NULL");
  expect_einval(validate_batch_create(2, n3, p, nullptr, 1.0), "lambda NULL");
  for (double tau : {0.0, kNaN}) expect_einval(validate_batch_create(2, n3, p, lam, tau), "tau");
  const int nbad[6] = {4, 5, 6, 12, 4097, 7};
  expect_einval(validate_batch_create(2, nbad, p, lam, 1.0), "batch n");
  for (int q : {0, 11}) {
    const int pb[2] = {2, q};
    expect_einval(validate_batch_create(2, n3, pb, lam, 1.0), "batch p");
  }
  const double lbad[2] = {1.0, kNaN};
  expect_einval(validate_batch_create(2, n3, p, lbad, 1.0), "batch lambda");
}

static void check_messages() {
  // a message longer than the buffer is cut, not overrun
  const std::string longs(2000, 'x');
  CHECK(hdg::fail(HDG_EINVAL, "%s", longs.c_str()) == HDG_EINVAL, "fail status");
  CHECK(std::strlen(hdg_last_error()) < 512, "message bounded");
}

int main() {
  check_tables();
  check_layout();
  check_create_validation();
  check_batch_validation();
  check_messages();
  if (g_failures) {
    std::printf("%d host checks failed\n", g_failures);
    return 1;
  }
  std::printf("host checks OK\n");
  return 0;
}
