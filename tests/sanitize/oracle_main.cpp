// Host driver for the sanitizer build of the oracle: compiles oracle.cpp into
// this translation unit and runs each of its functions on small inputs under
// AddressSanitizer and UBSan, with cross-checks between its two independent
// forms of K~ (the five-step matvec and the entry formula) and between the
// Cholesky solve and the exact matvec.  Exit status 0 = clean.
#include <cstdio>
#include <random>

#include "../../oracle/oracle.cpp"

static int g_fail = 0;
#define CHECK(c, ...)                        \
  do {                                       \
    if (!(c)) {                              \
      std::fprintf(stderr, "FAIL %s: ", #c); \
      std::fprintf(stderr, __VA_ARGS__);     \
      std::fprintf(stderr, "\n");            \
      ++g_fail;                              \
    }                                        \
  } while (0)

static double rel(const std::vector<double>& a, const std::vector<double>& b) {
  double num = 0, den = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    num += (a[i] - b[i]) * (a[i] - b[i]);
    den += b[i] * b[i];
  }
  return std::sqrt(num / den);
}

int main() {
  std::mt19937_64 rng(11);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  std::normal_distribution<double> N(0.0, 1.0);
  // Matern in its two forms
  for (double nu : {0.5, 1.5, 2.5})
    for (double r : {0.0, 0.1, 1.0, 3.0}) {
      const double a = orc_matern(nu, r), b = orc_matern_bessel(nu, r);
      CHECK(std::isfinite(a) && std::fabs(a - b) <= 1e-12, "matern nu=%g r=%g", nu, r);
      const double c = orc_matern_schoenberg(nu, r, -40.0, 5.0, 4000);
      CHECK(std::fabs(c - a) <= 1e-6, "schoenberg nu=%g r=%g %g %g", nu, r, c, a);
    }
  for (int d = 1; d <= 3; ++d)
    for (double nu : {0.5, 1.5, std::numeric_limits<double>::infinity()}) {
      const int n = d == 3 ? 18 : 24;
      std::vector<double> x(n * d), s(n), l(n), a(n);
      for (auto& v : x) v = U(rng);
      for (int i = 0; i < n; ++i) {
        s[i] = std::exp(0.2 * N(rng));
        l[i] = 0.2 + 0.2 * U(rng);
        a[i] = N(rng);
      }
      orc_plan p;
      p.d = d;
      p.nu = nu;
      p.t_min = -6;
      p.t_max = 4;
      p.n_t = std::isinf(nu) ? 0 : 10;
      p.s_min = 0.2 * 2 / std::sqrt(2.0);
      p.s_max = 0.4 * 2 / std::sqrt(2.0);
      p.n_sigma = 3;
      p.dw = 0.3;
      p.M = d == 3 ? 5 : 9;
      for (int r = 0; r < 3; ++r) p.center[r] = r < d ? 0.5 : 0.0;
      p.scale = 2.0;
      // t grid, nodes, weights
      std::vector<double> t(p.n_t + 1), vt(p.n_t + 1), chi(p.n_t + 1);
      orc_tgrid(&p, t.data(), vt.data(), chi.data());
      for (double v : vt) CHECK(std::isfinite(v) && v >= 0, "tgrid d=%d", d);
      std::vector<double> sk(p.n_sigma + 1), P(p.n_sigma + 1), wk((size_t)n * (p.n_sigma + 1));
      orc_sigma_nodes(&p, sk.data());
      orc_lagrange(p.n_sigma, sk.data(), 0.5 * (p.s_min + p.s_max), P.data());
      double psum = 0;
      for (double v : P) psum += v;
      CHECK(std::fabs(psum - 1) < 1e-13, "lagrange sum %g", psum);
      orc_weights(&p, n, s.data(), l.data(), wk.data());
      // K~ two ways
      std::vector<double> y1(n), K((size_t)n * n), y2(n, 0.0);
      CHECK(orc_ktilde_matvec(&p, n, x.data(), s.data(), l.data(), a.data(), y1.data()) == 0, "matvec");
      CHECK(orc_ktilde_entries(&p, n, x.data(), s.data(), l.data(), n, x.data(), s.data(), l.data(),
                               K.data()) == 0, "entries");
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) y2[i] += K[(size_t)i * n + j] * a[j];
      CHECK(rel(y1, y2) < 1e-11, "K~ two forms d=%d nu=%g: %g", d, nu, rel(y1, y2));
      std::vector<double> mu(5), mu2(5);
      CHECK(orc_ktilde_posterior(&p, n, x.data(), s.data(), l.data(), a.data(), 5, x.data(),
                                 s.data(), l.data(), mu.data()) == 0, "posterior");
      for (int i = 0; i < 5; ++i) CHECK(std::fabs(mu[i] - y1[i]) <= 1e-10 * (1 + std::fabs(y1[i])), "post %d", i);
      // exact kernel: block, rows, Cholesky solve
      std::vector<double> Kx((size_t)n * n), rows(n);
      orc_kernel_block(d, n, x.data(), s.data(), l.data(), n, x.data(), s.data(), l.data(), nu, Kx.data());
      orc_exact_matvec_rows(d, n, x.data(), s.data(), l.data(), nu, a.data(), 0, n, rows.data());
      std::vector<double> A = Kx, sol(n), back(n, 0.0);
      for (int i = 0; i < n; ++i) A[(size_t)i * n + i] += 0.25;
      CHECK(orc_cholesky(n, A.data()) == 0, "cholesky");
      orc_chol_solve(n, A.data(), rows.data(), sol.data());
      for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) back[i] += Kx[(size_t)i * n + j] * sol[j];
        back[i] += 0.25 * sol[i];
      }
      CHECK(rel(back, rows) < 1e-10, "chol solve d=%d: %g", d, rel(back, rows));
      orc_posterior_mean(d, n, x.data(), s.data(), l.data(), nu, a.data(), 5, x.data(), s.data(),
                         l.data(), mu2.data());
      for (int i = 0; i < 5; ++i) CHECK(std::fabs(mu2[i] - rows[i]) <= 1e-12 * (1 + std::fabs(rows[i])), "mean %d", i);
    }
  std::printf("oracle: %d failures\n", g_fail);
  return g_fail ? 1 : 0;
}
