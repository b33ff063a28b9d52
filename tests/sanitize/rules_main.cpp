// Host driver for the sanitizer build of the plan rules (gp_rules.cpp): runs
// the parameter choice, the host tables, the step-3 row map and the low-rank
// factorisation over a sweep of problems under AddressSanitizer and UBSan, and
// checks the invariants the device code relies on.  Exit status 0 = clean.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <random>
#include <vector>

#include "../../paper_2407_03608_amd/csrc/gp_rules.h"

using namespace gp;

static int g_fail = 0;
#define CHECK(c, ...)                                  \
  do {                                                 \
    if (!(c)) {                                        \
      std::fprintf(stderr, "FAIL %s: ", #c);           \
      std::fprintf(stderr, __VA_ARGS__);               \
      std::fprintf(stderr, "\n");                      \
      ++g_fail;                                        \
    }                                                  \
  } while (0)

static gp_opts default_opts() {
  gp_opts o;
  gp_opts_init(&o);
  return o;
}

// The plan's geometry as the spread, FFT and interpolation kernels assume it.
static void check_geometry(const PlanRules& P, const char* tag) {
  CHECK(P.w >= 2 && P.w <= 16, "%s w=%d", tag, P.w);
  CHECK(P.nk == P.n_sigma + 1 && P.npair == (P.nk + 1) / 2 && P.nkp % 2 == 0 && P.nkp >= P.nk,
        "%s nk=%d npair=%d nkp=%d", tag, P.nk, P.npair, P.nkp);
  CHECK(P.mcount == 2 * P.M + 1, "%s mcount", tag);
  CHECK(P.dw > 0 && P.dw < 0.5, "%s dw=%g", tag, P.dw);
  int64_t bins = 1;
  for (int r = 0; r < 3; ++r) {
    if (r >= P.d) {
      CHECK(P.nf[r] == 1 && P.na[r] == 1 && P.tile[r] == 1, "%s unused dim %d", tag, r);
      continue;
    }
    const int nf = P.nf[r];
    CHECK(P.fourstep ? (int64_t)P.L1 * P.L2 == nf : fft_length_supported(nf), "%s nf=%d", tag, nf);
    CHECK(nf >= P.mcount, "%s nf=%d < 2M+1=%lld", tag, nf, (long long)P.mcount);
    CHECK(P.tile[r] >= 1 && P.na[r] % P.tile[r] == 0, "%s na=%d tile=%d", tag, P.na[r], P.tile[r]);
    CHECK(P.lo[r] >= 0 && P.lo[r] + P.na[r] <= nf, "%s lo=%d na=%d nf=%d", tag, P.lo[r], P.na[r], nf);
    CHECK(P.nbins[r] * P.tile[r] == P.na[r], "%s nbins", tag);
    // every window of a point in [-1,1] lies in the active box
    const double g_lo = 0.5 * nf - nf * P.dw, g_hi = 0.5 * nf + nf * P.dw;
    const double s_lo = std::ceil(g_lo - 0.5 * P.w), s_hi = std::ceil(g_hi - 0.5 * P.w);
    CHECK(s_lo - P.lo[r] >= 0 && s_hi - P.lo[r] + P.w <= P.na[r], "%s window leaves box", tag);
    bins *= P.nbins[r];
  }
  CHECK(bins == P.n_bins, "%s n_bins", tag);
}

static void check_tables(PlanRules& P, const char* tag) {
  StepTables T;
  host_tables(&P, &T);
  CHECK((int)P.sig_nodes.size() == P.nk && (int)P.bary.size() == P.nk, "%s node tables", tag);
  for (int k = 0; k < P.nk; ++k)
    CHECK(P.sig_nodes[k] >= P.s_min * (1 - 1e-12) && P.sig_nodes[k] <= P.s_max * (1 + 1e-12),
          "%s node %d", tag, k);
  for (double v : T.tvt) CHECK(std::isfinite(v) && v >= 0, "%s tvt", tag);
  for (double v : T.g0) CHECK(std::isfinite(v) && v >= 0, "%s g0", tag);
  for (double v : T.dec) CHECK(std::isfinite(v) && v > 0, "%s dec", tag);
  const int64_t M1 = P.M + 1;
  CHECK((int64_t)T.g0.size() == (int64_t)P.nt_eff * P.nk * M1, "%s g0 size", tag);
  // low-rank factors of a few step-3 rows reproduce the rows
  std::vector<double> sv;
  std::vector<int> rowmap;
  const double boxes = std::pow((double)M1, (double)P.d);
  if (boxes <= 3e6) {
    step3_rows(P, sv, rowmap);
    CHECK(!sv.empty() && sv[0] == 0.0, "%s svals", tag);
    for (size_t i = 1; i < sv.size(); ++i) CHECK(sv[i] > sv[i - 1], "%s svals order", tag);
    if (P.d >= 2) {
      CHECK((int64_t)rowmap.size() == (int64_t)P.d * P.M * P.M + 1, "%s rowmap size", tag);
      for (size_t v = 0; v < rowmap.size(); ++v)
        if (rowmap[v] >= 0) CHECK(sv[rowmap[v]] == (double)v, "%s rowmap %zu", tag, v);
    }
  } else {
    for (int64_t m = 0; m <= P.M; m += std::max<int64_t>(1, P.M / 7)) sv.push_back((double)(m * m));
  }
  const int64_t rows = std::min<int64_t>((int64_t)sv.size(), 40);
  const int npk = P.nkp * (P.nkp + 1) / 2;
  std::vector<double> A((size_t)rows * npk, 0.0);
  for (int64_t r = 0; r < rows; ++r) {
    const double s2 = sv[(size_t)(r * (int64_t)sv.size() / rows)];
    for (int k1 = 0, p = 0; k1 < P.nkp; ++k1)
      for (int k2 = k1; k2 < P.nkp; ++k2, ++p) {
        double sum = 0;
        if (k1 < P.nk && k2 < P.nk)
          for (int j = 0; j < P.nt_eff; ++j)
            sum += T.tvt[j] * T.tcst[(size_t)j * P.nk + k1] * T.tcst[(size_t)j * P.nk + k2] *
                   std::exp(-(T.ttau[(size_t)j * P.nk + k1] + T.ttau[(size_t)j * P.nk + k2]) * s2);
        A[(size_t)r * npk + p] = sum;
      }
  }
  std::vector<int64_t> off;
  std::vector<double> fac;
  int rmax = 0;
  double rmean = 0;
  lowrank_rows(rows, P.nk, P.nkp, A, 1e-2 * P.tol, off, fac, &rmax, &rmean);
  CHECK((int64_t)off.size() == rows + 1 && off[rows] == (int64_t)fac.size(), "%s lr offsets", tag);
  CHECK(rmax <= P.nk && rmean <= rmax, "%s lr rank", tag);
  for (int64_t r = 0; r < rows; ++r) {
    const int rk = (int)((off[r + 1] - off[r]) / P.nkp);
    double dmax = 0, err = 0;
    for (int k1 = 0, p = 0; k1 < P.nkp; ++k1)
      for (int k2 = k1; k2 < P.nkp; ++k2, ++p) {
        double s = 0;
        for (int a = 0; a < rk; ++a)
          s += fac[off[r] + (size_t)a * P.nkp + k1] * fac[off[r] + (size_t)a * P.nkp + k2];
        err = std::max(err, std::fabs(s - A[(size_t)r * npk + p]));
        if (k1 == k2) dmax = std::max(dmax, A[(size_t)r * npk + p]);
      }
    // pivoted Cholesky stops when every remaining diagonal is <= rel * dmax;
    // the remainder is PSD, so its entries are bounded by that diagonal
    CHECK(err <= 1e-2 * P.tol * dmax * 1.0001 + 1e-300, "%s lr row %lld err %g dmax %g", tag,
          (long long)r, err, dmax);
  }
}

int main() {
  const double inf = std::numeric_limits<double>::infinity();
  const double nus[] = {0.5, 1.5, 2.5, inf};
  const double tols[] = {1e-4, 1e-6, 1e-8};
  const double lranges[][2] = {{0.02, 0.04}, {0.05, 0.5}, {0.1, 0.1}};
  int cases = 0;
  for (int d = 1; d <= 3; ++d)
    for (double nu : nus)
      for (double tol : tols)
        for (auto& lr : lranges)
          for (int prec = 0; prec < 2; ++prec)
            for (double ups : {0.0, 1.25, 2.0}) {
              gp_opts o = default_opts();
              o.precision = prec ? GP_FP32_BULK : GP_FP64;
              o.upsample = ups;
              if (d == 3 && tol < 1e-6) o.M_cap = 160;  // bounded host tables
              PlanRules P;
              P.d = d;
              P.nu = nu;
              P.se = std::isinf(nu);
              P.precision = o.precision;
              P.scale = 2.0;  // extent 1
              char tag[160];
              std::snprintf(tag, sizeof tag, "d=%d nu=%g tol=%g l=[%g,%g] prec=%d ups=%g", d, nu,
                            tol, lr[0], lr[1], prec, ups);
              try {
                choose_params(&P, d, nu, tol, lr[0], lr[1], o);
              } catch (const Error& e) {
                // a grid beyond the compiled FFT lengths is a documented refusal
                CHECK(e.code == GP_EUNSUPPORTED, "%s threw %d %s", tag, e.code, e.msg.c_str());
                continue;
              }
              check_geometry(P, tag);
              // host tables for the cases whose tables stay small (the
              // d=2 N=1e6 workload's plan is run once more below)
              if (ups == 0.0 && prec == 0 && (double)P.nt_eff * P.nk * (P.M + 1) <= 4e5)
                check_tables(P, tag);
              ++cases;
            }
  // the d=2 N=1e6 workload's plan: nu = 1/2, tol 1e-8, l in [0.02, 0.04]
  {
    gp_opts o = default_opts();
    PlanRules P;
    P.d = 2;
    P.nu = 0.5;
    P.scale = 2.0;
    choose_params(&P, 2, 0.5, 1e-8, 0.02, 0.04, o);
    CHECK(P.M == 2047 && P.nf[0] == 6144, "d=2 workload M=%lld nf=%d", (long long)P.M, P.nf[0]);
    check_geometry(P, "d=2 workload");
    check_tables(P, "d=2 workload");
    ++cases;
  }
  // explicit overrides: N_sigma, N_t and the t range, dw, M; keep_t
  {
    gp_opts o = default_opts();
    o.n_sigma = 5;
    o.n_t = 12;
    o.t_min = -4;
    o.t_max = 3;
    o.dw = 0.1;
    o.M = 40;
    o.keep_t = 1;
    PlanRules P;
    P.d = 2;
    P.nu = 1.5;
    P.scale = 2.0;
    choose_params(&P, 2, 1.5, 1e-6, 0.05, 0.2, o);
    CHECK(P.n_sigma == 5 && P.n_t == 12 && P.M == 40 && P.dw == 0.1 && P.n_flat == 0, "overrides");
    check_geometry(P, "overrides");
    check_tables(P, "overrides");
    ++cases;
  }
  // input validation: good inputs, then each kind of bad input throws
  {
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    const int n = 257, d = 2;
    std::vector<double> x(n * d), s(n, 1.0), l(n, 0.1);
    for (auto& v : x) v = U(rng);
    gp_opts o = default_opts();
    InputRanges R;
    input_ranges(d, n, x.data(), s.data(), l.data(), o, &R);
    PlanRules P;
    P.d = d;
    map_box(&P, R);
    for (int i = 0; i < n; ++i)
      for (int r = 0; r < d; ++r) {
        const double xp = (x[i * d + r] - P.center[r]) * P.scale;
        CHECK(xp >= -1 - 1e-12 && xp <= 1 + 1e-12, "map_box");
      }
    auto expect_throw = [&](int code, const char* what) {
      try {
        input_ranges(d, n, x.data(), s.data(), l.data(), o, &R);
        CHECK(false, "%s did not throw", what);
      } catch (const Error& e) {
        CHECK(e.code == code, "%s code %d", what, e.code);
      }
    };
    x[17] = std::numeric_limits<double>::quiet_NaN();
    expect_throw(GP_EDOMAIN, "NaN coordinate");
    x[17] = 0.5;
    l[3] = 0.0;
    expect_throw(GP_EDOMAIN, "l = 0");
    l[3] = 0.1;
    s[9] = -1.0;
    expect_throw(GP_EDOMAIN, "sigma < 0");
    s[9] = 1.0;
    o.use_box = 1;
    o.box_lo[0] = o.box_lo[1] = 0.2;
    o.box_hi[0] = o.box_hi[1] = 1.0;
    expect_throw(GP_ERANGE, "box");
  }
  // twiddles: unit modulus, exact quarter turns
  for (int L : {8, 24, 6144, 8192}) {
    std::vector<double> t;
    twiddle_table(L, t);
    for (int k = 0; k < L; ++k)
      CHECK(std::fabs(std::hypot(t[2 * k], t[2 * k + 1]) - 1) < 1e-15, "twiddle %d %d", L, k);
    CHECK(std::fabs(t[2 * (L / 4) + 1] + 1) < 1e-15, "twiddle quarter %d", L);
  }
  std::printf("rules: %d plan cases, %d failures\n", cases, g_fail);
  return g_fail ? 1 : 0;
}
