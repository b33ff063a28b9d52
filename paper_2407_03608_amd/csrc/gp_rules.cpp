// Host-side rules of a plan (plain C++): parameter choice (section 3.5), the
// host tables of the operator and the low-rank factors of the step-3 rows.
#include "gp_rules.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

namespace gp {

static const double PI = 3.14159265358979323846264338327950288;

bool fft_length_supported(int L) {
  switch (L) {
    case 8: case 16: case 32: case 64: case 128: case 256: case 512: case 1024: case 2048:
    case 4096: case 8192: case 24: case 48: case 96: case 192: case 384: case 768: case 1536:
    case 3072: case 6144:
      return true;
    default:
      return false;
  }
}

namespace {

// ------------------------------------------------------------ host maths ----

// Matern phi_nu(r) through its Gaussian-mixture representation eq:schoenberg2
// with u, chi of eq:maternpres (fine trapezoid on a wide t range); used only to
// size the aliasing margin, so a few digits suffice.  SE: exp(-r^2/2).
double phi_of_r(double nu, double r) {
  if (std::isinf(nu)) return std::exp(-0.5 * r * r);
  const double tmin = -60.0 / nu - 20.0, tmax = 6.0;
  const int nt = 6000;
  const double dt = (tmax - tmin) / nt, lg = std::lgamma(nu);
  double s = 0;
  for (int j = 0; j <= nt; ++j) {
    double t = tmin + j * dt;
    double f = std::exp(nu * t - std::exp(t) - lg - r * r * nu / (2.0 * std::exp(t)));
    s += (j == 0 || j == nt) ? 0.5 * f : f;
  }
  return s * dt;
}

// Max over the sample radii of |trapezoid sum of eq:trapsum - phi_nu(r)|, the
// sum over t_j = t_min + j (t_max - t_min)/n_t of u(t_j) exp(-r^2 nu/(2 e^t_j))
// with halved end weights (eq:maternpres, eq:schoenberg2 at chi^2 = e^t/nu).
double trap_error(double nu, double tmin, double tmax, int nt, const std::vector<double>& rs,
                  const std::vector<double>& ref) {
  const double h = (tmax - tmin) / nt, lg = std::lgamma(nu);
  double worst = 0;
  for (size_t i = 0; i < rs.size(); ++i) {
    double s = 0;
    for (int j = 0; j <= nt; ++j) {
      const double t = tmin + j * h;
      const double f = std::exp(nu * t - std::exp(t) - lg - rs[i] * rs[i] * nu / (2.0 * std::exp(t)));
      s += (j == 0 || j == nt) ? 0.5 * f : f;
    }
    worst = std::max(worst, std::fabs(s * h - ref[i]));
  }
  return worst;
}

// Smallest r with phi_nu(r) <= target (bisection; phi is decreasing).
// Depends on (nu, target) alone, so results are cached.
double r_at_level(double nu, double target) {
  static std::mutex mu;
  static std::map<std::pair<double, double>, double> cache;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({nu, target});
    if (it != cache.end()) return it->second;
  }
  double lo = 0, hi = 1;
  while (phi_of_r(nu, hi) > target && hi < 1e4) hi *= 2;
  for (int it = 0; it < 80; ++it) {
    double mid = 0.5 * (lo + hi);
    (phi_of_r(nu, mid) > target ? lo : hi) = mid;
  }
  std::lock_guard<std::mutex> lk(mu);
  cache[{nu, target}] = hi;
  return hi;
}

// Continued fraction of the regularized incomplete beta function I_x(a, b)
// (DLMF 8.17.22), evaluated by the modified Lentz method; for x below the
// mean (a+1)/(a+b+2) it converges in a few dozen terms.
double betainc_cf(double a, double b, double x) {
  const double tiny = 1e-300;
  double c = 1.0, d = 1.0 - (a + b) * x / (a + 1.0);
  if (std::fabs(d) < tiny) d = tiny;
  d = 1.0 / d;
  double f = d;
  for (int m = 1; m <= 400; ++m) {
    const double m2 = 2.0 * m;
    double num = m * (b - m) * x / ((a + m2 - 1.0) * (a + m2));  // even step
    d = 1.0 + num * d;
    c = 1.0 + num / c;
    if (std::fabs(d) < tiny) d = tiny;
    if (std::fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    f *= d * c;
    num = -(a + m) * (a + b + m) * x / ((a + m2) * (a + m2 + 1.0));  // odd step
    d = 1.0 + num * d;
    c = 1.0 + num / c;
    if (std::fabs(d) < tiny) d = tiny;
    if (std::fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = d * c;
    f *= del;
    if (std::fabs(del - 1.0) < 1e-15) break;
  }
  return f;
}

double betainc_reg(double a, double b, double x) {
  if (x <= 0.0) return 0.0;
  if (x >= 1.0) return 1.0;
  const double lbeta = std::lgamma(a) + std::lgamma(b) - std::lgamma(a + b);
  if (x < (a + 1.0) / (a + b + 2.0))
    return std::exp(a * std::log(x) + b * std::log1p(-x) - lbeta) * betainc_cf(a, b, x) / a;
  return 1.0 - std::exp(b * std::log1p(-x) + a * std::log(x) - lbeta) * betainc_cf(b, a, 1.0 - x) / b;
}

// Regularized upper incomplete gamma Q(a, x): power series of P below a + 1,
// Legendre's continued fraction (modified Lentz) above.
double gammaincc_reg(double a, double x) {
  if (x <= 0.0) return 1.0;
  const double lg = std::lgamma(a);
  if (x < a + 1.0) {
    double term = 1.0 / a, sum = term;
    for (int n = 1; n < 1000; ++n) {
      term *= x / (a + n);
      sum += term;
      if (term < sum * 1e-17) break;
    }
    return 1.0 - sum * std::exp(-x + a * std::log(x) - lg);
  }
  const double tiny = 1e-300;
  double bq = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / bq, h = d;
  for (int i = 1; i < 1000; ++i) {
    const double an = -i * (i - a);
    bq += 2.0;
    d = an * d + bq;
    if (std::fabs(d) < tiny) d = tiny;
    c = bq + an / c;
    if (std::fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = d * c;
    h *= del;
    if (std::fabs(del - 1.0) < 1e-15) break;
  }
  return std::exp(-x + a * std::log(x) - lg) * h;
}

// Fraction of the spectral mass of the stationary kernel with length ell that
// lies outside the radius Omega (Fourier convention of Appendix D).  In
// t = 2 pi ell w the Matern density (1 + t^2/(2 nu))^-(nu + d/2) is a
// multivariate t with 2 nu degrees of freedom, whose mass beyond |t| = T is
// I_{2nu/(2nu+T^2)}(nu, d/2); the squared exponential's is Gaussian, with
// mass Q(d/2, T^2/2) beyond T.
double spectral_tail(double nu, int d, double ell, double Omega) {
  const double T = 2 * PI * ell * Omega;
  if (std::isinf(nu)) return gammaincc_reg(0.5 * d, 0.5 * T * T);
  return betainc_reg(nu, 0.5 * d, 2.0 * nu / (2.0 * nu + T * T));
}

// t grid of eq:trapsum for (nu, eps): closed-form start (the three terms of
// lemma lem:dt at eps/10 with unit constants), then the smallest N_t whose
// trapezoid sum reproduces phi_nu to eps/10 on sampled r.  The lemma leaves
// its constants open, and the discretisation term alone is up to 100x larger
// than e^(-pi^2/dt) for nu >= 3/2.  N_t costs plan time only (step 3 uses the
// precomputed tensor).  Depends on (nu, eps) alone, so results are cached.
void t_grid_rule(double nu, double eps, double* tmin_out, double* tmax_out, int* nt_out) {
  static std::mutex mu;
  static std::map<std::pair<double, double>, std::tuple<double, double, int>> cache;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({nu, eps});
    if (it != cache.end()) {
      std::tie(*tmin_out, *tmax_out, *nt_out) = it->second;
      return;
    }
  }
  double tmin, tmax;
  const double L10 = std::log(10.0 / eps);
  tmin = std::log(eps / 10.0) / nu;
  tmax = std::log(2.0 * L10) + 0.5;
  const double dt = PI * PI / L10;
  const int n0 = std::max(1, (int)std::ceil((tmax - tmin) / dt));
  const double target = eps / 10.0;
  const double rmax = r_at_level(nu, target);
  std::vector<double> rs, ref;
  for (int i = 0; i <= 160; ++i) {
    rs.push_back(rmax * i / 160.0);
    ref.push_back(phi_of_r(nu, rs.back()));
  }
  auto err = [&](int m) { return trap_error(nu, tmin, tmax, m, rs, ref); };
  int nt = n0;
  for (int round = 0; round < 6; ++round) {
    int lo = std::max(1, (int)std::ceil((tmax - tmin) / dt));
    nt = lo;
    if (err(lo) <= target) break;
    // doubling, then bisection for the smallest passing count
    int hi = lo;
    bool ok = false;
    while (hi < 8 * lo) {
      hi = std::min(2 * hi, 8 * lo);
      if (err(hi) <= target) {
        ok = true;
        break;
      }
    }
    nt = hi;
    if (!ok) {  // the truncation below t_min dominates: extend the range
      tmin -= std::log(10.0) / nu;
      continue;
    }
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      (err(mid) <= target ? hi : lo) = mid;
    }
    nt = hi;
    break;
  }
  std::lock_guard<std::mutex> lk(mu);
  cache[{nu, eps}] = std::make_tuple(tmin, tmax, nt);
  *tmin_out = tmin;
  *tmax_out = tmax;
  *nt_out = nt;
}

// Sup over (x, sigma) of the Chebyshev interpolation error of lemma lem:interp,
// sampled on a grid (the Lagrange basis evaluated in barycentric form).
double cheb_interp_error(double smin, double smax, int ns) {
  std::vector<double> sk(ns + 1), lam(ns + 1);
  for (int k = 0; k <= ns; ++k) {
    sk[k] = 0.5 * (std::cos(PI * k / ns) + 1.0) * (smax - smin) + smin;
    lam[k] = ((k % 2) ? -1.0 : 1.0) * ((k == 0 || k == ns) ? 0.5 : 1.0);
  }
  const int nsg = 97, nx = 97;
  std::vector<double> xs(nx), E((size_t)nx * (ns + 1));  // node Gaussians at the sample x
  for (int b = 0; b < nx; ++b) {
    xs[b] = 6.0 * smax * b / (nx - 1);
    for (int k = 0; k <= ns; ++k) E[(size_t)b * (ns + 1) + k] = std::exp(-xs[b] * xs[b] / (2 * sk[k] * sk[k]));
  }
  double worst = 0;
  std::vector<double> P(ns + 1);
  for (int a = 0; a < nsg; ++a) {
    double s = smin + (smax - smin) * (a + 0.5) / nsg;
    double den = 0;
    for (int k = 0; k <= ns; ++k) den += lam[k] / (s - sk[k]);
    for (int k = 0; k <= ns; ++k) P[k] = lam[k] / (s - sk[k]) / den;
    for (int b = 0; b < nx; ++b) {
      double ap = 0;
      const double* e = &E[(size_t)b * (ns + 1)];
      for (int k = 0; k <= ns; ++k) ap += P[k] * e[k];
      worst = std::max(worst, std::fabs(ap - std::exp(-xs[b] * xs[b] / (2 * s * s))));
    }
  }
  return worst;
}

// Gauss-Legendre nodes/weights on [-1,1] (Newton on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double dp = n * (z * p1 - p0) / (z * z - 1);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double dp = n * (z * p1 - p0) / (z * z - 1);
    x[i] = z;
    w[i] = 2.0 / ((1 - z * z) * dp * dp);
  }
}

// Fourier transform of the exponential-of-semicircle window
// psi(z) = exp(beta (sqrt(1 - (2z/w)^2) - 1)), |z| <= w/2 (grid units), at xi.
double es_hat(double xi, int w, double beta, const std::vector<double>& gx,
              const std::vector<double>& gw) {
  double s = 0;
  for (size_t q = 0; q < gx.size(); ++q) {
    double z = 0.5 * w * gx[q];
    double a = 2 * z / w;
    s += 0.5 * w * gw[q] * std::exp(beta * (std::sqrt(std::max(0.0, 1 - a * a)) - 1)) *
         std::cos(xi * z);
  }
  return s;
}

// Smallest FFT length >= need that the pass kernel supports (single pass).
int fft_len_at_least(int64_t need) {
  int best = 0;
  for (int a = 3; a <= 13; ++a)
    for (int t = 1; t <= 3; t += 2) {
      int64_t L = (int64_t)t << a;
      if (L >= need && fft_length_supported((int)L) && (best == 0 || L < best)) best = (int)L;
    }
  return best;
}

}  // namespace

void input_ranges(int d, int64_t n, const double* x, const double* sigma, const double* l,
                  const gp_opts& opts, InputRanges* R) {
  for (int r = 0; r < 3; ++r) {
    R->lo[r] = r < d ? std::numeric_limits<double>::infinity() : 0.0;
    R->hi[r] = r < d ? -std::numeric_limits<double>::infinity() : 0.0;
  }
  R->lmin = std::numeric_limits<double>::infinity();
  R->lmax = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int r = 0; r < d; ++r) {
      const double v = x[i * d + r];
      if (!std::isfinite(v)) throw Error{GP_EDOMAIN, "non-finite point coordinate"};
      R->lo[r] = std::min(R->lo[r], v);
      R->hi[r] = std::max(R->hi[r], v);
    }
    if (!(sigma[i] > 0) || !std::isfinite(sigma[i]))
      throw Error{GP_EDOMAIN, "sigma must be finite and > 0"};
    if (!(l[i] > 0) || !std::isfinite(l[i])) throw Error{GP_EDOMAIN, "l must be finite and > 0"};
    R->lmin = std::min(R->lmin, l[i]);
    R->lmax = std::max(R->lmax, l[i]);
  }
  if (opts.use_box) {
    for (int r = 0; r < d; ++r) {
      if (!(opts.box_lo[r] <= R->lo[r] && opts.box_hi[r] >= R->hi[r]))
        throw Error{GP_ERANGE, "points outside gp_opts box"};
      R->lo[r] = opts.box_lo[r];
      R->hi[r] = opts.box_hi[r];
    }
  }
  if (opts.l_lo > 0) R->lmin = std::min(R->lmin, opts.l_lo);
  if (opts.l_hi > 0) R->lmax = std::max(R->lmax, opts.l_hi);
}

void map_box(PlanRules* P, const InputRanges& R) {
  double ext = 0;
  for (int r = 0; r < 3; ++r) P->center[r] = 0;
  for (int r = 0; r < P->d; ++r) {
    P->center[r] = 0.5 * (R.lo[r] + R.hi[r]);
    ext = std::max(ext, R.hi[r] - R.lo[r]);
  }
  if (!(ext > 0)) ext = 2.0;
  P->scale = 2.0 / ext;
  P->l_range_lo = R.lmin;
  P->l_range_hi = R.lmax;
}

void choose_params(PlanRules* P, int d, double nu, double tol, double lmin, double lmax,
                   const gp_opts& opts) {
  // ---- width range (sigma_p = l'/sqrt 2) and Chebyshev degree (section 3.3)
  const double sq2 = std::sqrt(2.0);
  double smin = lmin * P->scale / sq2, smax = lmax * P->scale / sq2;
  if (opts.s_min > 0 || opts.s_max > 0) {
    if (!(opts.s_min > 0 && opts.s_max >= opts.s_min))
      throw Error{GP_EINVAL, "s_min/s_max must both be set, 0 < s_min <= s_max"};
    if (opts.s_min > smin * (1 + 1e-12) || opts.s_max < smax * (1 - 1e-12))
      throw Error{GP_ERANGE, "gp_opts width range does not contain the data's"};
    smin = opts.s_min;
    smax = opts.s_max;
  }
  const double eps = tol;
  if (opts.n_sigma >= 0) {
    P->n_sigma = opts.n_sigma;
  } else if (smax <= smin * (1 + 1e-13)) {
    P->n_sigma = 0;
  } else {
    const double kappa = smax / smin;
    const double target = eps / 10;
    int nb = 1;
    while (2 * (kappa - 1) * std::pow((kappa - 1) / (kappa + 1), nb) > target && nb < 200) ++nb;
    // smallest ns in [1, nb] meeting the target (the error falls with ns)
    int lo_ns = 0, ns = nb;
    while (ns - lo_ns > 1) {
      const int mid = (lo_ns + ns) / 2;
      (cheb_interp_error(smin, smax, mid) > target ? lo_ns : ns) = mid;
    }
    if (ns % 2 == 0) ++ns;  // N_sigma + 1 even: grids pack in complex pairs
    P->n_sigma = ns;
  }
  if (P->n_sigma == 0) smax = smin;
  P->s_min = smin;
  P->s_max = smax;
  if (P->n_sigma > 47) throw Error{GP_EUNSUPPORTED, "N_sigma > 47 not supported"};

  // ---- t discretisation (section 3.2, lemma lem:dt)
  if (P->se) {
    P->t_min = P->t_max = 0;
    P->n_t = 0;
  } else if (opts.n_t >= 1) {
    if (!(opts.t_max > opts.t_min)) throw Error{GP_EINVAL, "t_max must exceed t_min"};
    P->t_min = opts.t_min;
    P->t_max = opts.t_max;
    P->n_t = opts.n_t;
  } else {
    t_grid_rule(nu, eps, &P->t_min, &P->t_max, &P->n_t);
  }

  // ---- Fourier grid spacing: aliasing images at distance >= 1/dw - 2 see the
  // kernel's own tail; ask phi_nu(r) <= eps/10 there for the widest length.
  const double lpmax = lmax * P->scale, lpmin = lmin * P->scale;
  if (opts.dw > 0) {
    P->dw = opts.dw;
  } else {
    double r_eps = r_at_level(nu, eps / 10);
    P->dw = std::min(0.45, 1.0 / (2.0 + lpmax * r_eps));
  }
  if (!(P->dw > 0 && P->dw < 0.5)) throw Error{GP_EINVAL, "Delta-omega must be in (0, 1/2)"};

  // ---- Fourier half-width: spectral tail of the narrowest kernel <= eps
  int64_t mcap = opts.M_cap > 0 ? opts.M_cap : (d == 1 ? (int64_t)1 << 18 : 2047);
  if (opts.M > 0) {
    P->M = opts.M;
  } else {
    double lo_O = 1e-3, hi_O = 1.0;
    while (spectral_tail(nu, d, lpmin, hi_O) > eps && hi_O < 1e12) hi_O *= 2;
    for (int it = 0; it < 60; ++it) {
      double mid = std::sqrt(lo_O * hi_O);
      (spectral_tail(nu, d, lpmin, mid) > eps ? lo_O : hi_O) = mid;
    }
    int64_t M = (int64_t)std::ceil(hi_O / P->dw);
    M = std::max<int64_t>(M, 4);
    if (M > mcap) {
      M = mcap;
      P->m_capped = 1;
    }
    P->M = M;
  }
  P->pred_tail = spectral_tail(nu, d, lpmin, P->M * P->dw);
  P->mcount = 2 * P->M + 1;

  // ---- flat t nodes (rem:step3): G^_kj[n] = C_kj exp(-tau_kj |n|^2) with
  // tau_kj = 2 pi^2 sigma_k^2 chi_j^2 dw^2; where even the largest exponent
  // over the mode box, tau at sigma_max times d M^2, is <= 1e-3 tol, the term
  // is constant over the box to that accuracy.  chi_j grows with j, so these
  // are the leading nodes; two or more of them are merged into one term.
  P->tol = tol;
  P->n_flat = 0;
  if (!P->se && !opts.keep_t) {
    const double dt = (P->t_max - P->t_min) / P->n_t;
    const double smax2 = P->s_max * P->s_max;
    int nf0 = 0;
    for (int j = 0; j <= P->n_t; ++j) {
      const double t = P->t_min + j * dt;
      const double chi2 = std::exp(t) / nu;
      const double x = 2 * PI * PI * smax2 * chi2 * P->dw * P->dw * (double)d * (double)P->M * (double)P->M;
      if (!(x <= 1e-3 * tol)) break;
      ++nf0;
    }
    P->n_flat = nf0 >= 2 ? nf0 : 0;
  }
  P->nt_eff = P->se ? 1 : P->n_t + 1 - P->n_flat + (P->n_flat > 0 ? 1 : 0);

  // ---- spreading window (exponential of semicircle) and oversampled grid
  double ntol = opts.nufft_tol > 0 ? opts.nufft_tol : eps;
  if (P->precision == GP_FP32_BULK) ntol = std::max(ntol, 1e-6);
  ntol = std::min(ntol, 1e-1);
  P->nufft_tol = ntol;
  // Exponential-of-semicircle window for oversampling sigma (Barnett, Magland
  // and af Klinteberg 2019): the width whose error estimate
  // exp(-pi w sqrt(1 - 1/sigma)) reaches ntol/10 (at sigma = 2 their
  // w = ceil(log10(10/ntol))), and the shape parameter of their rule.
  // Automatic: 1.25 in 2-D, where the FFT passes dominate and the grids
  // shrink to (6144/8192)^2 = 0.56x at the d=2 N=1e6 workload (fp64 step
  // 9.8 -> 9.1 ms, fp32 3.2 -> 2.4 ms); 2 in 3-D, where spreading dominates
  // and the wider window costs more than the grid saves (w^3: 125 -> 216),
  // and in 1-D.
  const double ups = opts.upsample > 0 ? opts.upsample : (d == 2 ? 1.25 : 2.0);
  if (!(ups >= 1.25 && ups <= 2.0)) throw Error{GP_EINVAL, "upsample must be in [1.25, 2]"};
  auto set_window = [&](double sg) {
    if (sg >= 2.0) {
      P->w = (int)std::ceil(std::log10(1.0 / ntol)) + 1;
      P->w = std::max(2, std::min(16, P->w));
      P->beta = 2.30 * P->w;
    } else {
      P->w = (int)std::ceil(std::log(10.0 / ntol) / (PI * std::sqrt(1.0 - 1.0 / sg)));
      P->w = std::max(2, std::min(16, P->w));
      P->beta = 0.97 * PI * (1.0 - 0.5 / sg) * P->w;
    }
  };
  set_window(ups);
  const int64_t need_os = (int64_t)std::ceil(ups * (double)P->mcount);
  const double margin = 0.5 * P->w + 2.0;
  const int64_t need_wrap = (int64_t)std::ceil(margin / (0.5 - P->dw));
  const int64_t need = std::max<int64_t>({need_os, need_wrap, 2 * (int64_t)P->w, 16});
  int nf = fft_len_at_least(need);
  P->fourstep = 0;
  if (nf == 0) {
    if (d != 1) throw Error{GP_EUNSUPPORTED, "Fourier grid too large for d >= 2 (reduce M)"};
    // d = 1: nf = L1 * L2 with both factors single-pass lengths
    int64_t best = 0;
    int b1 = 0, b2 = 0;
    for (int a1 = 3; a1 <= 13; ++a1)
      for (int t1 = 1; t1 <= 3; t1 += 2)
        for (int a2 = 3; a2 <= 13; ++a2)
          for (int t2 = 1; t2 <= 3; t2 += 2) {
            int64_t L1 = (int64_t)t1 << a1, L2 = (int64_t)t2 << a2;
            if (!fft_length_supported((int)L1) || !fft_length_supported((int)L2)) continue;
            int64_t L = L1 * L2;
            if (L >= need && (best == 0 || L < best || (L == best && std::llabs(L1 - L2) < std::llabs(b1 - b2)))) {
              best = L;
              b1 = (int)L1;
              b2 = (int)L2;
            }
          }
    if (best == 0) throw Error{GP_EUNSUPPORTED, "Fourier grid too large"};
    if (best > (int64_t)1 << 26) throw Error{GP_EUNSUPPORTED, "Fourier grid too large"};
    nf = (int)best;
    P->fourstep = 1;
    P->L1 = b1;  // contiguous factor
    P->L2 = b2;
  }
  // FFT lengths come in steps of 4/3 and 3/2, so the grid is usually finer
  // than asked: size the window for the oversampling reached (never wider
  // than the first choice, so the margins above still hold).
  P->upsample = std::min(2.0, (double)nf / (double)P->mcount);
  if (ups < 2.0) set_window(P->upsample);
  const int tile_d[4] = {0, 256, 16, 8};
  for (int r = 0; r < 3; ++r) {
    if (r >= d) {
      P->nf[r] = 1;
      P->lo[r] = 0;
      P->na[r] = 1;
      P->tile[r] = 1;
      P->nbins[r] = 1;
      continue;
    }
    P->nf[r] = nf;
    int a0 = (int)std::floor(0.5 * nf - nf * P->dw - 0.5 * P->w) - 1;
    int a1 = (int)std::ceil(0.5 * nf + nf * P->dw + 0.5 * P->w) + 1;
    a0 = std::max(a0, 0);
    a1 = std::min(a1, nf - 1);
    // the largest tile (a power of two, at most the default) for which a
    // whole number of tiles covers cells a0..a1 inside the grid
    int tl = tile_d[d], na = 0;
    for (;; tl /= 2) {
      na = ((a1 - a0 + 1 + tl - 1) / tl) * tl;
      if (na <= nf || tl == 1) break;
    }
    a0 = std::min(a0, nf - na);
    P->lo[r] = a0;
    P->na[r] = na;
    P->tile[r] = tl;
    P->nbins[r] = na / tl;
  }
  P->n_bins = (int64_t)P->nbins[0] * P->nbins[1] * P->nbins[2];
  // a point's window starts in its own tile and reaches at most nsrc - 1
  // tiles further along each dimension
  P->nsrc = 2;
  for (int r = 0; r < d; ++r) P->nsrc = std::max(P->nsrc, (P->w - 2) / P->tile[r] + 2);
  P->nk = P->n_sigma + 1;
  P->npair = (P->nk + 1) / 2;
  P->nkp = P->nk + (P->nk & 1);
}

void step3_rows(const PlanRules& P, std::vector<double>& svals, std::vector<int>& rowmap) {
  const int64_t M = P.M;
  svals.clear();
  rowmap.clear();
  if (P.d == 1) {
    svals.resize(M + 1);
    for (int64_t m = 0; m <= M; ++m) svals[m] = (double)(m * m);
    return;
  }
  const int64_t smax = (int64_t)P.d * M * M;
  std::vector<char> present(smax + 1, 0);
  if (P.d == 2) {
    for (int64_t a0 = 0; a0 <= M; ++a0)
      for (int64_t a1 = 0; a1 <= M; ++a1) present[a0 * a0 + a1 * a1] = 1;
  } else {
    for (int64_t a0 = 0; a0 <= M; ++a0)
      for (int64_t a1 = 0; a1 <= M; ++a1)
        for (int64_t a2 = 0; a2 <= M; ++a2) present[a0 * a0 + a1 * a1 + a2 * a2] = 1;
  }
  rowmap.assign(smax + 1, -1);
  for (int64_t v = 0; v <= smax; ++v)
    if (present[v]) {
      rowmap[v] = (int)svals.size();
      svals.push_back((double)v);
    }
}

void host_tables(PlanRules* P, StepTables* T) {
  const int d = P->d;
  const double smin = P->s_min, smax = P->s_max;
  // Chebyshev-Lobatto nodes on [s_min, s_max] and their barycentric weights
  // (eq:chebscheme)
  P->sig_nodes.resize(P->nk);
  P->bary.resize(P->nk);
  for (int k = 0; k < P->nk; ++k) {
    if (P->n_sigma == 0) {
      P->sig_nodes[k] = smin;
      P->bary[k] = 1;
    } else {
      P->sig_nodes[k] = 0.5 * (std::cos(PI * k / P->n_sigma) + 1.0) * (smax - smin) + smin;
      P->bary[k] = ((k % 2) ? -1.0 : 1.0) * ((k == 0 || k == P->n_sigma) ? 0.5 : 1.0);
    }
  }
  // trapezoid nodes in t (eq:trapsum, eq:dtscheme) with the factor dw^d
  const int nt_paper = P->se ? 1 : P->n_t + 1;
  P->vt.resize(nt_paper);
  P->chi.resize(nt_paper);
  const double dwd = std::pow(P->dw, d);
  if (P->se) {
    P->vt[0] = dwd;
    P->chi[0] = 1.0;
  } else {
    const double dt = (P->t_max - P->t_min) / P->n_t, lg = std::lgamma(P->nu);
    for (int j = 0; j <= P->n_t; ++j) {
      double t = P->t_min + (double)j / P->n_t * (P->t_max - P->t_min);
      double u = std::exp(P->nu * t - std::exp(t) - lg);        // eq:maternpres
      double ch = std::exp(0.5 * t) / std::sqrt(P->nu);
      double v = std::pow(ch, -(double)d) * u;                  // eq:v
      P->vt[j] = dwd * v * dt * ((j == 0 || j == P->n_t) ? 0.5 : 1.0);  // eq:trapsum
      P->chi[j] = ch;
    }
  }
  // The step-3 terms: per table node j and width k, the weight v~_j, the
  // constant C_kj and the exponent tau_kj of G^_kj[n] = C_kj exp(-tau_kj |n|^2).
  // The merged flat nodes form one term with tau = 0: their C_kj =
  // (2 pi chi_j^2)^(d/2) sigma_k^d, so sum_j v~_j C_k'j C_kj over them is
  // W sigma_k'^d sigma_k^d with W = sum_j v~_j (2 pi chi_j^2)^d.
  T->tvt.assign(P->nt_eff, 0.0);
  T->tcst.assign((size_t)P->nt_eff * P->nk, 0.0);
  T->ttau.assign((size_t)P->nt_eff * P->nk, 0.0);
  int jt = 0;
  if (P->n_flat > 0) {
    double W = 0.0;
    for (int j = 0; j < P->n_flat; ++j) W += P->vt[j] * std::pow(2 * PI * P->chi[j] * P->chi[j], (double)d);
    T->tvt[0] = W;
    for (int k = 0; k < P->nk; ++k) {
      T->tcst[k] = std::pow(P->sig_nodes[k], (double)d);
      T->ttau[k] = 0.0;
    }
    jt = 1;
  }
  for (int j = P->n_flat; j < nt_paper && jt < P->nt_eff; ++j, ++jt) {
    T->tvt[jt] = P->vt[j];
    for (int k = 0; k < P->nk; ++k) {
      const double s2 = P->sig_nodes[k] * P->sig_nodes[k] * P->chi[j] * P->chi[j];
      T->tcst[(size_t)jt * P->nk + k] = std::pow(2 * PI * s2, 0.5 * d);
      T->ttau[(size_t)jt * P->nk + k] = 2 * PI * PI * s2 * P->dw * P->dw;
    }
  }
  if (jt != P->nt_eff) throw Error{GP_EDEVICE, "internal: t node count"};
  // Fourier multipliers of G_{k,t_j} (eq:Gkt) on the grid, separated by
  // dimension: G^_{kj}[n] = C_kj prod_r exp(-tau_kj n_r^2); g0 carries the
  // constant and dimension 0, e1 the rest.
  const int64_t M1 = P->M + 1;
  T->g0.assign((size_t)P->nt_eff * P->nk * M1, 0.0);
  T->e1.assign((size_t)P->nt_eff * P->nk * M1, 0.0);
  for (int j = 0; j < P->nt_eff; ++j)
    for (int k = 0; k < P->nk; ++k) {
      const double cst = T->tcst[(size_t)j * P->nk + k];
      const double tau = T->ttau[(size_t)j * P->nk + k];
      for (int64_t m = 0; m < M1; ++m) {
        const double e = std::exp(-tau * (double)m * (double)m);
        T->g0[((size_t)j * P->nk + k) * M1 + m] = cst * e;
        T->e1[((size_t)j * P->nk + k) * M1 + m] = e;
      }
    }
  // deconvolution 1/psi^(2 pi n / nf) of the window (Appendix D NUFFTs)
  std::vector<double> gx, gw;
  gauss_legendre(120 + 8 * P->w, gx, gw);
  T->dec.assign((size_t)d * M1, 0.0);
  for (int r = 0; r < d; ++r)
    for (int64_t m = 0; m < M1; ++m)
      T->dec[r * M1 + m] = 1.0 / es_hat(2 * PI * (double)m / P->nf[r], P->w, P->beta, gx, gw);
}

void lowrank_rows(int64_t nrows, int nk, int nkp, const std::vector<double>& A, double rel,
                  std::vector<int64_t>& off, std::vector<double>& rows, int* rank_max,
                  double* rank_mean) {
  const int npk = nkp * (nkp + 1) / 2;
  std::vector<int> rank(nrows);
  std::vector<double> fac((size_t)nrows * nk * nkp);  // up to nk factors per row
  auto work = [&](int64_t r0, int64_t r1) {
    std::vector<double> S((size_t)nk * nk), L((size_t)nk * nk);
    std::vector<int> perm(nk);
    for (int64_t r = r0; r < r1; ++r) {
      const double* a = A.data() + (size_t)r * npk;
      for (int k1 = 0, p = 0; k1 < nkp; ++k1)
        for (int k2 = k1; k2 < nkp; ++k2, ++p)
          if (k1 < nk && k2 < nk) S[(size_t)k1 * nk + k2] = S[(size_t)k2 * nk + k1] = a[p];
      double dmax = 0.0;
      for (int k = 0; k < nk; ++k) {
        perm[k] = k;
        dmax = std::max(dmax, S[(size_t)k * nk + k]);
      }
      std::fill(L.begin(), L.end(), 0.0);  // L[k][a]: factor a at width k (original order)
      int rk = 0;
      for (int a = 0; a < nk; ++a) {
        int best = a;
        for (int i = a + 1; i < nk; ++i)
          if (S[(size_t)perm[i] * nk + perm[i]] > S[(size_t)perm[best] * nk + perm[best]]) best = i;
        std::swap(perm[a], perm[best]);
        const int pa = perm[a];
        const double dd = S[(size_t)pa * nk + pa];
        if (!(dmax > 0.0) || !(dd > rel * dmax)) break;
        const double lv = std::sqrt(dd);
        for (int i = a; i < nk; ++i) L[(size_t)perm[i] * nk + a] = S[(size_t)perm[i] * nk + pa] / lv;
        for (int i = a + 1; i < nk; ++i)
          for (int q = a + 1; q < nk; ++q)
            S[(size_t)perm[i] * nk + perm[q]] -= L[(size_t)perm[i] * nk + a] * L[(size_t)perm[q] * nk + a];
        ++rk;
      }
      rank[r] = rk;
      double* f = fac.data() + (size_t)r * nk * nkp;
      for (int a = 0; a < rk; ++a)
        for (int k = 0; k < nkp; ++k) f[(size_t)a * nkp + k] = k < nk ? L[(size_t)k * nk + a] : 0.0;
    }
  };
  const int nth = (int)std::max<unsigned>(1, std::min<unsigned>(16, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  const int64_t chunk = (nrows + nth - 1) / nth;
  for (int t = 0; t < nth; ++t) {
    const int64_t r0 = t * chunk, r1 = std::min<int64_t>(nrows, r0 + chunk);
    if (r0 < r1) th.emplace_back(work, r0, r1);
  }
  for (auto& t : th) t.join();
  off.assign(nrows + 1, 0);
  int64_t sum = 0;
  int mx = 0;
  for (int64_t r = 0; r < nrows; ++r) {
    off[r + 1] = off[r] + (int64_t)rank[r] * nkp;
    sum += rank[r];
    mx = std::max(mx, rank[r]);
  }
  rows.resize((size_t)off[nrows]);
  for (int64_t r = 0; r < nrows; ++r)
    std::copy(fac.begin() + (size_t)r * nk * nkp, fac.begin() + (size_t)r * nk * nkp + (off[r + 1] - off[r]),
              rows.begin() + off[r]);
  *rank_max = mx;
  *rank_mean = nrows > 0 ? (double)sum / nrows : 0.0;
}

void twiddle_table(int L, std::vector<double>& t) {
  t.resize(2 * (size_t)L);
  for (int k = 0; k < L; ++k) {
    const long double a = -2.0L * 3.14159265358979323846264338327950288L * k / L;
    t[2 * k] = (double)cosl(a);
    t[2 * k + 1] = (double)sinl(a);
  }
}

}  // namespace gp

// Defaults of the plan options (host only; declared in the C interface).
extern "C" int gp_opts_init(gp_opts* o) {
  if (!o) return GP_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->precision = GP_FP64;
  o->n_sigma = -1;
  o->n_t = -1;
  return GP_OK;
}
