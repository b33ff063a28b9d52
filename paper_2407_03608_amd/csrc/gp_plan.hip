// Plan construction: parameter choice, tables, point records and bin sort.
//
// The plan fixes the operator K~ of eq:Ktilde (section 3.5): the trapezoid
// rule in t (eq:trapsum, eq:dtscheme), the Chebyshev-Lobatto grid in the width
// (eq:chebscheme), and the Fourier grid Delta-omega {-M..M}^d (section 3.4),
// plus the spreading window and oversampled grid that realise the two NUFFTs
// (Appendix D).  It also sorts the points into spreading tiles so that every
// matvec works on bin-ordered records (the CG vectors stay in that order).
#include <algorithm>
#include <cmath>
#include <tuple>
#include <mutex>
#include <map>
#include <cstring>
#include <limits>
#include <thread>

#include "gp_internal.h"

namespace gp {

static const double PI = 3.14159265358979323846264338327950288;

void DevBuf::alloc(size_t b) {
  release();
  if (b == 0) b = 256;
  hipError_t e = hipMalloc(&p, b);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    throw Error{GP_ENOMEM, "hipMalloc(" + std::to_string(b) + " bytes) failed: " +
                               hipGetErrorString(e)};
  }
  bytes = b;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
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

// ---------------------------------------------------------- device parts ----

struct RecArgs {
  int d;
  int64_t n;
  double center[3], scale, dw;
  int nf[3], lo[3], tile[3], nbins[3], na[3];
  int w;
};

// Per point: mapped coordinate x' = (x - c) scale, fine-grid position
// g = nf/2 + nf dw x' (so theta + pi = 2 pi g / nf with theta = 2 pi dw x'),
// first window cell s = ceil(g - w/2), offset delta = s - g, its tile, and
// sigma_p = l'/sqrt(2), prefactor s(x) (2/(pi l'^2))^(d/4) of eq:Wk.
__global__ void records_kernel(RecArgs a, const double* __restrict__ pts,
                               const double* __restrict__ sig, const double* __restrict__ l,
                               int* __restrict__ bin_of, int* __restrict__ cell_tmp,
                               double* __restrict__ frac_tmp, double* __restrict__ sp_tmp,
                               double* __restrict__ pf_tmp, int* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  int64_t bin = 0, mul = 1;
  for (int r = 0; r < a.d; ++r) {
    double xp = (pts[i * a.d + r] - a.center[r]) * a.scale;
    double g = 0.5 * a.nf[r] + a.nf[r] * a.dw * xp;
    double s = ceil(g - 0.5 * a.w);
    int sa = (int)s - a.lo[r];
    if (!(sa >= 0 && sa + a.w <= a.na[r])) {
      atomicOr(bad, 1);
      sa = sa < 0 ? 0 : (sa + a.w > a.na[r] ? a.na[r] - a.w : sa);
    }
    cell_tmp[r * a.n + i] = sa;
    frac_tmp[r * a.n + i] = s - g;
    bin += (int64_t)(sa / a.tile[r]) * mul;
    mul *= a.nbins[r];
  }
  double lp = l[i] * a.scale;
  sp_tmp[i] = lp * 0.70710678118654752440;
  pf_tmp[i] = sig[i] * pow(2.0 / (3.14159265358979323846 * lp * lp), 0.25 * a.d);
  bin_of[i] = (int)bin;
}

// Scatter the per-point data into bin order and evaluate, once per plan, the
// window values psi(delta + q), q < w (exponential of semicircle) and the
// weights w_k(x) = s(x)(2/(pi l'^2))^(d/4) P_k(sigma_p(x)) of eq:Wk with the
// Lagrange basis in barycentric form on the Chebyshev-Lobatto nodes.
template <typename T>
__global__ void scatter_records_kernel(int d, int64_t n, int w, double beta, int nk, int nkp,
                                       int rs, const int* __restrict__ posv,
                                       const int* __restrict__ cell_tmp,
                                       const double* __restrict__ frac_tmp,
                                       const double* __restrict__ sp_tmp,
                                       const double* __restrict__ pf_tmp,
                                       const double* __restrict__ nodes,
                                       const double* __restrict__ bary, int* __restrict__ perm,
                                       int* __restrict__ cell, T* __restrict__ pw) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t pos = posv[i];
  perm[pos] = (int)i;
  T* row = pw + pos * rs;
  const double tw = 2.0 / w;
  for (int r = 0; r < d; ++r) {
    cell[r * n + pos] = cell_tmp[r * n + i];
    const double del = frac_tmp[r * n + i];
    for (int q = 0; q < w; ++q) {
      const double z = (del + q) * tw;
      const double u = 1.0 - z * z;
      row[r * w + q] = (T)(u >= 0.0 ? exp(beta * (sqrt(u) - 1.0)) : 0.0);
    }
  }
  const double sp = sp_tmp[i], pf = pf_tmp[i];
  int hit = -1;
  double den = 0;
  for (int k = 0; k < nk; ++k) {
    const double dk = sp - nodes[k];
    if (dk == 0.0) {
      hit = k;
      break;
    }
    den += bary[k] / dk;
  }
  for (int k = 0; k < nkp; ++k) {
    double v = 0;
    if (k < nk) v = hit >= 0 ? (k == hit ? 1.0 : 0.0) : bary[k] / (sp - nodes[k]) / den;
    row[d * w + k] = (T)(pf * v);
  }
}

// Row r of the precomputed step-3 tensor (rem:step3) at |n|^2 = svals[r]:
//   A_k'k = sum_j v~_j G^_k'j G^_kj = sum_j v~_j C_k'j C_kj exp(-(tau_k'j + tau_kj) |n|^2)
// (eq:Gkt on the grid), one thread per (row, upper-triangle entry), fp64.
template <typename T>
__global__ void atab_kernel(int64_t rows, int npk, int nkp, int nk, int nt,
                            const double* __restrict__ svals, const double* __restrict__ tau,
                            const double* __restrict__ cst, const double* __restrict__ vt,
                            T* __restrict__ A) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * npk) return;
  const int64_t r = e / npk;
  int p = (int)(e - r * npk);
  int k1 = 0;
  while (p >= nkp - k1) {
    p -= nkp - k1;
    ++k1;
  }
  const int k2 = k1 + p;
  double sum = 0;
  if (k1 < nk && k2 < nk) {
    const double sv = svals[r];
    for (int j = 0; j < nt; ++j)
      sum += vt[j] * cst[j * nk + k1] * cst[j * nk + k2] *
             exp(-(tau[j * nk + k1] + tau[j * nk + k2]) * sv);
  }
  A[e] = (T)sum;
}

}  // namespace

// Sort a point set into the plan's tiles and build its records (used for the
// training points at plan time and for posterior targets).
struct Records;  // fwd (defined in nufft.hip via Plan buffers)

// Chunk sizes of the work lists: a tile (bin) is split when it holds more
// than kImbalance times the mean load, so the densest tiles of clustered
// points do not serialise a launch; at least kMin*Chunk per item, and never
// more than about kMaxItems chunked items.
constexpr int64_t kImbalance = 4;
constexpr int64_t kMaxItems = 65536;
constexpr int64_t kMinSpreadChunk = 256;
constexpr int64_t kMinInterpChunk = 64;
constexpr int64_t kMinSuperChunk = 128;

static int64_t chunk_size(int64_t total, int64_t units, int64_t min_chunk) {
  const int64_t mean = (total + std::max<int64_t>(units, 1) - 1) / std::max<int64_t>(units, 1);
  return std::max({min_chunk, kImbalance * mean, total / kMaxItems});
}

static int64_t source_total_bound(const Plan* P, int64_t n) {
  int64_t m = 1;
  for (int r = 0; r < P->d; ++r) m *= P->nsrc;
  return n * m;
}

static int slot_pairs(const Plan* P) { return (int)std::min<int64_t>(8, P->npair); }

// Device bytes of the work lists and partial tiles, bounded before the bin
// sort is known (plan query) by the chunk-size rule.
size_t work_list_bound_bytes(const Plan* P, int64_t n, size_t cs) {
  const int64_t ts = source_total_bound(P, n);
  const int64_t qs = chunk_size(ts, P->n_bins, kMinSpreadChunk);
  const int64_t slots = 2 * ts / qs + 2;
  const int64_t tcells = (int64_t)P->tile[0] * P->tile[1] * P->tile[2];
  const int64_t items = P->n_bins + ts / qs + 1;
  const int64_t qi = chunk_size(n, P->n_bins, kMinInterpChunk);
  const int64_t iitems = P->n_bins + n / qi + 1;
  const int64_t nsup = (int64_t)((P->nbins[0] + 1) / 2) * ((P->nbins[1] + 1) / 2) *
                       (P->d > 2 ? P->nbins[2] : 1);
  const int64_t sitems = P->d >= 2 ? nsup + n / chunk_size(n, nsup, kMinSuperChunk) + 1 : 0;
  return (size_t)(2 * items + iitems + sitems) * 16 + (size_t)slots * tcells * slot_pairs(P) * cs;
}

// Build the spread and interpolation work lists from the bin offsets.  The
// source sequence of a tile is the concatenation of its source bins in the
// order the spread kernel visits them (offset q along each dimension, the
// first dimension fastest; bins before the grid start are skipped).
static void build_work_lists(Plan* P, Records& R, const std::vector<int>& start, size_t cs) {
  const int d = P->d, nsrc = P->nsrc;
  int nsrc_tot = 1;
  for (int r = 0; r < d; ++r) nsrc_tot *= nsrc;
  std::vector<int64_t> src(P->n_bins);
  int64_t ts = 0;
  for (int64_t t = 0; t < P->n_bins; ++t) {
    int tc[3] = {0, 0, 0};
    int64_t tb = t;
    for (int r = 0; r < d; ++r) {
      tc[r] = (int)(tb % P->nbins[r]);
      tb /= P->nbins[r];
    }
    int64_t cnt = 0;
    for (int sb = 0; sb < nsrc_tot; ++sb) {
      int64_t bin = 0, mul = 1;
      bool ok = true;
      int q = sb;
      for (int r = 0; r < d; ++r) {
        const int br = tc[r] - (q % nsrc);
        q /= nsrc;
        if (br < 0) ok = false;
        bin += (int64_t)br * mul;
        mul *= P->nbins[r];
      }
      if (ok) cnt += start[bin + 1] - start[bin];
    }
    src[t] = cnt;
    ts += cnt;
  }
  const int64_t qs = chunk_size(ts, P->n_bins, kMinSpreadChunk);
  std::vector<int> spw, spr;
  int64_t slots = 0;
  for (int64_t t = 0; t < P->n_bins; ++t) {
    const int64_t c = std::max<int64_t>(1, (src[t] + qs - 1) / qs);
    if (c == 1) {
      spw.insert(spw.end(), {(int)t, 0, (int)src[t], -1});
      continue;
    }
    // equal chunks
    for (int64_t j = 0; j < c; ++j)
      spw.insert(spw.end(), {(int)t, (int)(src[t] * j / c), (int)(src[t] * (j + 1) / c),
                             (int)(slots + j)});
    spr.insert(spr.end(), {(int)t, (int)slots, (int)c, 0});
    slots += c;
  }
  const int64_t qi = chunk_size(R.n, P->n_bins, kMinInterpChunk);
  std::vector<int> inw;
  for (int64_t b = 0; b < P->n_bins; ++b) {
    const int64_t cnt = start[b + 1] - start[b];
    if (cnt == 0) continue;
    const int64_t c = (cnt + qi - 1) / qi;
    for (int64_t j = 0; j < c; ++j)
      inw.insert(inw.end(), {(int)b, (int)(start[b] + cnt * j / c), (int)(start[b] + cnt * (j + 1) / c), 0});
  }
  // 2x2 super-bins (d = 2): the points of bin rows 2sy and 2sy+1, bins
  // 2sx..2sx+1 of each, in that order
  std::vector<int> inw2;
  if (d >= 2) {
    const int nsb0 = (P->nbins[0] + 1) / 2, nsb1 = (P->nbins[1] + 1) / 2;
    const int nsb2 = d > 2 ? P->nbins[2] : 1;
    const int64_t q2 = chunk_size(R.n, (int64_t)nsb0 * nsb1 * nsb2, kMinSuperChunk);
    for (int sz = 0; sz < nsb2; ++sz)
      for (int sy = 0; sy < nsb1; ++sy)
        for (int sx = 0; sx < nsb0; ++sx) {
          const int bx0 = 2 * sx, bx1 = std::min(2 * sx + 1, P->nbins[0] - 1);
          int64_t cnt = 0;
          for (int q = 0; q < 2; ++q) {
            const int by = 2 * sy + q;
            if (by >= P->nbins[1]) break;
            const int64_t rowbin = ((int64_t)sz * P->nbins[1] + by) * P->nbins[0];
            cnt += start[rowbin + bx1 + 1] - start[rowbin + bx0];
          }
          if (cnt == 0) continue;
          const int64_t c = (cnt + q2 - 1) / q2;
          const int sb = (sz * nsb1 + sy) * nsb0 + sx;
          for (int64_t j = 0; j < c; ++j)
            inw2.insert(inw2.end(), {sb, (int)(cnt * j / c), (int)(cnt * (j + 1) / c), 0});
        }
  }
  hipStream_t s = P->stream;
  R.n_in_work2 = (int64_t)inw2.size() / 4;
  if (!inw2.empty()) {
    R.in_work2.alloc(inw2.size() * sizeof(int));
    GP_HIP(hipMemcpyAsync(R.in_work2.p, inw2.data(), inw2.size() * sizeof(int), hipMemcpyHostToDevice, s));
  }
  R.n_sp_work = (int64_t)spw.size() / 4;
  R.n_sp_red = (int64_t)spr.size() / 4;
  R.n_in_work = (int64_t)inw.size() / 4;
  R.n_slots = slots;
  R.sp_work.alloc(spw.size() * sizeof(int));
  GP_HIP(hipMemcpyAsync(R.sp_work.p, spw.data(), spw.size() * sizeof(int), hipMemcpyHostToDevice, s));
  if (!spr.empty()) {
    R.sp_red.alloc(spr.size() * sizeof(int));
    GP_HIP(hipMemcpyAsync(R.sp_red.p, spr.data(), spr.size() * sizeof(int), hipMemcpyHostToDevice, s));
    const int64_t tcells = (int64_t)P->tile[0] * P->tile[1] * P->tile[2];
    R.part.alloc((size_t)slots * tcells * slot_pairs(P) * cs);
  }
  if (!inw.empty()) {
    R.in_work.alloc(inw.size() * sizeof(int));
    GP_HIP(hipMemcpyAsync(R.in_work.p, inw.data(), inw.size() * sizeof(int), hipMemcpyHostToDevice, s));
  }
  // the host vectors are released when this returns: wait for the copies
  GP_HIP(hipStreamSynchronize(s));
}

void build_records_into(Plan* P, int64_t n, const double* pts, const double* sig,
                        const double* l, Records& R, int* out_of_box) {
  hipStream_t s = P->stream;
  const int d = P->d;
  RecArgs a;
  a.d = d;
  a.n = n;
  for (int r = 0; r < 3; ++r) {
    a.center[r] = P->center[r];
    a.nf[r] = P->nf[r];
    a.lo[r] = P->lo[r];
    a.tile[r] = P->tile[r];
    a.nbins[r] = P->nbins[r];
    a.na[r] = P->na[r];
  }
  a.scale = P->scale;
  a.dw = P->dw;
  a.w = P->w;
  const size_t tsz = P->precision == GP_FP64 ? sizeof(double) : sizeof(float);
  DevBuf bin_of, posd, cell_tmp, frac_tmp, sp_tmp, pf_tmp, bad;
  bin_of.alloc(n * sizeof(int));
  posd.alloc(n * sizeof(int));
  cell_tmp.alloc(n * d * sizeof(int));
  frac_tmp.alloc(n * d * sizeof(double));
  sp_tmp.alloc(n * sizeof(double));
  pf_tmp.alloc(n * sizeof(double));
  bad.alloc(sizeof(int));
  GP_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
  const int bs = 256;
  const unsigned nb = (unsigned)((n + bs - 1) / bs);
  hipLaunchKernelGGL(records_kernel, dim3(nb), dim3(bs), 0, s, a, pts, sig, l, bin_of.as<int>(),
                     cell_tmp.as<int>(), frac_tmp.as<double>(), sp_tmp.as<double>(),
                     pf_tmp.as<double>(), bad.as<int>());
  GP_CHECK_LAUNCH();
  // Stable counting sort by tile on the host (plan time): points keep their
  // caller order inside a tile, so every plan of the same input is identical.
  std::vector<int> hb(n);
  int hbad = 0;
  GP_HIP(hipMemcpyAsync(hb.data(), bin_of.p, n * sizeof(int), hipMemcpyDeviceToHost, s));
  GP_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  GP_HIP(hipStreamSynchronize(s));
  if (out_of_box) *out_of_box = hbad;
  std::vector<int> start(P->n_bins + 1, 0);
  for (int64_t i = 0; i < n; ++i) start[hb[i] + 1] += 1;
  for (int64_t b = 0; b < P->n_bins; ++b) start[b + 1] += start[b];
  std::vector<int> fill(start.begin(), start.end() - 1), hpos(n);
  for (int64_t i = 0; i < n; ++i) hpos[i] = fill[hb[i]]++;
  R.n = n;
  R.rs = d * P->w + P->nkp;
  R.perm.alloc(n * sizeof(int));
  R.cell.alloc(n * d * sizeof(int));
  R.pw.alloc((size_t)n * R.rs * tsz);
  R.bin_start.alloc((P->n_bins + 1) * sizeof(int));
  GP_HIP(hipMemcpyAsync(R.bin_start.p, start.data(), (P->n_bins + 1) * sizeof(int),
                        hipMemcpyHostToDevice, s));
  GP_HIP(hipMemcpyAsync(posd.p, hpos.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
  build_work_lists(P, R, start, P->precision == GP_FP64 ? 16 : 8);
#define GP_SCATTER(T)                                                                            \
  hipLaunchKernelGGL(scatter_records_kernel<T>, dim3(nb), dim3(bs), 0, s, d, n, P->w, P->beta, \
                     P->nk, P->nkp, R.rs, posd.as<int>(), cell_tmp.as<int>(),                  \
                     frac_tmp.as<double>(),                                                    \
                     sp_tmp.as<double>(), pf_tmp.as<double>(), P->nodes_d.as<double>(),        \
                     P->bary_d.as<double>(), R.perm.as<int>(), R.cell.as<int>(), R.pw.as<T>())
  if (P->precision == GP_FP64)
    GP_SCATTER(double);
  else
    GP_SCATTER(float);
#undef GP_SCATTER
  GP_CHECK_LAUNCH();
  GP_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------ build_plan ----

// The plan's numbers from the problem's ranges alone (no device data): the
// Chebyshev degree, t grid, Fourier spacing and half-width, window and
// oversampled grid, the active box and its tiles.  Needs P->d, nu, se,
// precision and scale (the box map) set; lmin, lmax in the caller's units.
void choose_params(Plan* P, int d, double nu, double tol, double lmin, double lmax,
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
    int tl = tile_d[d];
    int a0 = (int)std::floor(0.5 * nf - nf * P->dw - 0.5 * P->w) - 1;
    int a1 = (int)std::ceil(0.5 * nf + nf * P->dw + 0.5 * P->w) + 1;
    a0 = std::max(a0, 0);
    a1 = std::min(a1, nf - 1);
    int na = a1 - a0 + 1;
    na = ((na + tl - 1) / tl) * tl;
    if (a0 + na > nf) a0 = nf - na;
    if (a0 < 0) {
      // grid smaller than a tile multiple: shrink the tile
      tl = 1;
      while (tl * 2 <= nf && tl < tile_d[d]) tl *= 2;
      na = nf;
      a0 = 0;
      na = (na / tl) * tl;
    }
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
}

// Low-rank factors of the step-3 rows (rem:step3, last paragraph): row r of A
// (nk x nk, symmetric positive semidefinite, stored as the upper triangle of
// width nkp) is factored by pivoted Cholesky, A ~ sum_a R_a R_a', taking
// pivots while the largest remaining diagonal exceeds rel times the row's
// largest diagonal; the rank so revealed varies by row.  Output: rows[off[r]
// .. off[r+1]) holds rank_r vectors of nkp entries (R_a[k], zero for k >= nk).
// Rows are independent and are factored by several host threads.
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

int build_plan(int d, int64_t n, const double* pts, const double* sigma, const double* l,
               double nu, double eta, double tol, const gp_opts* opts_in, Plan* P,
               bool query_only, size_t* bytes_out) {
  gp_opts opts;
  if (opts_in)
    opts = *opts_in;
  else
    gp_opts_init(&opts);
  if (d < 1 || d > 3) throw Error{GP_EINVAL, "d must be 1, 2 or 3"};
  if (n < 1 || n > (int64_t)std::numeric_limits<int>::max() / 4)
    throw Error{GP_EINVAL, "n must be in [1, 2^29)"};
  if (!pts || !sigma || !l) throw Error{GP_EINVAL, "null input pointer"};
  if (!(nu > 0)) throw Error{GP_EDOMAIN, "nu must be > 0"};
  if (!(eta >= 0) || !std::isfinite(eta)) throw Error{GP_EDOMAIN, "eta must be finite and >= 0"};
  if (!(tol > 0) || !(tol < 1)) throw Error{GP_EDOMAIN, "tol must be in (0, 1)"};
  if (opts.precision != GP_FP64 && opts.precision != GP_FP32_BULK)
    throw Error{GP_EINVAL, "unknown precision"};

  P->d = d;
  P->n = n;
  P->precision = opts.precision;
  P->nu = nu;
  P->eta = eta;
  P->se = std::isinf(nu);
  P->stream = static_cast<hipStream_t>(opts.stream);
  GP_HIP(hipGetDevice(&P->device));
  hipStream_t s = P->stream;

  // ---- host copies for validation and ranges
  std::vector<double> hx(n * d), hs(n), hl(n);
  GP_HIP(hipMemcpyAsync(hx.data(), pts, n * d * sizeof(double), hipMemcpyDeviceToHost, s));
  GP_HIP(hipMemcpyAsync(hs.data(), sigma, n * sizeof(double), hipMemcpyDeviceToHost, s));
  GP_HIP(hipMemcpyAsync(hl.data(), l, n * sizeof(double), hipMemcpyDeviceToHost, s));
  GP_HIP(hipStreamSynchronize(s));
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int r = 0; r < d; ++r) {
    lo[r] = std::numeric_limits<double>::infinity();
    hi[r] = -lo[r];
  }
  double lmin = std::numeric_limits<double>::infinity(), lmax = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int r = 0; r < d; ++r) {
      double v = hx[i * d + r];
      if (!std::isfinite(v)) throw Error{GP_EDOMAIN, "non-finite point coordinate"};
      lo[r] = std::min(lo[r], v);
      hi[r] = std::max(hi[r], v);
    }
    if (!(hs[i] > 0) || !std::isfinite(hs[i])) throw Error{GP_EDOMAIN, "sigma must be finite and > 0"};
    if (!(hl[i] > 0) || !std::isfinite(hl[i])) throw Error{GP_EDOMAIN, "l must be finite and > 0"};
    lmin = std::min(lmin, hl[i]);
    lmax = std::max(lmax, hl[i]);
  }
  if (opts.use_box) {
    for (int r = 0; r < d; ++r) {
      if (!(opts.box_lo[r] <= lo[r] && opts.box_hi[r] >= hi[r]))
        throw Error{GP_ERANGE, "points outside gp_opts box"};
      lo[r] = opts.box_lo[r];
      hi[r] = opts.box_hi[r];
    }
  }
  if (opts.l_lo > 0) lmin = std::min(lmin, opts.l_lo);
  if (opts.l_hi > 0) lmax = std::max(lmax, opts.l_hi);

  // ---- isotropic map onto [-1,1]^d (section 5 assumes the points lie there)
  double ext = 0;
  for (int r = 0; r < d; ++r) {
    P->center[r] = 0.5 * (lo[r] + hi[r]);
    ext = std::max(ext, hi[r] - lo[r]);
  }
  if (!(ext > 0)) ext = 2.0;
  P->scale = 2.0 / ext;
  P->l_range_lo = lmin;
  P->l_range_hi = lmax;

  choose_params(P, d, nu, tol, lmin, lmax, opts);
  const int nf = P->nf[0];
  const double smin = P->s_min, smax = P->s_max;
  P->nk = P->n_sigma + 1;
  P->npair = (P->nk + 1) / 2;

  // ---- step 3 variant; radial rows of the precomputed tensor
  if (opts.step3 < 0 || opts.step3 > 2) throw Error{GP_EINVAL, "opts.step3 must be 0, 1 or 2"};
  P->step3 = opts.step3;
  if (opts.spread < 0 || opts.spread > 2) throw Error{GP_EINVAL, "opts.spread must be 0, 1 or 2"};
  P->spread_mode = opts.spread != GP_SPREAD_AUTO ? opts.spread : GP_SPREAD_OWNER;
  if (opts.interp < 0 || opts.interp > 2) throw Error{GP_EINVAL, "opts.interp must be 0, 1 or 2"};
  P->interp_mode = opts.interp;
  P->nkp = P->nk + (P->nk & 1);
  std::vector<double> svals;
  std::vector<int> rowmap;
  if (P->step3 != 1) {
    const int64_t M = P->M;
    if (d == 1) {
      svals.resize(M + 1);
      for (int64_t m = 0; m <= M; ++m) svals[m] = (double)(m * m);
    } else {
      const int64_t smax = (int64_t)d * M * M;
      std::vector<char> present(smax + 1, 0);
      if (d == 2) {
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
    P->a_rows = (int64_t)svals.size();
  }

  // ---- memory
  const size_t cs = P->precision == GP_FP64 ? 16 : 8;  // complex element
  const size_t ts = cs / 2;
  int64_t szA = 1, szB = 1, szB2 = 0, szC = 1;
  const int64_t mc = P->mcount;
  if (d == 1) {
    szA = P->fourstep ? nf : P->na[0];
    szB = P->fourstep ? nf : mc;
    szC = P->fourstep ? nf : mc;
  } else if (d == 2) {
    szA = (int64_t)P->na[0] * P->na[1];
    szB = (int64_t)P->na[1] * mc;
    szC = mc * mc;
  } else {
    szA = (int64_t)P->na[0] * P->na[1] * P->na[2];
    szB = (int64_t)P->na[2] * P->na[1] * mc;
    szB2 = (int64_t)P->na[2] * mc * mc;
    szC = mc * mc * mc;
  }
  const int64_t G = P->npair;
  size_t bytes = 0;
  bytes += (size_t)G * (szA + szB + szB2 + szC) * cs;
  bytes += (size_t)n * (sizeof(int) * (1 + d) + ts * (d * P->w + P->nk + 1));
  bytes += (size_t)(P->n_bins + 1) * sizeof(int);
  bytes += work_list_bound_bytes(P, n, cs);
  if (P->step3 != 1)  // the low-rank rows (step3 = 2) hold at most the full row's size
    bytes += (size_t)P->a_rows * (P->nkp * (P->nkp + 1) / 2) * ts + rowmap.size() * sizeof(int) +
             (P->step3 == 2 ? (size_t)(P->a_rows + 1) * sizeof(int64_t) : 0);
  else
    bytes += (size_t)P->nt_eff * P->nk * (P->M + 1) * ts * 2;
  bytes += (size_t)n * 8 * sizeof(double) + (kCgBlocks + kCgScalars) * sizeof(double);  // vectors
  bytes += (size_t)nf * cs * 2;
  P->device_bytes = bytes;
  if (bytes_out) *bytes_out = bytes;
  if (query_only) return GP_OK;
  if (opts.max_device_bytes > 0 && bytes > opts.max_device_bytes)
    throw Error{GP_ENOMEM, "plan needs " + std::to_string(bytes) + " device bytes, over the limit"};

  // ---- host tables: sigma nodes, barycentric weights, t grid
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
  const int nt_paper = P->se ? 1 : P->n_t + 1;
  P->vt.resize(nt_paper);
  P->chi.resize(nt_paper);
  const double dwd = std::pow(P->dw, d);
  if (P->se) {
    P->vt[0] = dwd;
    P->chi[0] = 1.0;
  } else {
    const double dt = (P->t_max - P->t_min) / P->n_t, lg = std::lgamma(nu);
    for (int j = 0; j <= P->n_t; ++j) {
      double t = P->t_min + (double)j / P->n_t * (P->t_max - P->t_min);
      double u = std::exp(nu * t - std::exp(t) - lg);          // eq:maternpres
      double ch = std::exp(0.5 * t) / std::sqrt(nu);
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
  std::vector<double> tvt(P->nt_eff), tcst((size_t)P->nt_eff * P->nk), ttau((size_t)P->nt_eff * P->nk);
  {
    int jt = 0;
    if (P->n_flat > 0) {
      double W = 0.0;
      for (int j = 0; j < P->n_flat; ++j) W += P->vt[j] * std::pow(2 * PI * P->chi[j] * P->chi[j], (double)d);
      tvt[0] = W;
      for (int k = 0; k < P->nk; ++k) {
        tcst[k] = std::pow(P->sig_nodes[k], (double)d);
        ttau[k] = 0.0;
      }
      jt = 1;
    }
    for (int j = P->n_flat; j < nt_paper; ++j, ++jt) {
      tvt[jt] = P->vt[j];
      for (int k = 0; k < P->nk; ++k) {
        const double s2 = P->sig_nodes[k] * P->sig_nodes[k] * P->chi[j] * P->chi[j];
        tcst[(size_t)jt * P->nk + k] = std::pow(2 * PI * s2, 0.5 * d);
        ttau[(size_t)jt * P->nk + k] = 2 * PI * PI * s2 * P->dw * P->dw;
      }
    }
    if (jt != P->nt_eff) throw Error{GP_EDEVICE, "internal: t node count"};
  }

  // Fourier multipliers of G_{k,t_j} (eq:Gkt) on the grid, separated by
  // dimension: G^_{kj}[n] = C_kj prod_r exp(-tau_kj n_r^2), C_kj = (2 pi s^2)^(d/2),
  // tau_kj = 2 pi^2 s^2 dw^2, s = sigma_k chi_j.  gtab carries the constant and
  // dimension 0, etab the rest.
  const int64_t M1 = P->M + 1;
  std::vector<double> g0((size_t)P->nt_eff * P->nk * M1), e1((size_t)P->nt_eff * P->nk * M1);
  for (int j = 0; j < P->nt_eff; ++j)
    for (int k = 0; k < P->nk; ++k) {
      const double cst = tcst[(size_t)j * P->nk + k];
      const double tau = ttau[(size_t)j * P->nk + k];
      for (int64_t m = 0; m < M1; ++m) {
        double e = std::exp(-tau * (double)m * (double)m);
        g0[((size_t)j * P->nk + k) * M1 + m] = cst * e;
        e1[((size_t)j * P->nk + k) * M1 + m] = e;
      }
    }
  // deconvolution 1/psi^(2 pi n / nf) of the window (Appendix D NUFFTs)
  std::vector<double> gx, gw;
  gauss_legendre(120 + 8 * P->w, gx, gw);
  std::vector<double> dec((size_t)d * M1);
  for (int r = 0; r < d; ++r)
    for (int64_t m = 0; m < M1; ++m)
      dec[r * M1 + m] = 1.0 / es_hat(2 * PI * (double)m / P->nf[r], P->w, P->beta, gx, gw);

  auto upload = [&](DevBuf& buf, const std::vector<double>& v) {
    if (P->precision == GP_FP64) {
      buf.alloc(v.size() * sizeof(double));
      GP_HIP(hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, s));
      GP_HIP(hipStreamSynchronize(s));
    } else {
      std::vector<float> f(v.begin(), v.end());
      buf.alloc(f.size() * sizeof(float));
      GP_HIP(hipMemcpyAsync(buf.p, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, s));
      GP_HIP(hipStreamSynchronize(s));
    }
  };
  if (P->step3 == 1) {
    upload(P->gtab, g0);
    upload(P->etab, e1);
  } else {
    // precomputed tensor, one row per distinct |n|^2
    const std::vector<double>& tau = ttau;
    const std::vector<double>& cst = tcst;
    DevBuf dsv, dtau, dcst, dvt;
    auto up64 = [&](DevBuf& b, const std::vector<double>& v) {
      b.alloc(v.size() * sizeof(double));
      GP_HIP(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, s));
    };
    up64(dsv, svals);
    up64(dtau, tau);
    up64(dcst, cst);
    up64(dvt, tvt);
    const int npk = P->nkp * (P->nkp + 1) / 2;
    const int64_t tot = P->a_rows * npk;
    const unsigned nb = (unsigned)((tot + 255) / 256);
    if (P->step3 == 0) {
      P->atab.alloc((size_t)tot * ts);
      if (P->precision == GP_FP64)
        hipLaunchKernelGGL(atab_kernel<double>, dim3(nb), dim3(256), 0, s, P->a_rows, npk, P->nkp,
                           P->nk, P->nt_eff, dsv.as<double>(), dtau.as<double>(), dcst.as<double>(),
                           dvt.as<double>(), P->atab.as<double>());
      else
        hipLaunchKernelGGL(atab_kernel<float>, dim3(nb), dim3(256), 0, s, P->a_rows, npk, P->nkp,
                           P->nk, P->nt_eff, dsv.as<double>(), dtau.as<double>(), dcst.as<double>(),
                           dvt.as<double>(), P->atab.as<float>());
      GP_CHECK_LAUNCH();
    } else {
      // low-rank form of rem:step3 (last paragraph): the fp64 rows, factored
      // on the host row by row as A ~ R' R by pivoted Cholesky, keeping the
      // factors whose pivots exceed tol/100 of the row's largest diagonal
      DevBuf full;
      full.alloc((size_t)tot * sizeof(double));
      hipLaunchKernelGGL(atab_kernel<double>, dim3(nb), dim3(256), 0, s, P->a_rows, npk, P->nkp,
                         P->nk, P->nt_eff, dsv.as<double>(), dtau.as<double>(), dcst.as<double>(),
                         dvt.as<double>(), full.as<double>());
      GP_CHECK_LAUNCH();
      std::vector<double> hA((size_t)tot);
      GP_HIP(hipMemcpyAsync(hA.data(), full.p, hA.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      GP_HIP(hipStreamSynchronize(s));
      std::vector<int64_t> off;
      std::vector<double> rows;
      lowrank_rows(P->a_rows, P->nk, P->nkp, hA, 1e-2 * tol, off, rows, &P->lr_rank_max,
                   &P->lr_rank_mean);
      P->lr_off.alloc(off.size() * sizeof(int64_t));
      GP_HIP(hipMemcpyAsync(P->lr_off.p, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
      upload(P->atab, rows);
    }
    if (d > 1) {
      P->rowidx.alloc(rowmap.size() * sizeof(int));
      GP_HIP(hipMemcpyAsync(P->rowidx.p, rowmap.data(), rowmap.size() * sizeof(int),
                            hipMemcpyHostToDevice, s));
    }
    GP_HIP(hipStreamSynchronize(s));
  }
  upload(P->vtd, tvt);
  upload(P->dec, dec);
  P->nodes_d.alloc(P->nk * sizeof(double));
  P->bary_d.alloc(P->nk * sizeof(double));
  GP_HIP(hipMemcpyAsync(P->nodes_d.p, P->sig_nodes.data(), P->nk * sizeof(double), hipMemcpyHostToDevice, s));
  GP_HIP(hipMemcpyAsync(P->bary_d.p, P->bary.data(), P->nk * sizeof(double), hipMemcpyHostToDevice, s));

  // FFT twiddles exp(-2 pi i k / L) for the pass lengths in use
  auto twiddles = [&](DevBuf& buf, int L) {
    std::vector<double> t(2 * (size_t)L);
    for (int k = 0; k < L; ++k) {
      long double a = -2.0L * 3.14159265358979323846264338327950288L * k / L;
      t[2 * k] = (double)cosl(a);
      t[2 * k + 1] = (double)sinl(a);
    }
    upload(buf, t);
  };
  if (P->fourstep) {
    twiddles(P->tw[0], P->L1);
    twiddles(P->tw[1], P->L2);
    twiddles(P->tw4, nf);
  } else {
    twiddles(P->tw[0], nf);
  }

  // ---- points: records and bin sort
  int oob = 0;
  build_records_into(P, n, pts, sigma, l, P->rec, &oob);
  if (oob) throw Error{GP_EDEVICE, "internal: a point's window left the active grid"};

  // ---- grids and vectors
  P->gridA.alloc((size_t)G * szA * cs);
  P->gridB.alloc((size_t)G * szB * cs);
  if (szB2) P->gridB2.alloc((size_t)G * szB2 * cs);
  P->gridC.alloc((size_t)G * szC * cs);
  if (P->fourstep) GP_HIP(hipMemsetAsync(P->gridA.p, 0, P->gridA.bytes, s));
  P->grid_elems[0] = szA;
  P->grid_elems[1] = szB;
  P->grid_elems[2] = szB2;
  P->grid_elems[3] = szC;
  P->gv.A = P->gridA.p;
  P->gv.B = P->gridB.p;
  P->gv.B2 = P->gridB2.p;
  P->gv.C = P->gridC.p;
  P->gv.nsets = 1;
  P->gv.cur = 0;
  P->vec.alloc((size_t)n * 8 * sizeof(double));
  P->cg_part.alloc(kCgBlocks * sizeof(double));
  P->cg_S.alloc(kCgScalars * sizeof(double));
  GP_HIP(hipHostMalloc((void**)&P->cg_hS, kCgScalars * sizeof(double), hipHostMallocDefault));
  GP_HIP(hipStreamSynchronize(s));
  return GP_OK;
}

}  // namespace gp
