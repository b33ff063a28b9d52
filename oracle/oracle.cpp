// Plain CPU oracle for the non-stationary Matern GPR matvec and solve.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// CPU-baseline leg of the benchmark may load this library.  The product path
// never calls it and shares no code with it.
//
// Everything here is fp64 and written for clarity, not speed: every function
// follows one formula of Kielstra & Lindsey, "Gaussian process regression with
// log-linear scaling for common non-stationary kernels" (arXiv 2407.03608),
// cited by section / equation / lemma label.
//
// Two results are computed:
//   O1 - the exact kernel matrix K of eq:nonstat2 (section 3), its matvec and
//        a Cholesky solve of (K + eta^2 I) alpha = y  (eq:gprsolve).
//   O2 - the approximate operator K~ of eq:Ktilde (section 3.5), applied by
//        direct non-uniform DFTs (Appendix D definitions, no window, no FFT)
//        in the order of the five steps of section 4.2, and K~ entries formed
//        a second way from per-dimension theta sums (small N only).
//
// User-level parameterisation (a reading; the paper absorbs the amplitude into
// w(x)): the caller gives a vertical scale sig(x) and a length scale l(x).  With
//   sigma_p(x) = l(x)/sqrt(2),  w(x) = sig(x) * (sqrt(2 pi) l(x))^(d/2)
// eq:nonstat2 becomes the Paciorek-Schervish normalised kernel, for which
// K(x,x) = sig(x)^2 and constant sig, l give sig^2 phi_nu(|x-y|/l).

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

typedef std::complex<double> cplx;

static const double PI = 3.14159265358979323846264338327950288;

extern "C" {

// ---------------------------------------------------------------- phi_nu ----

// Matern function of eq:matern in its Bessel form, 2^(1-nu)/Gamma(nu) z^nu K_nu(z)
// with z = sqrt(2 nu) r; phi(0) = 1.  std::cyl_bessel_k is the library routine.
double orc_matern_bessel(double nu, double r) {
  if (r == 0.0) return 1.0;
  double z = std::sqrt(2.0 * nu) * std::fabs(r);
  double lg = std::lgamma(nu);
  return std::exp((1.0 - nu) * std::log(2.0) - lg + nu * std::log(z)) * std::cyl_bessel_k(nu, z);
}

// phi_nu with the closed forms for half-integer nu (section 2, the remark after
// eq:matern) and the squared exponential eq:squaredexp for nu = +inf.
double orc_matern(double nu, double r) {
  r = std::fabs(r);
  if (std::isinf(nu)) return std::exp(-0.5 * r * r);
  if (nu == 0.5) return std::exp(-r);
  if (nu == 1.5) {
    double a = std::sqrt(3.0) * r;
    return (1.0 + a) * std::exp(-a);
  }
  if (nu == 2.5) {
    double a = std::sqrt(5.0) * r;
    return (1.0 + a + 5.0 * r * r / 3.0) * std::exp(-a);
  }
  return orc_matern_bessel(nu, r);
}

// Schoenberg representation eq:schoenberg2 with the Matern data of
// eq:maternpres, u(t) = e^(nu t - e^t)/Gamma(nu), chi(t) = e^(t/2)/sqrt(nu),
// integrated by the trapezoid rule of eq:trapsum/eq:dtscheme on [tmin,tmax].
double orc_matern_schoenberg(double nu, double r, double tmin, double tmax, int nt) {
  double dt = (tmax - tmin) / nt;
  double s = 0.0;
  for (int j = 0; j <= nt; ++j) {
    double t = tmin + j * dt;
    double u = std::exp(nu * t - std::exp(t) - std::lgamma(nu));
    double chi2 = std::exp(t) / nu;
    double f = std::exp(-r * r / (2.0 * chi2)) * u;
    s += (j == 0 || j == nt) ? 0.5 * f * dt : f * dt;
  }
  return s;
}

// ------------------------------------------------------- exact kernel O1 ----

// K(x,y) of eq:nonstat2 with sigma_p = l/sqrt(2), w = sig (sqrt(2 pi) l)^(d/2).
double orc_kernel(int d, const double* x, double sx, double lx, const double* y, double sy,
                  double ly, double nu) {
  double spx2 = 0.5 * lx * lx, spy2 = 0.5 * ly * ly;  // sigma_p^2
  double wx = sx * std::pow(std::sqrt(2.0 * PI) * lx, 0.5 * d);
  double wy = sy * std::pow(std::sqrt(2.0 * PI) * ly, 0.5 * d);
  double r2 = 0.0;
  for (int a = 0; a < d; ++a) r2 += (x[a] - y[a]) * (x[a] - y[a]);
  double ssum = spx2 + spy2;
  return wx * wy * std::pow(2.0 * PI * ssum, -0.5 * d) * orc_matern(nu, std::sqrt(r2 / ssum));
}

// Dense block K[i*nc + j] = K(xr_i, xc_j)   (eq:boldK).
void orc_kernel_block(int d, int64_t nr, const double* xr, const double* sr, const double* lr,
                      int64_t nc, const double* xc, const double* sc, const double* lc, double nu,
                      double* K) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < nr; ++i)
    for (int64_t j = 0; j < nc; ++j)
      K[i * nc + j] = orc_kernel(d, xr + i * d, sr[i], lr[i], xc + j * d, sc[j], lc[j], nu);
}

// Rows r0..r1-1 of K alpha, rows formed on the fly, Kahan-compensated sums.
void orc_exact_matvec_rows(int d, int64_t n, const double* x, const double* s, const double* l,
                           double nu, const double* alpha, int64_t r0, int64_t r1, double* out) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = r0; i < r1; ++i) {
    double sum = 0.0, c = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      double term = orc_kernel(d, x + i * d, s[i], l[i], x + j * d, s[j], l[j], nu) * alpha[j];
      double yv = term - c;
      double t = sum + yv;
      c = (t - sum) - yv;
      sum = t;
    }
    out[i - r0] = sum;
  }
}

// In-place Cholesky A = L L^T of a dense symmetric positive definite n x n
// matrix (row-major, lower triangle used and overwritten).  Returns 0, or
// -(j+1) if the pivot of column j is not positive.
int orc_cholesky(int64_t n, double* A) {
  for (int64_t j = 0; j < n; ++j) {
    double djj = A[j * n + j];
    for (int64_t k = 0; k < j; ++k) djj -= A[j * n + k] * A[j * n + k];
    if (!(djj > 0.0)) return (int)(-(j + 1));
    double ljj = std::sqrt(djj);
    A[j * n + j] = ljj;
#pragma omp parallel for schedule(static)
    for (int64_t i = j + 1; i < n; ++i) {
      double v = A[i * n + j];
      for (int64_t k = 0; k < j; ++k) v -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = v / ljj;
    }
  }
  return 0;
}

// Solve L L^T x = b by forward then backward substitution.
void orc_chol_solve(int64_t n, const double* L, const double* b, double* x) {
  std::vector<double> z(n);
  for (int64_t i = 0; i < n; ++i) {
    double v = b[i];
    for (int64_t k = 0; k < i; ++k) v -= L[i * n + k] * z[k];
    z[i] = v / L[i * n + i];
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    double v = z[i];
    for (int64_t k = i + 1; k < n; ++k) v -= L[k * n + i] * x[k];
    x[i] = v / L[i * n + i];
  }
}

// ------------------------------------------------ approximate operator O2 ----

// The parameters that define K~ (section 3.5): t_min, t_max, N_t, the sigma
// range and N_sigma, Delta-omega and M, plus the affine map of the points into
// [-1,1]^d assumed by section 5 (x' = (x - center) * scale, l' = l * scale).
// nu = +inf selects the squared exponential (N_t = 0, v_0 = 1, chi = 1).
typedef struct {
  int d;
  double nu;
  double t_min, t_max;
  int n_t;
  double s_min, s_max;
  int n_sigma;
  double dw;
  int64_t M;
  double center[3];
  double scale;
} orc_plan;

static bool is_se(const orc_plan* p) { return std::isinf(p->nu); }

// t nodes of eq:dtscheme and the trapezoid weights v_j of eq:trapsum with
// v(t) = chi(t)^(-d) u(t) (eq:v) and Matern u, chi of eq:maternpres; the
// scaled weights v~_j = (Delta omega)^d v_j of section 3.5.  Squared exponential:
// t_0 = 0, v_0 = 1, chi_0 = 1 (section 3.2).
void orc_tgrid(const orc_plan* p, double* t, double* vtilde, double* chi) {
  double dwd = std::pow(p->dw, p->d);
  if (is_se(p)) {
    t[0] = 0.0;
    chi[0] = 1.0;
    vtilde[0] = dwd;
    return;
  }
  double nu = p->nu;
  double dt = (p->t_max - p->t_min) / p->n_t;
  for (int j = 0; j <= p->n_t; ++j) {
    double tj = p->t_min + (double)j / p->n_t * (p->t_max - p->t_min);
    double u = std::exp(nu * tj - std::exp(tj) - std::lgamma(nu));
    double ch = std::exp(0.5 * tj) / std::sqrt(nu);
    double v = std::pow(ch, -(double)p->d) * u;
    double vj = (j == 0 || j == p->n_t) ? v * dt * 0.5 : v * dt;
    t[j] = tj;
    chi[j] = ch;
    vtilde[j] = dwd * vj;
  }
}

// Chebyshev-Lobatto nodes of eq:chebscheme (k = 0 is sigma_max).  N_sigma = 0
// is the stationary case sigma_min = sigma_max with the single node sigma_min.
void orc_sigma_nodes(const orc_plan* p, double* sk) {
  if (p->n_sigma == 0) {
    sk[0] = p->s_min;
    return;
  }
  for (int k = 0; k <= p->n_sigma; ++k)
    sk[k] = 0.5 * (std::cos(PI * k / p->n_sigma) + 1.0) * (p->s_max - p->s_min) + p->s_min;
}

// Lagrange basis P_k(s) on the nodes sk (section 3.3), by the product formula.
void orc_lagrange(int nsig, const double* sk, double s, double* P) {
  for (int k = 0; k <= nsig; ++k) {
    double v = 1.0;
    for (int m = 0; m <= nsig; ++m)
      if (m != k) v *= (s - sk[m]) / (sk[k] - sk[m]);
    P[k] = v;
  }
}

// Per-point weights w_k(x_i) of eq:Wk: w(x)(2 pi sigma_p(x)^2)^(-d/2) P_k(sigma_p(x)),
// with sigma_p = l'/sqrt(2) and w = sig (sqrt(2 pi) l')^(d/2) in the mapped
// coordinates.  Output wk[i*(nsig+1) + k].
void orc_weights(const orc_plan* p, int64_t n, const double* sig, const double* l, double* wk) {
  int ns = p->n_sigma + 1;
  std::vector<double> sk(ns);
  orc_sigma_nodes(p, sk.data());
  for (int64_t i = 0; i < n; ++i) {
    double lp = l[i] * p->scale;
    double sp = lp / std::sqrt(2.0);
    double w = sig[i] * std::pow(std::sqrt(2.0 * PI) * lp, 0.5 * p->d);
    double pre = w * std::pow(2.0 * PI * sp * sp, -0.5 * p->d);
    std::vector<double> P(ns);
    orc_lagrange(p->n_sigma, sk.data(), sp, P.data());
    for (int k = 0; k < ns; ++k) wk[i * ns + k] = pre * P[k];
  }
}

// Fourier multiplier of the Gaussian convolution G_{k,t} (eq:Gkt) on the grid
// point n Delta-omega: the transform of exp(-|z|^2/(2 s^2)) with s = sigma_k chi_j
// is (sqrt(2 pi) s)^d exp(-(2 pi s)^2 |omega|^2 / 2)  (proof of lemma stage3warmup).
static double ghat(int d, double sk, double chij, double dw, double n2) {
  double s2 = sk * sk * chij * chij;
  return std::pow(2.0 * PI * s2, 0.5 * d) * std::exp(-2.0 * PI * PI * s2 * dw * dw * n2);
}

// Map the points into the analysis box (section 5): x' = (x - center) * scale.
static std::vector<double> mapped(const orc_plan* p, int64_t n, const double* x) {
  std::vector<double> xp(n * p->d);
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < p->d; ++a) xp[i * p->d + a] = (x[i * p->d + a] - p->center[a]) * p->scale;
  return xp;
}

// Number of Fourier grid points (2M+1)^d and the multi-index of a flat index.
static int64_t n_modes(const orc_plan* p) {
  int64_t m = 1;
  for (int a = 0; a < p->d; ++a) m *= (2 * p->M + 1);
  return m;
}
static void mode_index(const orc_plan* p, int64_t f, int64_t* nv) {
  for (int a = 0; a < p->d; ++a) {
    nv[a] = f % (2 * p->M + 1) - p->M;
    f /= (2 * p->M + 1);
  }
}

// out = K~ alpha by the five steps of section 4.2, every NUFFT replaced by its
// defining sum (Appendix D):
//   (1) c_{k,i} = w_k(x_i) alpha_i                               eq:c
//   (2) b_k[n]  = sum_i c_{k,i} exp(-2 pi i (n dw).x_i)          type 1
//   (3) a_k'[n] = sum_j v~_j G^_{k'j}[n] sum_k G^_{kj}[n] b_k[n]
//   (4) beta_{k,i} = sum_n a_k[n] exp(+2 pi i (n dw).x_i)        type 2
//   (5) out_i  = sum_k w_k(x_i) beta_{k,i}   (real part)
// The factor exp(-2 pi i n.x) is formed as the product of its d one-dimensional
// factors, tabulated per point and per dimension.
int orc_ktilde_matvec(const orc_plan* p, int64_t n, const double* x, const double* sig,
                      const double* l, const double* alpha, double* out) {
  const int d = p->d;
  const int ns = p->n_sigma + 1;
  const int nt = is_se(p) ? 1 : p->n_t + 1;
  const int64_t L = 2 * p->M + 1;
  const int64_t NM = n_modes(p);
  std::vector<double> xp = mapped(p, n, x);
  std::vector<double> wk(n * ns);
  orc_weights(p, n, sig, l, wk.data());
  std::vector<double> t(nt), vt(nt), chi(nt), sk(ns);
  orc_tgrid(p, t.data(), vt.data(), chi.data());
  orc_sigma_nodes(p, sk.data());

  // phase tables e^{-2 pi i dw n x_{i,a}}, [i][a][n + M]
  std::vector<cplx> ph((size_t)n * d * L);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < d; ++a)
      for (int64_t m = 0; m < L; ++m) {
        double ang = -2.0 * PI * p->dw * (double)(m - p->M) * xp[i * d + a];
        ph[((size_t)i * d + a) * L + m] = cplx(std::cos(ang), std::sin(ang));
      }

  // (1)+(2): b[k][f]
  std::vector<cplx> b((size_t)ns * NM);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t f = 0; f < NM; ++f) {
    int64_t nv[3];
    mode_index(p, f, nv);
    std::vector<cplx> acc(ns, cplx(0.0, 0.0));
    for (int64_t i = 0; i < n; ++i) {
      cplx e(1.0, 0.0);
      for (int a = 0; a < d; ++a) e *= ph[((size_t)i * d + a) * L + (nv[a] + p->M)];
      for (int k = 0; k < ns; ++k) acc[k] += (wk[i * ns + k] * alpha[i]) * e;
    }
    for (int k = 0; k < ns; ++k) b[(size_t)k * NM + f] = acc[k];
  }

  // (3): a[k'][f]
  std::vector<cplx> am((size_t)ns * NM);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t f = 0; f < NM; ++f) {
    int64_t nv[3];
    mode_index(p, f, nv);
    double n2 = 0.0;
    for (int a = 0; a < d; ++a) n2 += (double)nv[a] * (double)nv[a];
    std::vector<cplx> acc(ns, cplx(0.0, 0.0));
    std::vector<double> g(ns);
    for (int j = 0; j < nt; ++j) {
      cplx s(0.0, 0.0);
      for (int k = 0; k < ns; ++k) {
        g[k] = ghat(d, sk[k], chi[j], p->dw, n2);
        s += g[k] * b[(size_t)k * NM + f];
      }
      for (int k = 0; k < ns; ++k) acc[k] += vt[j] * g[k] * s;
    }
    for (int k = 0; k < ns; ++k) am[(size_t)k * NM + f] = acc[k];
  }

  // (4)+(5)
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < n; ++i) {
    std::vector<cplx> beta(ns, cplx(0.0, 0.0));
    for (int64_t f = 0; f < NM; ++f) {
      int64_t nv[3];
      mode_index(p, f, nv);
      cplx e(1.0, 0.0);
      for (int a = 0; a < d; ++a) e *= std::conj(ph[((size_t)i * d + a) * L + (nv[a] + p->M)]);
      for (int k = 0; k < ns; ++k) beta[k] += am[(size_t)k * NM + f] * e;
    }
    double o = 0.0;
    for (int k = 0; k < ns; ++k) o += wk[i * ns + k] * beta[k].real();
    out[i] = o;
  }
  return 0;
}

// K~(x, y) formed a second way.  Inserting eq:BWG into eq:Ktilde gives
//   K~(x,y) = sum_{k',k} w_k'(x) w_k(y) sum_j v~_j sum_{n in G} G^_{k'j}[n] G^_{kj}[n] e^{2 pi i dw n.(x'-y')}
// and because G^ factorises over dimensions and G is a box, the n-sum is a
// product of d one-dimensional even (cosine) sums
//   S_a = sum_{m=-M..M} exp(-tau m^2) cos(2 pi dw m delta_a)
//       = 1 + 2 sum_{m=1..M} exp(-tau m^2) cos(2 pi dw m delta_a),
// tau = 2 pi^2 (s_k'^2 + s_k^2) chi_j^2 dw^2 (s = sigma_k chi_j as in ghat).
// The Gaussian factors exp(-tau m^2) depend only on (k', k, j) and m, and the
// cosines only on the pair of points, so both are tabulated once (the pairs
// k' <= k: the t-sum is symmetric in k', k).  Entries K[i*ny + j].
int orc_ktilde_entries(const orc_plan* p, int64_t nx, const double* x, const double* sx,
                       const double* lx, int64_t ny, const double* y, const double* sy,
                       const double* ly, double* K) {
  const int d = p->d;
  const int ns = p->n_sigma + 1;
  const int nt = is_se(p) ? 1 : p->n_t + 1;
  const int64_t M = p->M;
  std::vector<double> xp = mapped(p, nx, x), yp = mapped(p, ny, y);
  std::vector<double> wx(nx * ns), wy(ny * ns);
  orc_weights(p, nx, sx, lx, wx.data());
  orc_weights(p, ny, sy, ly, wy.data());
  std::vector<double> t(nt), vt(nt), chi(nt), sk(ns);
  orc_tgrid(p, t.data(), vt.data(), chi.data());
  orc_sigma_nodes(p, sk.data());
  // pair index q of (k', k), k' <= k, and its (k', k)
  std::vector<int> qa, qb;
  for (int kp = 0; kp < ns; ++kp)
    for (int k = kp; k < ns; ++k) {
      qa.push_back(kp);
      qb.push_back(k);
    }
  const int64_t nq = (int64_t)qa.size();
  // per (q, j): the constant (2 pi sa2)^(d/2) (2 pi sb2)^(d/2) v~_j and the
  // Gaussian factors exp(-tau m^2), m = 1..M
  std::vector<double> pref((size_t)nq * nt), gau((size_t)nq * nt * M);
#pragma omp parallel for schedule(static)
  for (int64_t qj = 0; qj < nq * nt; ++qj) {
    const int64_t q = qj / nt;
    const int j = (int)(qj % nt);
    const double sa2 = sk[qa[q]] * sk[qa[q]] * chi[j] * chi[j];
    const double sb2 = sk[qb[q]] * sk[qb[q]] * chi[j] * chi[j];
    pref[qj] = vt[j] * std::pow(2.0 * PI * sa2, 0.5 * d) * std::pow(2.0 * PI * sb2, 0.5 * d);
    const double tau = 2.0 * PI * PI * (sa2 + sb2) * p->dw * p->dw;
    for (int64_t m = 1; m <= M; ++m) gau[(size_t)qj * M + (m - 1)] = std::exp(-tau * (double)(m * m));
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < nx; ++i) {
    std::vector<double> cs((size_t)d * M);
    for (int64_t jj = 0; jj < ny; ++jj) {
      for (int a = 0; a < d; ++a) {
        const double delta = xp[i * d + a] - yp[jj * d + a];
        for (int64_t m = 1; m <= M; ++m)
          cs[(size_t)a * M + (m - 1)] = std::cos(2.0 * PI * p->dw * (double)m * delta);
      }
      double total = 0.0;
      for (int64_t q = 0; q < nq; ++q) {
        const int kp = qa[q], k = qb[q];
        double sum_t = 0.0;
        for (int j = 0; j < nt; ++j) {
          const double* g = &gau[((size_t)q * nt + j) * M];
          double prod = pref[q * nt + j];
          for (int a = 0; a < d; ++a) {
            const double* c = &cs[(size_t)a * M];
            double s1 = 0.0;
            for (int64_t m = 0; m < M; ++m) s1 += g[m] * c[m];
            prod *= 1.0 + 2.0 * s1;
          }
          sum_t += prod;
        }
        double wpair = wx[i * ns + kp] * wy[jj * ns + k];
        if (k != kp) wpair += wx[i * ns + k] * wy[jj * ns + kp];
        total += wpair * sum_t;
      }
      K[i * ny + jj] = total;
    }
  }
  return 0;
}

// Posterior mean eq:postmean with the exact kernel: mu(x*) = sum_n alpha_n K(x*, x_n).
void orc_posterior_mean(int d, int64_t n, const double* x, const double* s, const double* l,
                        double nu, const double* alpha, int64_t m, const double* xt,
                        const double* st, const double* lt, double* mu) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < m; ++i) {
    double sum = 0.0;
    for (int64_t j = 0; j < n; ++j)
      sum += orc_kernel(d, xt + i * d, st[i], lt[i], x + j * d, s[j], l[j], nu) * alpha[j];
    mu[i] = sum;
  }
}

// K~-based posterior mean at targets: the same five steps as orc_ktilde_matvec
// with step (4)-(5) evaluated at the targets (eq:postmean with K~).
int orc_ktilde_posterior(const orc_plan* p, int64_t n, const double* x, const double* sig,
                         const double* l, const double* alpha, int64_t m, const double* xt,
                         const double* st, const double* lt, double* mu) {
  // K~(x*, x_j) alpha_j summed over j equals the x* row of K~ times alpha; use
  // the entry formula, which is exact for any pair of points inside the box.
  std::vector<double> Kt((size_t)m * n);
  int rc = orc_ktilde_entries(p, m, xt, st, lt, n, x, sig, l, Kt.data());
  if (rc) return rc;
  for (int64_t i = 0; i < m; ++i) {
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) s += Kt[(size_t)i * n + j] * alpha[j];
    mu[i] = s;
  }
  return 0;
}

}  // extern "C"
