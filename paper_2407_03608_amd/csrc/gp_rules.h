// Host-side rules of a plan, in plain C++ (no HIP): the numbers of section 3.5
// chosen from the problem's ranges, the tables derived from them on the host,
// and the low-rank factorisation of the step-3 rows.  Nothing here touches a
// device, so the file also builds with a host compiler alone (the host
// sanitizer test compiles it with g++ under AddressSanitizer and UBSan).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gpnufft.h"

namespace gp {

struct Error {
  int code;
  std::string msg;
};

// Lengths the FFT pass kernel is compiled for (2^a and 3*2^a, 8 .. 8192).
bool fft_length_supported(int L);

// The plan's numbers (everything but device data).
struct PlanRules {
  // problem
  int d = 0;
  int precision = GP_FP64;
  double nu = 0;
  bool se = false;            // nu = inf: squared exponential
  // mapping into [-1,1]^d: x' = (x - center) scale
  double center[3] = {0, 0, 0};
  double scale = 1;
  // approximation parameters (section 3.5)
  double t_min = 0, t_max = 0;
  int n_t = 0;
  double s_min = 0, s_max = 0;
  int n_sigma = 0;
  double dw = 0;
  int64_t M = 0;
  double pred_tail = 0;
  int m_capped = 0;
  double l_range_lo = 0, l_range_hi = 0;  // admissible user length scales
  // spreading / FFT geometry
  double nufft_tol = 0;
  int w = 0;
  double beta = 0;
  double upsample = 2.0;
  int nf[3] = {1, 1, 1};
  int lo[3] = {0, 0, 0};
  int na[3] = {1, 1, 1};      // active-box length (multiple of tile)
  int tile[3] = {1, 1, 1};
  int nbins[3] = {1, 1, 1};
  int64_t n_bins = 1;
  int nsrc = 2;               // source bins per dimension that reach a tile
  int fourstep = 0;           // d = 1 and nf > 8192: nf = L1 * L2
  int L1 = 0, L2 = 0;
  int nk = 0;                 // real grids = N_sigma + 1
  int npair = 0;              // complex grids = ceil(nk/2)
  int nkp = 0;                // table width: nk rounded up to even
  int nt_eff = 0;             // t nodes in the step-3 tables (N_t + 1 - n_flat + [n_flat > 0], or 1 for SE)
  int n_flat = 0;             // leading t nodes merged into one constant term (0: none)
  double tol = 0;             // the plan's accuracy target
  int64_t mcount = 0;         // (2M+1)
  int64_t a_rows = 0;         // distinct |n|^2 values (rows of the step-3 tensor)
  // host tables: sigma_k, barycentric weights, v~_j and chi_j of eq:trapsum
  std::vector<double> sig_nodes, bary, vt, chi;
};

// Coordinate box and length-scale range of host inputs in caller order
// (x: n*d, sigma, l: n).  Throws GP_EDOMAIN for non-finite coordinates or a
// sigma or l that is not finite and > 0, GP_ERANGE for a point outside an
// explicit gp_opts box (which then replaces the data's box); gp_opts l_lo and
// l_hi widen the length range.
struct InputRanges {
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  double lmin = 0, lmax = 0;
};
void input_ranges(int d, int64_t n, const double* x, const double* sigma, const double* l,
                  const gp_opts& opts, InputRanges* r);
// The isotropic map of the box onto [-1,1]^d (section 5 assumes the points
// lie there): sets center, scale, l_range_lo/hi.
void map_box(PlanRules* P, const InputRanges& r);

// The plan's numbers from the problem's ranges alone (no device data): the
// Chebyshev degree, t grid, Fourier spacing and half-width, window and
// oversampled grid, the active box and its tiles, nk/npair/nkp.  Needs d, nu,
// se, precision and scale set; lmin, lmax in the caller's units.
void choose_params(PlanRules* P, int d, double nu, double tol, double lmin, double lmax,
                   const gp_opts& opts);

// The distinct values of |n|^2 over the mode box {-M..M}^d (ascending) and,
// for d >= 2, the map |n|^2 -> row (-1 where absent; length d M^2 + 1).
void step3_rows(const PlanRules& P, std::vector<double>& svals, std::vector<int>& rowmap);

// Host tables of the operator: fills P->sig_nodes, bary, vt, chi and
//  tvt[j], tcst[j][k], ttau[j][k]: the step-3 terms v~_j C_kj exp(-tau_kj |n|^2)
//                                  (merged flat nodes first, tau = 0)
//  g0[j][k][m] = C_kj exp(-tau_kj m^2), e1[j][k][m] = exp(-tau_kj m^2), m <= M
//  dec[r][m]   = 1 / psi^(2 pi m / nf_r), the window deconvolution
struct StepTables {
  std::vector<double> tvt, tcst, ttau, g0, e1, dec;
};
void host_tables(PlanRules* P, StepTables* T);

// Low-rank factors of the step-3 rows by pivoted Cholesky (rem:step3, last
// paragraph).  A: nrows rows of the upper triangle (width nkp) of an nk x nk
// symmetric positive semidefinite matrix.  A row keeps pivots while the largest
// remaining diagonal exceeds rel times the row's largest diagonal.  Output:
// rows[off[r] .. off[r+1]) holds rank_r vectors of nkp entries (R_a[k], zero
// for k >= nk) with A_r ~ sum_a R_a R_a'.
void lowrank_rows(int64_t nrows, int nk, int nkp, const std::vector<double>& A, double rel,
                  std::vector<int64_t>& off, std::vector<double>& rows, int* rank_max,
                  double* rank_mean);

// exp(-2 pi i k / L), k < L, as interleaved (re, im) doubles.
void twiddle_table(int L, std::vector<double>& t);

}  // namespace gp
