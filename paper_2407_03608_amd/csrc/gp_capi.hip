// C ABI of gpnufft (declarations and contracts in include/gpnufft.h).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "gp_internal.h"

namespace gp {
namespace {
thread_local std::string g_err;
}
void set_error(const std::string& m) { g_err = m; }
void clear_error() { g_err.clear(); }

__global__ void axpy_kernel(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}
__global__ void sub_kernel(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                           double* __restrict__ c) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    c[i] = a[i] - b[i];
}
static unsigned blocks(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 4096); }

const char* const kPhaseNames[PH_COUNT] = {"spread", "fft_fwd_0", "fft_fwd_1", "fft_fwd_2",
                                           "mode",   "fft_inv_2", "fft_inv_1", "fft_inv_0",
                                           "interp", "cg_vec"};

static hipEvent_t take_event(Plan* P) {
  if (!P->pool.empty()) {
    hipEvent_t e = P->pool.back();
    P->pool.pop_back();
    return e;
  }
  hipEvent_t e;
  GP_HIP(hipEventCreate(&e));
  return e;
}

PhaseScope::PhaseScope(Plan* p, int ph) : P(p), phase(ph) {
  if (!P->timing) return;
  b = take_event(P);
  GP_HIP(hipEventRecord(b, P->stream));
}

PhaseScope::~PhaseScope() {
  if (!P->timing || !b) return;
  hipEvent_t e = nullptr;
  if (!P->pool.empty()) {
    e = P->pool.back();
    P->pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return;
  }
  if (hipEventRecord(e, P->stream) != hipSuccess) return;
  P->events.push_back(Plan::Ev{phase, b, e});
}

Plan::~Plan() {
  // work still queued on the plan's stream may use its buffers
  if (cg_part.p || gridA.p) (void)hipStreamSynchronize(stream);
  pinned_scalars_put(cg_hS);
  for (auto& ev : events) {
    (void)hipEventDestroy(ev.a);
    (void)hipEventDestroy(ev.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

// Iterative refinement in the caller's point order (the two plans may sort the
// points differently): r = y - A_outer x; A_inner d = r by CG to
// max(tol ||y||/||r||, inner_tol); x += d; until ||r||/||y|| <= tol.
int cg_refined_user(Plan* Pi, Plan* Po, const double* y, double* alpha, double tol,
                    double inner_tol, int max_iter, int max_refine, int replace_every,
                    int* iters_out, double* rel_out, int* passes_out) {
  if (Pi->n != Po->n || Pi->d != Po->d) throw Error{GP_EINVAL, "plans differ in n or d"};
  if (Pi->stream != Po->stream) throw Error{GP_EINVAL, "plans must share a stream"};
  if (Pi == Po) throw Error{GP_EINVAL, "inner and outer plans must be distinct plans"};
  const int64_t n = Po->n;
  hipStream_t s = Po->stream;
  // The outer plan only applies its operator (vectors 0, 1) and holds the
  // sorted right-hand side and residual (6, 7); its vectors 2..4 carry the
  // caller-order residual, correction and operator output.
  double* Vo = Po->vec.as<double>();
  double* Vi = Pi->vec.as<double>();
  double* r = Vo + 2 * n;  // user order
  double* dl = Vo + 3 * n;
  double* tmp = Vo + 4 * n;
  GP_HIP(hipMemsetAsync(alpha, 0, n * sizeof(double), s));
  gather_sorted(Po, y, Vo + 6 * n);
  const double bb = dot_sorted(Po, Vo + 6 * n, Vo + 6 * n, n);
  int total = 0, passes = 0;
  double rel = 1.0, inner_rel = 0;
  int progress = 0;
  if (const char* e = std::getenv("GPNUFFT_PROGRESS")) progress = std::atoi(e);
  while (true) {
    gather_sorted(Po, alpha, Vo);
    matvec_sorted(Po, Vo, Vo + n, 1);
    scatter_user(Po, Vo + n, tmp);
    hipLaunchKernelGGL(sub_kernel, dim3(blocks(n)), dim3(256), 0, s, n, y, tmp, r);
    GP_CHECK_LAUNCH();
    gather_sorted(Po, r, Vo + 7 * n);
    const double rr = dot_sorted(Po, Vo + 7 * n, Vo + 7 * n, n);
    rel = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    if (progress > 0) {
      std::fprintf(stderr, "[gpnufft] refine pass=%d inner_iters=%d outer_rel_res=%.3e\n", passes,
                   total, rel);
      std::fflush(stderr);
    }
    if (rel <= tol || passes >= max_refine || total >= max_iter) break;
    const double itol = std::max(tol / std::max(rel, 1e-300), inner_tol);
    gather_sorted(Pi, r, Vi + 6 * n);
    GP_HIP(hipMemsetAsync(Vi + 2 * n, 0, n * sizeof(double), s));
    int it = 0;
    (void)cg_solve_sorted(Pi, Vi + 6 * n, Vi + 2 * n, true, itol, max_iter - total, replace_every,
                          &it, &inner_rel);
    total += it;
    scatter_user(Pi, Vi + 2 * n, dl);
    hipLaunchKernelGGL(axpy_kernel, dim3(blocks(n)), dim3(256), 0, s, n, 1.0, dl, alpha);
    GP_CHECK_LAUNCH();
    ++passes;
  }
  GP_HIP(hipStreamSynchronize(s));
  *iters_out = total;
  *rel_out = rel;
  *passes_out = passes;
  return rel <= tol ? GP_OK : GP_ENOCONV;
}
}  // namespace gp

using namespace gp;

template <class F>
static int guarded(F&& f) {
  try {
    clear_error();
    return f();
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GP_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return GP_EDEVICE;
  } catch (...) {
    set_error("unknown error");
    return GP_EDEVICE;
  }
}

extern "C" {

int gp_plan(int d, int64_t n, const double* pts, const double* sigma, const double* l, double nu,
            double eta, double tol, const gp_opts* opts, gp_plan_t* out) {
  return guarded([&] {
    if (!out) throw Error{GP_EINVAL, "out is null"};
    gp_plan_s* h = new gp_plan_s();
    try {
      build_plan(d, n, pts, sigma, l, nu, eta, tol, opts, &h->P, false, nullptr);
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
    return GP_OK;
  });
}

int gp_plan_query(int d, int64_t n, const double* pts, const double* sigma, const double* l,
                  double nu, double eta, double tol, const gp_opts* opts, size_t* bytes) {
  return guarded([&] {
    if (!bytes) throw Error{GP_EINVAL, "bytes is null"};
    Plan P;
    build_plan(d, n, pts, sigma, l, nu, eta, tol, opts, &P, true, bytes);
    return GP_OK;
  });
}

static void fill_params(const Plan& P, gp_plan_params* o) {
  std::memset(o, 0, sizeof(*o));
  o->d = P.d;
  o->n = P.n;
  o->precision = P.precision;
  o->nu = P.nu;
  o->eta = P.eta;
  o->t_min = P.t_min;
  o->t_max = P.t_max;
  o->n_t = P.n_t;
  o->s_min = P.s_min;
  o->s_max = P.s_max;
  o->n_sigma = P.n_sigma;
  o->dw = P.dw;
  o->M = P.M;
  for (int r = 0; r < 3; ++r) {
    o->center[r] = P.center[r];
    o->nf[r] = P.nf[r];
    o->lo[r] = P.lo[r];
    o->na[r] = P.na[r];
    o->tile[r] = P.tile[r];
  }
  o->scale = P.scale;
  o->w = P.w;
  o->beta = P.beta;
  o->upsample = P.upsample;
  o->nufft_tol = P.nufft_tol;
  o->n_pairs = P.npair;
  o->device_bytes = P.device_bytes;
  o->pred_tail = P.pred_tail;
  o->m_capped = P.m_capped;
  o->step3 = P.step3;
  o->spread = P.spread_mode;
  o->interp = P.interp_mode;
  o->a_rows = P.a_rows;
  o->n_t_merged = P.n_flat;
  o->lr_rank_max = P.lr_rank_max;
  o->lr_rank_mean = P.lr_rank_mean;
}

int gp_plan_info(gp_plan_t h, gp_plan_params* o) {
  return guarded([&] {
    if (!h || !o) throw Error{GP_EINVAL, "null argument"};
    fill_params(h->P, o);
    return GP_OK;
  });
}

int gp_plan_rules(int d, double nu, double tol, double l_min, double l_max, double extent,
                  const gp_opts* opts_in, gp_plan_params* out) {
  return guarded([&] {
    if (!out) throw Error{GP_EINVAL, "null argument"};
    gp_opts opts;
    if (opts_in)
      opts = *opts_in;
    else
      gp_opts_init(&opts);
    if (d < 1 || d > 3) throw Error{GP_EINVAL, "d must be 1, 2 or 3"};
    if (!(nu > 0)) throw Error{GP_EDOMAIN, "nu must be > 0"};
    if (!(tol > 0) || !(tol < 1)) throw Error{GP_EDOMAIN, "tol must be in (0, 1)"};
    if (!(l_min > 0) || !(l_max >= l_min) || !std::isfinite(l_max))
      throw Error{GP_EDOMAIN, "need 0 < l_min <= l_max < inf"};
    if (!(extent > 0) || !std::isfinite(extent)) throw Error{GP_EDOMAIN, "extent must be > 0"};
    if (opts.precision != GP_FP64 && opts.precision != GP_FP32_BULK)
      throw Error{GP_EINVAL, "unknown precision"};
    Plan P;
    P.d = d;
    P.nu = nu;
    P.se = std::isinf(nu);
    P.precision = opts.precision;
    P.scale = 2.0 / extent;
    double lmin = l_min, lmax = l_max;
    if (opts.l_lo > 0) lmin = std::min(lmin, opts.l_lo);
    if (opts.l_hi > 0) lmax = std::max(lmax, opts.l_hi);
    choose_params(&P, d, nu, tol, lmin, lmax, opts);
    fill_params(P, out);
    return GP_OK;
  });
}

int gp_matvec(gp_plan_t h, const double* alpha, double* out, int add_noise) {
  return guarded([&] {
    if (!h || !alpha || !out) throw Error{GP_EINVAL, "null argument"};
    if (alpha == out) throw Error{GP_EINVAL, "alpha and out may not alias"};
    Plan* P = &h->P;
    double* xs = P->vec.as<double>();
    double* ys = xs + P->n;
    gather_sorted(P, alpha, xs);
    matvec_sorted(P, xs, ys, add_noise ? 1 : 0);
    scatter_user(P, ys, out);
    return GP_OK;
  });
}

int gp_cg_solve(gp_plan_t h, const double* y, double* alpha, int use_x0, double tol, int max_iter,
                int replace_every, gp_cg_info* info) {
  return guarded([&] {
    if (!h || !y || !alpha) throw Error{GP_EINVAL, "null argument"};
    if (!(tol > 0) || max_iter < 0) throw Error{GP_EINVAL, "tol must be > 0, max_iter >= 0"};
    Plan* P = &h->P;
    auto t0 = std::chrono::steady_clock::now();
    double* V = P->vec.as<double>();
    double* bs = V + 6 * P->n;
    double* xs = V + 2 * P->n;
    gather_sorted(P, y, bs);
    if (use_x0)
      gather_sorted(P, alpha, xs);
    else
      GP_HIP(hipMemsetAsync(xs, 0, P->n * sizeof(double), P->stream));
    int iters = 0;
    double rr = 0;
    int st = cg_solve_sorted(P, bs, xs, !use_x0, tol, max_iter, replace_every, &iters, &rr);
    scatter_user(P, xs, alpha);
    GP_HIP(hipStreamSynchronize(P->stream));
    if (info) {
      info->iters = iters;
      info->status = st;
      info->rel_res = rr;
      info->rel_res_true = -1.0;
      info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      info->refinements = 0;
    }
    if (st != GP_OK) set_error("CG reached max_iter before the tolerance");
    return st;
  });
}

int gp_cg_solve_refined(gp_plan_t hin, gp_plan_t hout, const double* y, double* alpha, double tol,
                        double inner_tol, int max_iter, int max_refine, int replace_every,
                        gp_cg_info* info) {
  return guarded([&] {
    if (!hin || !hout || !y || !alpha) throw Error{GP_EINVAL, "null argument"};
    auto t0 = std::chrono::steady_clock::now();
    int iters = 0, passes = 0;
    double rel = 0;
    const int st = cg_refined_user(&hin->P, &hout->P, y, alpha, tol, inner_tol, max_iter,
                                   max_refine, replace_every, &iters, &rel, &passes);
    if (info) {
      info->iters = iters;
      info->status = st;
      info->rel_res = rel;
      info->rel_res_true = rel;
      info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      info->refinements = passes;
    }
    if (st != GP_OK) set_error("refined CG did not reach the tolerance");
    return st;
  });
}

int gp_cg_solve_multi(gp_plan_t h, int m, const double* y, double* alpha, double tol, int max_iter,
                      int block, int* iters, double* rel_res, gp_cg_info* info) {
  return guarded([&] {
    if (!h || !y || !alpha) throw Error{GP_EINVAL, "null argument"};
    if (m < 1) throw Error{GP_EINVAL, "m must be >= 1"};
    if (!(tol > 0) || max_iter < 0) throw Error{GP_EINVAL, "tol must be > 0, max_iter >= 0"};
    Plan* P = &h->P;
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = P->n;
    hipStream_t s = P->stream;
    if (block != 0 && block != 1) throw Error{GP_EINVAL, "block must be 0 or 1"};
    int mb = multi_capacity(P, block ? std::min(m, 16) : m);
    DevBuf bs, xs;
    bs.alloc((size_t)mb * n * sizeof(double), s);
    xs.alloc((size_t)mb * n * sizeof(double), s);
    std::vector<int> it(m);
    std::vector<double> rr(m);
    int status = GP_OK;
    for (int j0 = 0; j0 < m; j0 += mb) {
      const int nb = std::min(mb, m - j0);
      for (int j = 0; j < nb; ++j) {
        gather_sorted(P, y + (int64_t)(j0 + j) * n, bs.as<double>() + (int64_t)j * n);
        zero_sorted(P, xs.as<double>() + (int64_t)j * n);
      }
      const int st = block ? cg_block_sorted(P, nb, bs.as<double>(), xs.as<double>(), tol,
                                             max_iter, it.data() + j0, rr.data() + j0)
                           : cg_multi_sorted(P, nb, bs.as<double>(), xs.as<double>(), tol,
                                             max_iter, it.data() + j0, rr.data() + j0);
      if (st != GP_OK) status = st;
      for (int j = 0; j < nb; ++j)
        scatter_user(P, xs.as<double>() + (int64_t)j * n, alpha + (int64_t)(j0 + j) * n);
    }
    GP_HIP(hipStreamSynchronize(s));
    if (iters) for (int j = 0; j < m; ++j) iters[j] = it[j];
    if (rel_res) for (int j = 0; j < m; ++j) rel_res[j] = rr[j];
    if (info) {
      info->iters = *std::max_element(it.begin(), it.end());
      info->status = status;
      info->rel_res = *std::max_element(rr.begin(), rr.end());
      info->rel_res_true = -1.0;
      info->refinements = 0;
      info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (status != GP_OK) set_error("a column reached max_iter before the tolerance");
    return status;
  });
}

// Targets must lie in the plan's box and length-scale range (host check).
static void validate_targets(Plan* P, int64_t m, const double* targets, const double* sigma_t,
                             const double* l_t) {
  std::vector<double> hx(m * P->d), hl(m), hs(m);
  GP_HIP(hipMemcpyAsync(hx.data(), targets, m * P->d * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  GP_HIP(hipMemcpyAsync(hl.data(), l_t, m * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  GP_HIP(hipMemcpyAsync(hs.data(), sigma_t, m * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  GP_HIP(hipStreamSynchronize(P->stream));
  for (int64_t i = 0; i < m; ++i) {
    for (int r = 0; r < P->d; ++r) {
      double xp = (hx[i * P->d + r] - P->center[r]) * P->scale;
      if (!std::isfinite(xp)) throw Error{GP_EDOMAIN, "non-finite target"};
      if (xp < -1.0 - 1e-12 || xp > 1.0 + 1e-12) throw Error{GP_ERANGE, "target outside the plan's box"};
    }
    if (!(hs[i] > 0) || !(hl[i] > 0)) throw Error{GP_EDOMAIN, "target scales must be > 0"};
    double sp = hl[i] * P->scale * 0.70710678118654752440;
    if (P->n_sigma > 0 && (sp < P->s_min * (1 - 1e-12) || sp > P->s_max * (1 + 1e-12)))
      throw Error{GP_ERANGE, "target length scale outside the plan's range"};
    if (P->n_sigma == 0 && std::fabs(sp - P->s_min) > 1e-12 * P->s_min)
      throw Error{GP_ERANGE, "stationary plan: target length scale differs"};
  }
}

int gp_posterior_mean(gp_plan_t h, const double* alpha, int64_t m, const double* targets,
                      const double* sigma_t, const double* l_t, double* mu) {
  return guarded([&] {
    if (!h || !alpha || !targets || !sigma_t || !l_t || !mu) throw Error{GP_EINVAL, "null argument"};
    if (m < 1) throw Error{GP_EINVAL, "m must be >= 1"};
    Plan* P = &h->P;
    validate_targets(P, m, targets, sigma_t, l_t);
    double* xs = P->vec.as<double>();
    gather_sorted(P, alpha, xs);
    posterior_sorted(P, xs, m, targets, sigma_t, l_t, mu);
    return GP_OK;
  });
}

__global__ void unit_vector_kernel(int64_t m, int64_t pos, double* e) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) e[i] = i == pos ? 1.0 : 0.0;
}

// column j of the covariance from sorted-order prior and cross terms
__global__ void cov_column_kernel(int64_t m, const int* __restrict__ perm,
                                  const double* __restrict__ prior, const double* __restrict__ cross,
                                  int64_t j, double* __restrict__ cov, double* __restrict__ var) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m) return;
  const int64_t i = perm[s];
  const double c = prior[s] - cross[s];
  if (cov) cov[i * m + j] = c;
  if (var && i == j) var[j] = c;
}

int gp_posterior_cov(gp_plan_t h, int64_t m, const double* targets, const double* sigma_t,
                     const double* l_t, double tol, int max_iter, double* cov, double* var,
                     gp_cg_info* info) {
  return guarded([&] {
    if (!h || !targets || !sigma_t || !l_t || (!cov && !var)) throw Error{GP_EINVAL, "null argument"};
    if (m < 1) throw Error{GP_EINVAL, "m must be >= 1"};
    if (!(tol > 0) || max_iter < 1) throw Error{GP_EINVAL, "tol must be > 0 and max_iter >= 1"};
    Plan* P = &h->P;
    validate_targets(P, m, targets, sigma_t, l_t);
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = P->stream;
    Records T;
    int oob = 0;
    build_records_into(P, m, targets, sigma_t, l_t, T, &oob);
    if (oob) throw Error{GP_ERANGE, "target outside the plan's box"};
    build_spread_lists(P, T);  // the targets are spread for K~(x*, .)
    std::vector<int> perm(m), inv(m);
    GP_HIP(hipMemcpyAsync(perm.data(), T.perm.p, m * sizeof(int), hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
    for (int64_t q = 0; q < m; ++q) inv[perm[q]] = (int)q;
    const int64_t n = P->n;
    // targets in blocks of mb: the block's right-hand sides k_j = K~(X, x*_j)
    // are solved together by one multi-right-hand-side CG (each operator
    // application shared by the block)
    const int mb = multi_capacity(P, (int)std::min<int64_t>(m, 16));
    DevBuf e, prior, cross, kb, vb;
    e.alloc(m * sizeof(double), s);
    prior.alloc((size_t)mb * m * sizeof(double), s);
    cross.alloc(m * sizeof(double), s);
    kb.alloc((size_t)mb * n * sizeof(double), s);
    vb.alloc((size_t)mb * n * sizeof(double), s);
    const unsigned mblk = (unsigned)((m + 255) / 256);
    int64_t total = 0;
    double worst = 0.0;
    int status = GP_OK;
    std::vector<int> it(mb);
    std::vector<double> rel(mb);
    for (int64_t j0 = 0; j0 < m; j0 += mb) {
      const int nb = (int)std::min<int64_t>(mb, m - j0);
      for (int q = 0; q < nb; ++q) {
        const int64_t j = j0 + q;
        // k_j = K~(X, x*_j) and the prior column K~(X*, x*_j) from one forward pass
        hipLaunchKernelGGL(unit_vector_kernel, dim3(mblk), dim3(256), 0, s, m, (int64_t)inv[j],
                           e.as<double>());
        GP_CHECK_LAUNCH();
        forward_from(P, T, e.as<double>());
        interp_from_grid(P, P->rec, kb.as<double>() + (int64_t)q * n);
        interp_from_grid(P, T, prior.as<double>() + (int64_t)q * m);
        zero_sorted(P, vb.as<double>() + (int64_t)q * n);
      }
      // v_j = (K~ + eta^2 I)^{-1} k_j for the block, by block CG
      const int st = cg_block_sorted(P, nb, kb.as<double>(), vb.as<double>(), tol, max_iter,
                                     it.data(), rel.data());
      if (st != GP_OK) status = st;
      for (int q = 0; q < nb; ++q) {
        const int64_t j = j0 + q;
        total += it[q];
        worst = std::max(worst, rel[q]);
        // cross term K~(X*, X) v_j
        forward_from(P, P->rec, vb.as<double>() + (int64_t)q * n);
        interp_from_grid(P, T, cross.as<double>());
        hipLaunchKernelGGL(cov_column_kernel, dim3(mblk), dim3(256), 0, s, m, T.perm.as<int>(),
                           prior.as<double>() + (int64_t)q * m, cross.as<double>(), j, cov, var);
        GP_CHECK_LAUNCH();
      }
    }
    GP_HIP(hipStreamSynchronize(s));
    if (info) {
      info->iters = (int)std::min<int64_t>(total, INT32_MAX);
      info->status = status;
      info->rel_res = worst;
      info->rel_res_true = -1.0;
      info->refinements = 0;
      info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (status != GP_OK) set_error("a CG solve reached max_iter before the tolerance");
    return status;
  });
}

int gp_residual(gp_plan_t h, const double* y, const double* alpha, double* rel_res) {
  return guarded([&] {
    if (!h || !y || !alpha || !rel_res) throw Error{GP_EINVAL, "null argument"};
    Plan* P = &h->P;
    double* V = P->vec.as<double>();
    gather_sorted(P, y, V + 6 * P->n);
    gather_sorted(P, alpha, V + 2 * P->n);
    double rr = 0, bb = 0;
    residual_norms(P, V + 6 * P->n, V + 2 * P->n, &rr, &bb);
    *rel_res = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    return GP_OK;
  });
}

int gp_plan_set_timing(gp_plan_t h, int enable) {
  return guarded([&] {
    if (!h) throw Error{GP_EINVAL, "null plan"};
    Plan* P = &h->P;
    GP_HIP(hipStreamSynchronize(P->stream));
    for (auto& ev : P->events) {
      P->pool.push_back(ev.a);
      P->pool.push_back(ev.b);
    }
    P->events.clear();
    P->timing = enable != 0;
    return GP_OK;
  });
}

int gp_plan_get_timing(gp_plan_t h, gp_timing* out) {
  return guarded([&] {
    if (!h || !out) throw Error{GP_EINVAL, "null argument"};
    Plan* P = &h->P;
    GP_HIP(hipStreamSynchronize(P->stream));
    std::memset(out, 0, sizeof(*out));
    out->n_phases = PH_COUNT;
    for (int k = 0; k < PH_COUNT; ++k) out->name[k] = kPhaseNames[k];
    for (auto& ev : P->events) {
      float ms = 0;
      GP_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
      out->ms[ev.phase] += ms;
      out->launches[ev.phase] += 1;
    }
    return GP_OK;
  });
}

int gp_plan_set_stream(gp_plan_t h, void* stream) {
  return guarded([&] {
    if (!h) throw Error{GP_EINVAL, "null plan"};
    // work queued on the old stream may still use the plan's buffers
    GP_HIP(hipStreamSynchronize(h->P.stream));
    h->P.stream = static_cast<hipStream_t>(stream);
    retag_plan_stream(&h->P, h->P.stream);
    return GP_OK;
  });
}

int gp_plan_destroy(gp_plan_t h) {
  return guarded([&] {
    if (!h) return GP_OK;
    (void)hipStreamSynchronize(h->P.stream);
    delete h;
    return GP_OK;
  });
}

const char* gp_last_error(void) { return g_err.c_str(); }

}  // extern "C"
