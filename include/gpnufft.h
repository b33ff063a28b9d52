/*
 * gpnufft — MI355X (gfx950) library for Gaussian-process regression with the
 * non-stationary isotropic Matern kernel, following Kielstra & Lindsey,
 * "Gaussian process regression with log-linear scaling for common
 * non-stationary kernels" (arXiv 2407.03608).
 *
 * The library applies the approximate kernel matrix K~ of eq:Ktilde (section
 * 3.5) by the five-step algorithm of section 4.2 (type-1 NUFFT, pointwise
 * Fourier mixing, type-2 NUFFT) and solves (K~ + eta^2 I) alpha = y
 * (eq:gprsolve) by conjugate gradients (section 1, section 6.2).
 *
 * Kernel, in the caller's parameterisation:
 *   K(x,y) = s(x) s(y) [2 l(x) l(y) / (l(x)^2 + l(y)^2)]^(d/2)
 *            * phi_nu(|x - y| sqrt(2 / (l(x)^2 + l(y)^2)))
 * with vertical scale s(x) > 0, length scale l(x) > 0 and phi_nu the Matern
 * function of eq:matern (phi(0) = 1); nu = +INFINITY is the squared
 * exponential eq:squaredexp.  This is eq:nonstat2 with sigma_p(x) = l(x)/sqrt(2)
 * and w(x) = s(x) (sqrt(2 pi) l(x))^(d/2), so K(x,x) = s(x)^2.
 *
 * Conventions for every entry point:
 *  - Return value 0 (GP_OK) or a negative GP_E* code; on error the message
 *    is available from gp_last_error() (thread-local) and outputs are left
 *    untouched unless stated otherwise.  No C++ exception crosses the ABI.
 *  - All array arguments are fp64 DEVICE pointers (HBM), in the caller's
 *    point order.  Points are row-major n x d.
 *  - Work is ordered on the plan's HIP stream (gp_opts.stream, default the
 *    null stream); entry points that return host-visible results
 *    (gp_cg_solve's info) synchronise that stream.
 *  - A plan copies what it needs at creation and keeps no reference to the
 *    caller's buffers.  One thread may use a plan at a time; distinct plans
 *    are independent and may be used concurrently on distinct streams.
 *  - Device memory is taken and released in stream order (HIP's stream-ordered
 *    allocator on the device's default pool, which keeps released memory for
 *    reuse): creating and destroying plans never waits for work on other
 *    streams.  The plan's stream must outlive the plan.
 *  - Results are deterministic: every reduction has a fixed order, so the
 *    same inputs and options give the same bits, alone or next to other work.
 */
#ifndef GPNUFFT_H
#define GPNUFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define GP_OK 0
#define GP_EINVAL (-1)      /* bad argument (null pointer, d not in 1..3, n < 1, ...) */
#define GP_EDOMAIN (-2)     /* s <= 0, l <= 0, nu <= 0, eta < 0, tol <= 0 or non-finite input */
#define GP_ERANGE (-3)      /* posterior target outside the plan's box or length-scale range */
#define GP_ENOMEM (-4)      /* device allocation failed or exceeds gp_opts.max_device_bytes */
#define GP_ENOCONV (-5)     /* CG hit max_iter; alpha holds the last iterate, info is filled */
#define GP_EDEVICE (-6)     /* HIP runtime error */
#define GP_EUNSUPPORTED (-7) /* parameters outside what the kernels support (e.g. n_f too large) */

/* ------------------------------------------------------ spreading variants */
#define GP_SPREAD_AUTO 0
#define GP_SPREAD_LDS_ATOMIC 1
#define GP_SPREAD_OWNER 2

/* --------------------------------------------------------------- precision */
#define GP_FP64 0           /* spread / FFT / mix / interpolate in fp64 */
#define GP_FP32_BULK 1      /* spread / FFT / mix / interpolate in fp32; fp64 vectors and dots */

typedef struct gp_plan_s* gp_plan_t;

/* Plan options.  Initialise with gp_opts_init(); every field then means
 * "choose automatically" until set.  The approximation parameters are those
 * of section 3.5 (t_min, t_max, N_t, N_sigma, M, Delta-omega); setting them
 * reproduces an exact operator K~ (for example to compare with a reference). */
typedef struct {
  int precision;            /* GP_FP64 (default) or GP_FP32_BULK */
  double nufft_tol;         /* spreading tolerance; 0 = tol (fp64) or max(tol, 1e-6) (fp32) */
  double upsample;          /* fine-grid oversampling sigma: n_f >= sigma (2M+1), sigma in
                               [1.25, 2]; 0 = automatic (1.25 for d = 2, where the FFT
                               passes dominate; 2 for d = 1, 3).  The window follows the exponential-of-
                               semicircle rules of Barnett, Magland and af Klinteberg (2019)
                               for the oversampling reached, s = min(2, n_f / (2M+1)):
                               s = 2: w = ceil(log10(1/tol)) + 1, beta = 2.30 w; s < 2:
                               w = ceil(ln(10/tol) / (pi sqrt(1 - 1/s))),
                               beta = 0.97 pi (1 - 1/(2 s)) w; w <= 16.  Outside the
                               range: GP_EINVAL */
  int n_sigma;              /* Chebyshev degree N_sigma (eq:chebscheme); -1 = auto */
  int n_t;                  /* trapezoid intervals N_t (eq:dtscheme); -1 = auto; ignored for SE */
  double t_min, t_max;      /* t range; used only when n_t >= 1 is set */
  double dw;                /* Fourier spacing Delta-omega (section 3.4); 0 = auto */
  int64_t M;                /* Fourier half-width M (grid {-M..M}^d); 0 = auto */
  int64_t M_cap;            /* upper bound for automatic M; 0 = library default */
  double s_min, s_max;      /* width range [sigma_min, sigma_max] in mapped units; 0 = from data */
  int use_box;              /* 1: map the box [box_lo, box_hi] (not the data's) onto [-1,1]^d */
  double box_lo[3], box_hi[3];
  double l_lo, l_hi;        /* widen the length-scale range (posterior targets); 0 = unused */
  size_t max_device_bytes;  /* admission limit for the plan's device memory; 0 = none */
  int spread;               /* type-1 spreading variant (GP_SPREAD_*): 0 = automatic
                               (GP_SPREAD_OWNER); 1 = per-(point, row) work items with LDS
                               atomics; 2 = each thread owns grid cells of a tile (or, for
                               fp32 grids in d >= 2, of a sub-tile with one wavefront each)
                               and sums in registers in a fixed order (deterministic) */
  int interp;               /* type-2 interpolation: 0 = default (d = 2: 2x2-bin tiles plus
                               halo staged in LDS one grid pair at a time; d = 1, 3: as 2);
                               1 = one thread per point reading its window through the
                               caches; 2 = each bin's tile plus halo staged in LDS for a
                               chunk of grid pairs, (point, window row, pair) items */
  int step3;                /* step 3 of section 4.2 (rem:step3): 0 = precomputed tensor
                               A_k'k, stored once per distinct |n|^2 (default); 1 = direct
                               sum over the t nodes at every mode; 2 = the precomputed rows
                               in low-rank form A ~ sum_a R_a R_a' (pivoted Cholesky of each
                               row to tol/100 of its largest diagonal; the rank is revealed
                               row by row) */
  void* stream;             /* hipStream_t; NULL = null stream */
  int keep_t;               /* 0 (default): the leading t nodes whose Fourier multipliers
                               G^_kj[n] are constant over the mode box to 1e-3 tol (the
                               exponent 2 pi^2 sigma_max^2 chi_j^2 dw^2 d M^2 <= 1e-3 tol)
                               are merged into one term before step 3 (their weights
                               C_kj = (2 pi chi_j^2)^(d/2) sigma_k^d factor, so the merged
                               term is exact up to that flatness); 1: keep every node */
} gp_opts;

/* What the plan chose (all in the mapped coordinates x' = (x - center) * scale). */
typedef struct {
  int d;
  int64_t n;
  int precision;
  double nu, eta;
  double t_min, t_max;
  int n_t;                  /* N_t (0 for SE) */
  double s_min, s_max;      /* sigma_min, sigma_max of eq:chebscheme */
  int n_sigma;              /* N_sigma */
  double dw;                /* Delta-omega */
  int64_t M;                /* Fourier grid {-M..M}^d */
  double center[3];
  double scale;             /* x' = (x - center) * scale, l' = l * scale */
  int nf[3];                /* oversampled FFT length per dimension */
  int w;                    /* spreading window width (cells) */
  double beta;              /* exponential-of-semicircle shape parameter */
  double upsample;          /* oversampling the window is sized for: min(2, n_f / (2M+1)),
                               n_f being the smallest supported length >= requested sigma (2M+1) */
  double nufft_tol;
  int lo[3], na[3];         /* active sub-box of the fine grid (offset, length) */
  int tile[3];              /* spreading tile per dimension */
  int n_pairs;              /* complex grids; each packs two real grids */
  size_t device_bytes;      /* device memory held by the plan */
  double pred_tail;         /* predicted spectral-tail error of the Fourier box, relative */
  int m_capped;             /* 1 if M was limited by M_cap */
  int step3;                /* variant of step 3 in use (see gp_opts.step3) */
  int spread;               /* spreading variant in use: GP_SPREAD_LDS_ATOMIC or
                               GP_SPREAD_OWNER (gp_opts.spread resolved) */
  int interp;               /* interpolation variant in use (see gp_opts.interp) */
  int64_t a_rows;           /* rows of the precomputed A table (distinct |n|^2) */
  int n_t_merged;           /* leading t nodes merged into one term (see gp_opts.keep_t) */
  int lr_rank_max;          /* step3 = 2: largest rank of a row of A (0 otherwise) */
  double lr_rank_mean;      /* step3 = 2: mean rank over the rows */
} gp_plan_params;

typedef struct {
  int iters;                /* CG iterations taken (all refinement passes) */
  int status;               /* GP_OK or GP_ENOCONV */
  double rel_res;           /* recursive ||r||/||y|| at exit */
  double rel_res_true;      /* refined solve: true residual with the outer operator; plain CG: -1 (use gp_residual) */
  double seconds;           /* wall time of the solve */
  int refinements;          /* outer refinement passes (gp_cg_solve_refined) */
} gp_cg_info;

/* Fill opts with "automatic" for every field.  Always returns GP_OK. */
int gp_opts_init(gp_opts* opts);

/* Build a plan for the kernel of this header on n points in d = 1..3
 * dimensions (eq:boldK).  pts (n x d), sigma (n), l (n): device fp64.
 * nu > 0 (INFINITY = squared exponential), eta >= 0 noise s.d. (eq:gprsolve),
 * tol > 0 target accuracy for the approximation (section 5 / section 6).
 * Parameter choices are reported in gp_plan_params and can be computed
 * without device data by gp_plan_rules.  On success
 * *out owns all device memory it needs; release it with gp_plan_destroy. */
int gp_plan(int d, int64_t n, const double* pts, const double* sigma, const double* l,
            double nu, double eta, double tol, const gp_opts* opts, gp_plan_t* out);

/* Device bytes a plan with these arguments would hold (admission control).
 * Same arguments as gp_plan; reads the points to size the grids. */
int gp_plan_query(int d, int64_t n, const double* pts, const double* sigma, const double* l,
                  double nu, double eta, double tol, const gp_opts* opts, size_t* bytes);

int gp_plan_info(gp_plan_t plan, gp_plan_params* out);

/* out = K~ alpha (add_noise = 0) or (K~ + eta^2 I) alpha (add_noise = 1):
 * the five steps of section 4.2.  alpha, out: device fp64, length n, caller
 * order; may not alias. */
int gp_matvec(gp_plan_t plan, const double* alpha, double* out, int add_noise);

/* Conjugate gradients on (K~ + eta^2 I) alpha = y (eq:gprsolve), unpreconditioned
 * as in section 6.2.  alpha: in = initial guess if use_x0, out = solution.
 * Stops when the recursive residual ||r||/||y|| <= tol or after max_iter
 * iterations (GP_ENOCONV, alpha = last iterate).  Vector arithmetic and dot
 * products are fp64 in both precisions; the residual is recomputed from the
 * operator every `replace_every` iterations (0 = never).  The stopping test
 * runs on the device and the host queues iterations in batches, reading the
 * result between them: alpha and info->iters are those of a loop that tests
 * after every iteration (a few queued iterations past convergence do no
 * update). */
int gp_cg_solve(gp_plan_t plan, const double* y, double* alpha, int use_x0, double tol,
                int max_iter, int replace_every, gp_cg_info* info);

/* gp_cg_solve for callers that cannot allocate memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): same
 * arguments, kernels, iterates and results as gp_cg_solve (bit for bit), but
 * it calls no hipMalloc, hipFree, hipHostMalloc or other allocating routine.
 * Its reduction scratch (512 per-block partial sums and 16 scalar slots,
 * 4.2 KB) is a static device array that each GPU holds for the life of the
 * process, looked up on the first call on that device; every n fits in it (the
 * reduction never uses more than 512 blocks).  The plan's device must be the
 * current device (GP_EINVAL otherwise).  The host reads the solver's scalars
 * through synchronous copies to its stack.  All calls on one GPU share the
 * scratch: calls that overlap in time on one GPU (other threads, other
 * streams) race and give undefined results; serialise them. */
int gp_cg_solve_noalloc(gp_plan_t plan, const double* y, double* alpha, int use_x0, double tol,
                        int max_iter, int replace_every, gp_cg_info* info);

/* Mixed-precision solve: CG with the operator of `inner` (typically
 * GP_FP32_BULK) inside fp64 iterative refinement with the operator of
 * `outer` (GP_FP64) on the same points: x_0 = 0; r = y - A_outer x;
 * solve A_inner d = r by CG to relative tolerance max(tol ||y||/||r||, inner_tol);
 * x += d; repeat while ||r||/||y|| > tol, at most max_refine passes. */
int gp_cg_solve_refined(gp_plan_t inner, gp_plan_t outer, const double* y, double* alpha,
                        double tol, double inner_tol, int max_iter, int max_refine,
                        int replace_every, gp_cg_info* info);

/* Posterior mean eq:postmean, mu(x*) = sum_n alpha_n K~(x*, x_n), at m
 * targets (m x d device fp64) with their own scales sigma_t, l_t.  Targets
 * must lie inside the plan's box and length-scale range (GP_ERANGE
 * otherwise; widen them at plan time with gp_opts.use_box / l_lo / l_hi). */
int gp_posterior_mean(gp_plan_t plan, const double* alpha, int64_t m, const double* targets,
                      const double* sigma_t, const double* l_t, double* mu);

/* Conjugate gradients for m right-hand sides at once (eq:gprsolve with m
 * observation vectors, e.g. the columns of eq:postcov): column j of y and
 * alpha (device fp64, caller order) starts at y + j n; alpha = 0 initially.
 * Stops when every column has relative residual <= tol, or after max_iter
 * iterations.  Every iteration applies the operator to all the search
 * directions at once: each column's spreading and interpolation, then one FFT
 * batch over all columns' grids and one pass of step 3 that reads each row of
 * its table once for all columns.
 *  block = 0: m CG recurrences in lockstep, each with its own step lengths and
 *    stopping test: each column's iterates and iteration count are bit for bit
 *    those of gp_cg_solve on that column (replace_every = 0).
 *  block = 1: block CG (O'Leary 1980) over blocks of up to 16 columns, the
 *    columns sharing one Krylov space (fewer iterations than separate solves);
 *    the search block is kept orthonormal by a pivoted Cholesky QR of its
 *    unit-scaled columns that drops directions below 1e-6 (deflation: exactly
 *    or nearly dependent columns share directions).
 * Columns are processed in blocks whose batched grids fit in half of the free
 * device memory.  iters, rel_res: host arrays of m entries (iterations of the
 * column's recurrence or block; final relative residual), or NULL.  info: the
 * largest iteration count, the worst final relative residual, GP_ENOCONV if
 * any column stopped at max_iter (alpha is then still written). */
int gp_cg_solve_multi(gp_plan_t plan, int m, const double* y, double* alpha, double tol,
                      int max_iter, int block, int* iters, double* rel_res, gp_cg_info* info);

/* Posterior covariance eq:postcov at m targets (m x d device fp64, scales
 * sigma_t, l_t as for gp_posterior_mean):
 *   Sigma(x*_i, x*_j) = K~(x*_i, x*_j) - K~(x*_i, X) (K~ + eta^2 I)^{-1} K~(X, x*_j),
 * every term with the plan's operator K~ (so Sigma is the Schur complement of
 * a positive semidefinite matrix).  The solves (K~ + eta^2 I)^{-1} K~(X, x*_j)
 * run as block CG (gp_cg_solve_multi with block = 1) over blocks of up to 16
 * targets (tolerance tol, at most max_iter iterations per block), plus two
 * operator applications per target.
 * cov: m x m row-major device fp64 (column j from solve j; symmetric up to the
 * CG tolerance), or NULL; var: the m variances Sigma(x*_j, x*_j), or NULL (not
 * both NULL).  info: total iterations over the solves, the worst final
 * relative residual, GP_ENOCONV if any solve stopped at max_iter (outputs are
 * then still written).  Same target rules and errors as gp_posterior_mean. */
int gp_posterior_cov(gp_plan_t plan, int64_t m, const double* targets, const double* sigma_t,
                     const double* l_t, double tol, int max_iter, double* cov, double* var,
                     gp_cg_info* info);

/* ||y - (K~ + eta^2 I) alpha|| / ||y|| with the plan's operator (the true
 * residual of eq:gprsolve).  Synchronises the plan's stream. */
int gp_residual(gp_plan_t plan, const double* y, const double* alpha, double* rel_res);

/* Per-kernel device timing.  With timing on, every kernel group of the matvec
 * and the CG vector update is bracketed by HIP events on the plan's stream;
 * gp_plan_get_timing synchronises and returns, per phase, the number of
 * launches and the summed event time.  gp_plan_set_timing(plan, 1) resets. */
#define GP_TIMING_PHASES 10
typedef struct {
  int n_phases;
  const char* name[GP_TIMING_PHASES];   /* spread, fft_fwd_0..2, mode, fft_inv_2..0, interp, cg_vec */
  int64_t launches[GP_TIMING_PHASES];
  double ms[GP_TIMING_PHASES];
} gp_timing;
int gp_plan_set_timing(gp_plan_t plan, int enable);
int gp_plan_get_timing(gp_plan_t plan, gp_timing* out);

/* ------------------------------------------------------------- serving -----
 * Continuous batching of many independent GPR solves (each request: its own
 * points, scales, nu, eta and y).  The server runs max_slots worker threads,
 * each with its own HIP stream.  A free slot admits a queued request whose
 * plans' device bytes fit in max_device_bytes next to the requests in flight
 * (or any request when none is in flight): with GP_SERVE_FIFO the oldest
 * (waiting while it does not fit), with GP_SERVE_SMALLEST the one with the
 * smallest bytes - aging_bytes_per_s x (seconds waited), so small requests
 * pass large ones but a waiting request gains priority over time.  Admitted
 * solves overlap on the device.  With precision GP_FP32_BULK a request is solved by fp32-bulk CG
 * inside fp64 iterative refinement (two plans, as gp_cg_solve_refined),
 * unless its fp64 plan needs fewer than fp64_below_bytes of device memory (a
 * small operator whose matvec is bound by launch latency, where the fp32 grids
 * save nothing); those, and every request under GP_FP64, are solved by plain
 * fp64 CG.  The caller's device buffers (pts, sigma, l, y,
 * alpha) must stay valid until the request completes; alpha receives the
 * solution in the caller's point order. */
typedef struct gp_server_s* gp_server_t;
#define GP_SERVE_FIFO 0
#define GP_SERVE_SMALLEST 1
typedef struct {
  int max_slots;            /* requests in flight at once (1..64) */
  size_t max_device_bytes;  /* admission budget for the plans of the requests in flight */
  int precision;            /* GP_FP32_BULK (default) or GP_FP64 */
  double plan_tol;          /* tolerance of the fp64 operator (default 1e-8) */
  double plan_tol_bulk;     /* tolerance of the fp32-bulk operator (default 1e-4) */
  double cg_tol;            /* relative residual target (default 1e-6) */
  double inner_tol;         /* inner fp32 CG tolerance per refinement pass (default 3e-3) */
  int max_iter;             /* CG iterations per request, all passes (default 20000) */
  int max_refine;           /* refinement passes (default 10) */
  size_t fp64_below_bytes;  /* fp64 CG for requests whose fp64 plan is smaller (default 256 MiB) */
  int policy;               /* GP_SERVE_SMALLEST (default) or GP_SERVE_FIFO */
  double aging_bytes_per_s; /* priority gained per second of waiting (default 1 GiB/s) */
} gp_server_opts;
typedef struct {
  int status;               /* GP_OK, GP_ENOCONV or an error code */
  int iters, refinements;
  double rel_res;           /* final relative residual (fp64 operator) */
  double t_submit, t_start, t_done;  /* seconds since the server was created */
  size_t device_bytes;      /* admission bytes of the request */
  int slot;                 /* worker slot that ran it */
  int precision;            /* path it was solved on: GP_FP64 or GP_FP32_BULK */
  double t_ready;           /* seconds since creation when its plans were built; its
                               first matvec is queued right after (t_ready - t_start is
                               the time from admission to the first matvec) */
} gp_request_info;
typedef struct {
  int64_t submitted, completed, queued;
  int running, peak_running;
  size_t bytes_in_use, peak_bytes;
  double seconds;           /* since creation */
} gp_server_counters;
int gp_server_opts_init(gp_server_opts* opts);
int gp_server_create(const gp_server_opts* opts, gp_server_t* out);
/* Queue one solve; returns after sizing the request (which reads its points
 * and scales), with its id.  Validates the inputs and sizes the request
 * (GP_ENOMEM if it can never fit the budget).  stream: the hipStream_t on
 * which pts, sigma, l and y were produced (NULL = the null stream); every
 * read of them by the server is ordered after the work queued on that stream
 * at the time of the call (an event recorded there), so the caller need not
 * synchronise before submitting. */
int gp_server_submit(gp_server_t srv, int d, int64_t n, const double* pts, const double* sigma,
                     const double* l, double nu, double eta, const double* y, double* alpha,
                     void* stream, int64_t* id);
/* Block until request id has finished; returns its status. */
int gp_server_wait(gp_server_t srv, int64_t id, gp_request_info* info);
int gp_server_poll(gp_server_t srv, int64_t id, int* done);
int gp_server_stats(gp_server_t srv, gp_server_counters* out);
/* Finish every queued request, then stop the workers and free the server. */
int gp_server_destroy(gp_server_t srv);

/* The numbers gp_plan would choose (N_sigma, the t grid, Delta-omega, M, the
 * window, the FFT length and active box, n_pairs; device_bytes and a_rows are
 * 0) for d-dimensional points whose bounding box has largest side `extent`
 * (the box's largest side if opts.use_box) and length scales in
 * [l_min, l_max], from those ranges alone: host arithmetic only, no device
 * memory or data.  Section 3 gives the discretisation these rules size
 * (lemma lem:interp, lemma lem:dt, eq:PSF, the spectral tail of the Matern
 * density); the readings are those of gp_plan.  Errors: GP_EINVAL, GP_EDOMAIN,
 * GP_EUNSUPPORTED as gp_plan. */
int gp_plan_rules(int d, double nu, double tol, double l_min, double l_max, double extent,
                  const gp_opts* opts, gp_plan_params* out);

/* Change the stream later work of this plan is ordered on.  Waits for the
   work queued on the old stream; the plan's device memory is afterwards
   released in the order of the new stream (which must outlive the plan). */
int gp_plan_set_stream(gp_plan_t plan, void* stream);

int gp_plan_destroy(gp_plan_t plan);

/* Message of the last error on this thread ("" if none). */
const char* gp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GPNUFFT_H */
