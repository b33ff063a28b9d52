// Conjugate gradients on (K~ + eta^2 I) x = b  (eq:gprsolve; section 6.2 wraps the
// matvec in CG with a relative-residual stopping rule).  Vectors are fp64 and
// live in the plan's bin-sorted point order; dot products are two-stage
// reductions with a fixed block count, so they are deterministic.  The step
// lengths alpha, beta and the stopping test stay on the device: the iteration
// that reaches the tolerance raises a done flag, after which the vector
// updates of iterations already queued do nothing.  The host queues
// iterations in batches and reads the flag between batches, so the iterate
// and the iteration count are those of a loop that tests every iteration.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "gp_internal.h"

namespace gp {
namespace {

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = kCgBlocks;

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kRedThreads / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kRedThreads / 64; ++k) s += red[k];
  return s;  // valid in thread 0
}

__global__ __launch_bounds__(kRedThreads) void dot_partial(int64_t n, const double* __restrict__ a,
                                                           const double* __restrict__ b,
                                                           double* __restrict__ part) {
  double v = 0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads)
    v += a[i] * b[i];
  v = block_sum(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// S layout: 0 rr, 1 pAp, 2 rr_new, 3 bb, 4 beta, 5 scratch, 6 stopping
// threshold on rr, 7 done flag, 8 completed iterations
// mode 0: S[slot] = sum; mode 1 (rr update, skipped once done): S[2] = sum,
// S[4] = sum / S[0], S[0] = sum, one more iteration, done if sum <= S[6]
__global__ __launch_bounds__(kRedThreads) void dot_final(int nparts, const double* __restrict__ part,
                                                         double* __restrict__ S, int slot, int mode) {
  double v = 0;
  for (int i = threadIdx.x; i < nparts; i += kRedThreads) v += part[i];
  v = block_sum(v);
  if (threadIdx.x == 0) {
    if (mode == 0) {
      S[slot] = v;
    } else if (S[7] == 0.0) {
      S[2] = v;
      S[4] = v / S[0];
      S[0] = v;
      S[8] += 1.0;
      if (v <= S[6]) S[7] = 1.0;
    }
  }
}

__global__ void cg_init_flags(double* S, double stop2) {
  if (threadIdx.x == 0) {
    S[6] = stop2;
    S[7] = 0.0;
    S[8] = 0.0;
  }
}

// x += a p ; r -= a Ap ; partial sums of r.r   with a = S[0]/S[1]
__global__ __launch_bounds__(kRedThreads) void update_xr(int64_t n, const double* __restrict__ S,
                                                         double* __restrict__ x,
                                                         double* __restrict__ r,
                                                         const double* __restrict__ p,
                                                         const double* __restrict__ Ap,
                                                         double* __restrict__ part) {
  if (S[7] != 0.0) return;
  const double a = S[0] / S[1];
  double v = 0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads) {
    x[i] += a * p[i];
    const double ri = r[i] - a * Ap[i];
    r[i] = ri;
    v += ri * ri;
  }
  v = block_sum(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// p = r + beta p, beta = S[4]
__global__ void update_p(int64_t n, const double* __restrict__ S, const double* __restrict__ r,
                         double* __restrict__ p) {
  if (S[7] != 0.0) return;
  const double b = S[4];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = r[i] + b * p[i];
}

// r = b - Ax
__global__ void residual(int64_t n, const double* __restrict__ b, const double* __restrict__ Ax,
                         double* __restrict__ r) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    r[i] = b[i] - Ax[i];
}

__global__ void zero_vec(int64_t n, double* __restrict__ a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0.0;
}

__global__ void copy_vec(int64_t n, const double* __restrict__ a, double* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

unsigned nblk(int64_t n) {
  int64_t b = (n + kRedThreads - 1) / kRedThreads;
  return (unsigned)std::min<int64_t>(std::max<int64_t>(b, 1), kRedBlocks);
}

void dot_into(Plan* P, const CgScratch& sc, const double* a, const double* b, int slot) {
  const unsigned nb = nblk(P->n);
  hipLaunchKernelGGL(dot_partial, dim3(nb), dim3(kRedThreads), 0, P->stream, P->n, a, b, sc.part);
  hipLaunchKernelGGL(dot_final, dim3(1), dim3(kRedThreads), 0, P->stream, (int)nb, sc.part, sc.S,
                     slot, 0);
  GP_CHECK_LAUNCH();
}

// Copy S[0 .. count) to the host and wait for it: into the pinned mirror when
// the scratch has one, else into `tmp` (pageable; the copy is then staged by
// the runtime).  Returns the host copy.
const double* read_S(Plan* P, const CgScratch& sc, int count, double* tmp) {
  double* dst = sc.hS ? sc.hS : tmp;
  GP_HIP(hipMemcpyAsync(dst, sc.S, count * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  GP_HIP(hipStreamSynchronize(P->stream));
  return dst;
}

double read_slot(Plan* P, const CgScratch& sc, int slot) {
  double tmp[kCgScalars];
  return read_S(P, sc, slot + 1, tmp)[slot];
}

}  // namespace

void zero_sorted(Plan* P, double* x) {
  hipLaunchKernelGGL(zero_vec, dim3(nblk(P->n)), dim3(kRedThreads), 0, P->stream, P->n, x);
  GP_CHECK_LAUNCH();
}

CgScratch plan_cg_scratch(Plan* P) {
  return CgScratch{P->cg_part.as<double>(), P->cg_S.as<double>(), P->cg_hS};
}

double dot_sorted(Plan* P, const double* a, const double* b, int64_t) {
  const CgScratch sc = plan_cg_scratch(P);
  dot_into(P, sc, a, b, 5);
  return read_slot(P, sc, 5);
}

void residual_norms(Plan* P, const double* b, const double* x, double* rr, double* bb) {
  double* t = P->vec.as<double>() + 7 * P->n;
  matvec_sorted(P, x, t, 1);
  hipLaunchKernelGGL(residual, dim3(nblk(P->n)), dim3(kRedThreads), 0, P->stream, P->n, b, t, t);
  GP_CHECK_LAUNCH();
  const CgScratch sc = plan_cg_scratch(P);
  dot_into(P, sc, t, t, 5);
  *rr = read_slot(P, sc, 5);
  dot_into(P, sc, b, b, 5);
  *bb = read_slot(P, sc, 5);
}

// x: in = initial guess (or zero if x_zero), out = solution (sorted order).
// Returns GP_OK or GP_ENOCONV.
int cg_solve_sorted(Plan* P, const double* b, double* x, bool x_zero, double tol, int max_iter,
                    int replace_every, int* iters, double* rel_res) {
  return cg_solve_sorted_with(P, plan_cg_scratch(P), b, x, x_zero, tol, max_iter, replace_every,
                              iters, rel_res);
}

int cg_solve_sorted_with(Plan* P, const CgScratch& sc, const double* b, double* x, bool x_zero,
                         double tol, int max_iter, int replace_every, int* iters,
                         double* rel_res) {
  const int64_t n = P->n;
  double* V = P->vec.as<double>();
  double* r = V + 3 * n;
  double* p = V + 4 * n;
  double* Ap = V + 5 * n;
  hipStream_t s = P->stream;
  const unsigned nb = nblk(n);

  if (x_zero) {
    hipLaunchKernelGGL(copy_vec, dim3(nb), dim3(kRedThreads), 0, s, n, b, r);
  } else {
    matvec_sorted(P, x, Ap, 1);
    hipLaunchKernelGGL(residual, dim3(nb), dim3(kRedThreads), 0, s, n, b, Ap, r);
  }
  hipLaunchKernelGGL(copy_vec, dim3(nb), dim3(kRedThreads), 0, s, n, r, p);
  GP_CHECK_LAUNCH();
  dot_into(P, sc, b, b, 3);
  dot_into(P, sc, r, r, 0);
  double tmp[kCgScalars];
  const double* hs = read_S(P, sc, 4, tmp);
  const double bb = hs[3];
  double rr = hs[0];
  if (bb == 0.0) {
    *iters = 0;
    *rel_res = 0;
    return GP_OK;
  }
  const double stop2 = tol * tol * bb;
  // optional progress lines on stderr every GPNUFFT_PROGRESS iterations
  int progress = 0;
  if (const char* e = std::getenv("GPNUFFT_PROGRESS")) progress = std::atoi(e);
  if (rr <= stop2) {
    *iters = 0;
    *rel_res = std::sqrt(rr / bb);
    return GP_OK;
  }
  hipLaunchKernelGGL(cg_init_flags, dim3(1), dim3(64), 0, s, sc.S, stop2);
  GP_CHECK_LAUNCH();
  // Batches grow with the iteration count (at most 1/16 of the iterations
  // done so far are queued beyond convergence) and stay short when an
  // iteration is long enough that the host round trip does not matter.
  int queued = 0, done_iters = 0, last_print = 0;
  bool done = false;
  double ms_per_iter = 0.0;
  while (queued < max_iter) {
    int cap = ms_per_iter > 1.0 ? 1 : (ms_per_iter > 0.25 ? 4 : 32);
    int batch = std::max(1, std::min(cap, queued / 16));
    batch = std::min(batch, max_iter - queued);
    const auto t0 = std::chrono::steady_clock::now();
    for (int k = 0; k < batch; ++k) {
      ++queued;
      matvec_sorted(P, p, Ap, 1);
      {
        PhaseScope ps(P, PH_CG);
        dot_into(P, sc, p, Ap, 1);
        hipLaunchKernelGGL(update_xr, dim3(nb), dim3(kRedThreads), 0, s, n, sc.S, x,
                           r, p, Ap, sc.part);
        GP_CHECK_LAUNCH();
      }
      if (replace_every > 0 && queued % replace_every == 0) {
        matvec_sorted(P, x, Ap, 1);
        hipLaunchKernelGGL(residual, dim3(nb), dim3(kRedThreads), 0, s, n, b, Ap, r);
        hipLaunchKernelGGL(dot_partial, dim3(nb), dim3(kRedThreads), 0, s, n, r, r,
                           sc.part);
        GP_CHECK_LAUNCH();
      }
      {
        PhaseScope ps(P, PH_CG);
        hipLaunchKernelGGL(dot_final, dim3(1), dim3(kRedThreads), 0, s, (int)nb,
                           sc.part, sc.S, 0, 1);
        hipLaunchKernelGGL(update_p, dim3(nb), dim3(kRedThreads), 0, s, n, sc.S, r, p);
        GP_CHECK_LAUNCH();
      }
    }
    hs = read_S(P, sc, 9, tmp);
    ms_per_iter = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                      .count() / batch;
    rr = hs[0];
    done = hs[7] != 0.0;
    done_iters = (int)hs[8];
    if (!std::isfinite(rr)) throw Error{GP_EDEVICE, "CG breakdown: non-finite residual"};
    if (progress > 0 && done_iters / progress > last_print) {
      last_print = done_iters / progress;
      std::fprintf(stderr, "[gpnufft] cg it=%d rel_res=%.3e\n", done_iters, std::sqrt(rr / bb));
      std::fflush(stderr);
    }
    if (done) break;
  }
  *iters = done_iters;
  *rel_res = std::sqrt(rr / bb);
  return done ? GP_OK : GP_ENOCONV;
}

}  // namespace gp
