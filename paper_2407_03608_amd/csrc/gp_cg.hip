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
#include <vector>

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

// ------------------------------------------------- multiple right-hand sides --
// The same kernels for m columns (blockIdx.y = column): column j of a vector
// argument starts at j n, its partial sums at j kCgBlocks and its scalar
// slots at j kCgScalars.  Every column does exactly the arithmetic of the
// one-column kernels above.
__global__ __launch_bounds__(kRedThreads) void dot_partial_m(int64_t n, const double* __restrict__ a,
                                                             const double* __restrict__ b,
                                                             double* __restrict__ part) {
  const int64_t col = blockIdx.y;
  a += col * n;
  b += col * n;
  double v = 0;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kRedThreads)
    v += a[i] * b[i];
  v = block_sum(v);
  if (threadIdx.x == 0) part[col * kRedBlocks + blockIdx.x] = v;
}

__global__ __launch_bounds__(kRedThreads) void dot_final_m(int nparts, const double* __restrict__ part,
                                                           double* __restrict__ S, int slot, int mode) {
  const int64_t col = blockIdx.y;
  part += col * kRedBlocks;
  S += col * kCgScalars;
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

// per column: stopping threshold tol^2 ||b||^2, done at once if ||b|| = 0 or
// the initial residual already meets it, no iterations yet
__global__ void cg_init_flags_m(int m, double* S, double tol) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= m) return;
  double* s = S + (int64_t)col * kCgScalars;
  s[6] = tol * tol * s[3];
  s[7] = (s[3] == 0.0 || s[0] <= s[6]) ? 1.0 : 0.0;
  s[8] = 0.0;
}

__global__ __launch_bounds__(kRedThreads) void update_xr_m(int64_t n, const double* __restrict__ S,
                                                           double* __restrict__ x,
                                                           double* __restrict__ r,
                                                           const double* __restrict__ p,
                                                           const double* __restrict__ Ap,
                                                           double* __restrict__ part) {
  const int64_t col = blockIdx.y;
  S += col * kCgScalars;
  if (S[7] != 0.0) return;
  x += col * n;
  r += col * n;
  p += col * n;
  Ap += col * n;
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
  if (threadIdx.x == 0) part[col * kRedBlocks + blockIdx.x] = v;
}

__global__ void update_p_m(int64_t n, const double* __restrict__ S, const double* __restrict__ r,
                           double* __restrict__ p) {
  const int64_t col = blockIdx.y;
  S += col * kCgScalars;
  if (S[7] != 0.0) return;
  r += col * n;
  p += col * n;
  const double b = S[4];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = r[i] + b * p[i];
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

// m right-hand sides at once: b, x are m consecutive sorted-order vectors; x
// must be zero on entry (x0 = 0).  Each column runs the recurrence of
// cg_solve_sorted (no residual replacement) with its own step lengths and
// stopping test; the operator is applied to all m directions at once
// (matvec_multi_sorted), so every column's iterates and iteration count equal
// those of cg_solve_sorted on that column alone.  iters[j], rel[j]: host
// arrays of length m.  Returns GP_OK if every column converged.
int cg_multi_sorted(Plan* P, int m, const double* b, double* x, double tol, int max_iter,
                    int* iters, double* rel) {
  const int64_t n = P->n;
  hipStream_t s = P->stream;
  DevBuf rb, pb, apb, partb, Sb;
  rb.alloc((size_t)m * n * sizeof(double), s);
  pb.alloc((size_t)m * n * sizeof(double), s);
  apb.alloc((size_t)m * n * sizeof(double), s);
  partb.alloc((size_t)m * kRedBlocks * sizeof(double), s);
  Sb.alloc((size_t)m * kCgScalars * sizeof(double), s);
  double* r = rb.as<double>();
  double* p = pb.as<double>();
  double* Ap = apb.as<double>();
  double* part = partb.as<double>();
  double* S = Sb.as<double>();
  const unsigned nb = nblk(n);
  const dim3 grid(nb, (unsigned)m);
  const unsigned mn = (unsigned)std::min<int64_t>(((int64_t)m * n + kRedThreads - 1) / kRedThreads,
                                                  (int64_t)kRedBlocks * 64);
  hipLaunchKernelGGL(copy_vec, dim3(mn), dim3(kRedThreads), 0, s, (int64_t)m * n, b, r);
  hipLaunchKernelGGL(copy_vec, dim3(mn), dim3(kRedThreads), 0, s, (int64_t)m * n, r, p);
  hipLaunchKernelGGL(dot_partial_m, grid, dim3(kRedThreads), 0, s, n, b, b, part);
  hipLaunchKernelGGL(dot_final_m, dim3(1, m), dim3(kRedThreads), 0, s, (int)nb, part, S, 3, 0);
  hipLaunchKernelGGL(dot_partial_m, grid, dim3(kRedThreads), 0, s, n, r, r, part);
  hipLaunchKernelGGL(dot_final_m, dim3(1, m), dim3(kRedThreads), 0, s, (int)nb, part, S, 0, 0);
  hipLaunchKernelGGL(cg_init_flags_m, dim3((m + 63) / 64), dim3(64), 0, s, m, S, tol);
  GP_CHECK_LAUNCH();
  std::vector<double> hS((size_t)m * kCgScalars);
  auto read_all = [&]() {
    GP_HIP(hipMemcpyAsync(hS.data(), S, hS.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
  };
  auto all_done = [&]() {
    for (int j = 0; j < m; ++j)
      if (hS[(size_t)j * kCgScalars + 7] == 0.0) return false;
    return true;
  };
  read_all();
  int queued = 0;
  double ms_per_iter = 0.0;
  while (!all_done() && queued < max_iter) {
    const int cap = ms_per_iter > 1.0 ? 1 : (ms_per_iter > 0.25 ? 4 : 32);
    int batch = std::max(1, std::min(cap, queued / 16));
    batch = std::min(batch, max_iter - queued);
    const auto t0 = std::chrono::steady_clock::now();
    for (int k = 0; k < batch; ++k) {
      ++queued;
      matvec_multi_sorted(P, m, p, Ap, 1);
      PhaseScope ps(P, PH_CG);
      hipLaunchKernelGGL(dot_partial_m, grid, dim3(kRedThreads), 0, s, n, p, Ap, part);
      hipLaunchKernelGGL(dot_final_m, dim3(1, m), dim3(kRedThreads), 0, s, (int)nb, part, S, 1, 0);
      hipLaunchKernelGGL(update_xr_m, grid, dim3(kRedThreads), 0, s, n, S, x, r, p, Ap, part);
      hipLaunchKernelGGL(dot_final_m, dim3(1, m), dim3(kRedThreads), 0, s, (int)nb, part, S, 0, 1);
      hipLaunchKernelGGL(update_p_m, grid, dim3(kRedThreads), 0, s, n, S, r, p);
      GP_CHECK_LAUNCH();
    }
    read_all();
    ms_per_iter = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                      .count() / batch;
    for (int j = 0; j < m; ++j)
      if (!std::isfinite(hS[(size_t)j * kCgScalars])) throw Error{GP_EDEVICE, "CG breakdown: non-finite residual"};
  }
  bool ok = true;
  for (int j = 0; j < m; ++j) {
    const double* sj = &hS[(size_t)j * kCgScalars];
    iters[j] = (int)sj[8];
    rel[j] = sj[3] > 0 ? std::sqrt(sj[0] / sj[3]) : 0.0;
    if (sj[7] == 0.0) ok = false;
  }
  return ok ? GP_OK : GP_ENOCONV;
}

// ------------------------------------------------------------- block CG ----
// Block conjugate gradients (O'Leary 1980) for m right-hand sides, the search
// block kept orthonormal: with X = 0, R = B, P = orth(R),
//   Q = A P;  alpha = (P'Q)^{-1} P'R;  X += P alpha;  R -= Q alpha;
//   beta = -(P'Q)^{-1} Q'R;  P = orth(R + P beta)
// until every column has ||R_j|| <= tol ||B_j||.  The columns share one
// Krylov space, so the block needs fewer iterations than m separate solves.
// orth() is a pivoted Cholesky QR of the Gram matrix of the block's columns
// scaled to unit length, dropping directions whose pivot falls below 1e-6
// (deflation: the block may shrink), followed by a second Cholesky QR pass.  Gram matrices are two-stage reductions with a fixed
// order; the m x m algebra runs on the host in fp64.  Deterministic.
namespace {

constexpr int kMaxBlock = 16;
constexpr int kGramRows = 32;  // rows staged per step of the Gram kernel

// part[b][a * nv + c] = sum over the rows of block b of U[a][i] V[c][i]
// (U: nu vectors, V: nv vectors, each n long and stored one after the other)
__global__ __launch_bounds__(kRedThreads) void gram_partial(int64_t n, const double* __restrict__ U,
                                                            int nu, const double* __restrict__ V,
                                                            int nv, double* __restrict__ part) {
  __shared__ double su[kMaxBlock][kGramRows], sv[kMaxBlock][kGramRows];
  const int ne = nu * nv;
  double acc[2] = {0.0, 0.0};  // entries threadIdx.x and threadIdx.x + 256 (ne <= 256 here)
  const int64_t nchunk = (n + kGramRows - 1) / kGramRows;
  for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const int64_t i0 = ch * kGramRows;
    __syncthreads();
    for (int e = threadIdx.x; e < (nu + nv) * kGramRows; e += kRedThreads) {
      const int vec = e / kGramRows, r = e % kGramRows;
      const int64_t i = i0 + r;
      if (vec < nu)
        su[vec][r] = i < n ? U[(int64_t)vec * n + i] : 0.0;
      else
        sv[vec - nu][r] = i < n ? V[(int64_t)(vec - nu) * n + i] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = threadIdx.x + h * kRedThreads;
      if (e < ne) {
        const int a = e / nv, c = e % nv;
        double t = 0.0;
#pragma unroll 8
        for (int r = 0; r < kGramRows; ++r) t += su[a][r] * sv[c][r];
        acc[h] += t;
      }
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = threadIdx.x + h * kRedThreads;
    if (e < ne) part[(int64_t)blockIdx.x * ne + e] = acc[h];
  }
}

// G[e] = sum over blocks b (in order) of part[b][e]
__global__ void gram_final(int nblocks, int ne, const double* __restrict__ part, double* __restrict__ G) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += part[(int64_t)b * ne + e];
  G[e] = s;
}

// Row-local block updates with the coefficients co (np x m, row-major):
// block_update_xr: X_j += sum_a P_a co_aj,  R_j -= sum_a Q_a co_aj  (co = alpha)
// block_update_z:  Z_j  = R_j + sum_a P_a co_aj                    (co = beta)
__global__ void block_update_xr(int64_t n, int np, int m, const double* __restrict__ co,
                                const double* __restrict__ P, const double* __restrict__ Q,
                                double* __restrict__ X, double* __restrict__ R) {
  __shared__ double al[kMaxBlock * kMaxBlock];
  for (int e = threadIdx.x; e < np * m; e += blockDim.x) al[e] = co[e];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double p[kMaxBlock], q[kMaxBlock];
#pragma unroll
    for (int a = 0; a < kMaxBlock; ++a) {
      p[a] = a < np ? P[(int64_t)a * n + i] : 0.0;
      q[a] = a < np ? Q[(int64_t)a * n + i] : 0.0;
    }
    for (int j = 0; j < m; ++j) {
      double dx = 0.0, dr = 0.0;
#pragma unroll
      for (int a = 0; a < kMaxBlock; ++a) {
        if (a < np) {
          dx += p[a] * al[a * m + j];
          dr += q[a] * al[a * m + j];
        }
      }
      X[(int64_t)j * n + i] += dx;
      R[(int64_t)j * n + i] -= dr;
    }
  }
}

__global__ void block_update_z(int64_t n, int np, int m, const double* __restrict__ co,
                               const double* __restrict__ P, const double* __restrict__ R,
                               double* __restrict__ Z) {
  __shared__ double be[kMaxBlock * kMaxBlock];
  for (int e = threadIdx.x; e < np * m; e += blockDim.x) be[e] = co[e];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double p[kMaxBlock];
#pragma unroll
    for (int a = 0; a < kMaxBlock; ++a) p[a] = a < np ? P[(int64_t)a * n + i] : 0.0;
    for (int j = 0; j < m; ++j) {
      double dz = 0.0;
#pragma unroll
      for (int a = 0; a < kMaxBlock; ++a)
        if (a < np) dz += p[a] * be[a * m + j];
      Z[(int64_t)j * n + i] = R[(int64_t)j * n + i] + dz;
    }
  }
}

// P_a = sum_b Z_{col_b} T[b][a], a < np (T: the kept columns' inverse Cholesky factor)
// (Z and P may be the same buffer: each row is read whole before it is written.)
__global__ void block_orth(int64_t n, int np, const int* __restrict__ cols, const double* __restrict__ T,
                           const double* Z, double* P) {
  __shared__ double t[kMaxBlock * kMaxBlock];
  __shared__ int c[kMaxBlock];
  for (int e = threadIdx.x; e < np * np; e += blockDim.x) t[e] = T[e];
  if (threadIdx.x < np) c[threadIdx.x] = cols[threadIdx.x];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double z[kMaxBlock];
#pragma unroll
    for (int b = 0; b < kMaxBlock; ++b) z[b] = b < np ? Z[(int64_t)c[b] * n + i] : 0.0;
    for (int a = 0; a < np; ++a) {
      double v = 0.0;
#pragma unroll
      for (int b = 0; b < kMaxBlock; ++b)
        if (b <= a && b < np) v += z[b] * t[b * np + a];
      P[(int64_t)a * n + i] = v;
    }
  }
}

// Pivoted Cholesky G = L L' (outer-product form, the largest remaining
// diagonal first) of the k x k Gram matrix of a block Z (row-major), stopping
// when the remaining diagonal falls below rel^2 times the largest diagonal of
// G.  Returns np; cols: the kept columns of Z in pivot order; T = L^{-T}
// (np x np, upper triangular, row-major), so that Z_cols T has the identity as
// Gram matrix.
int pivoted_chol_inv(int k, std::vector<double> A, double rel, std::vector<int>& cols,
                     std::vector<double>& T) {
  std::vector<int> perm(k);
  for (int i = 0; i < k; ++i) perm[i] = i;
  double dmax = 0.0;
  for (int i = 0; i < k; ++i) dmax = std::max(dmax, A[(size_t)i * k + i]);
  std::vector<double> L((size_t)k * k, 0.0);  // L[i][j], rows in pivot order
  int np = 0;
  for (int j = 0; j < k; ++j) {
    int best = j;
    for (int i = j + 1; i < k; ++i)
      if (A[(size_t)perm[i] * k + perm[i]] > A[(size_t)perm[best] * k + perm[best]]) best = i;
    if (best != j) {
      std::swap(perm[j], perm[best]);
      for (int q = 0; q < j; ++q) std::swap(L[(size_t)j * k + q], L[(size_t)best * k + q]);
    }
    const int pj = perm[j];
    const double d = A[(size_t)pj * k + pj];
    if (!(dmax > 0.0) || !(d > rel * rel * dmax)) break;
    const double l = std::sqrt(d);
    L[(size_t)j * k + j] = l;
    for (int i = j + 1; i < k; ++i) L[(size_t)i * k + j] = A[(size_t)perm[i] * k + pj] / l;
    // Schur complement of the trailing block
    for (int i = j + 1; i < k; ++i)
      for (int q = j + 1; q < k; ++q)
        A[(size_t)perm[i] * k + perm[q]] -= L[(size_t)i * k + j] * L[(size_t)q * k + j];
    ++np;
  }
  cols.assign(perm.begin(), perm.begin() + np);
  // T = L^{-T}: solve L' T = I column by column (back substitution)
  T.assign((size_t)np * np, 0.0);
  for (int c = 0; c < np; ++c)
    for (int r = np - 1; r >= 0; --r) {
      double v = r == c ? 1.0 : 0.0;
      for (int q = r + 1; q < np; ++q) v -= L[(size_t)q * k + r] * T[(size_t)q * np + c];
      T[(size_t)r * np + c] = v / L[(size_t)r * k + r];
    }
  return np;
}

// Solve S Y = B for the SPD np x np matrix S (row-major) and np x m right-hand
// sides B (row-major), by Cholesky; Y overwrites B.
void spd_solve(int np, int m, std::vector<double> S, std::vector<double>& B) {
  for (int j = 0; j < np; ++j) {
    double d = S[j * np + j];
    for (int q = 0; q < j; ++q) d -= S[j * np + q] * S[j * np + q];
    if (!(d > 0.0)) throw Error{GP_EDEVICE, "block CG: P'AP is not positive definite"};
    const double l = std::sqrt(d);
    S[j * np + j] = l;
    for (int i = j + 1; i < np; ++i) {
      double v = S[i * np + j];
      for (int q = 0; q < j; ++q) v -= S[i * np + q] * S[j * np + q];
      S[i * np + j] = v / l;
    }
  }
  for (int c = 0; c < m; ++c) {
    for (int i = 0; i < np; ++i) {
      double v = B[i * m + c];
      for (int q = 0; q < i; ++q) v -= S[i * np + q] * B[q * m + c];
      B[i * m + c] = v / S[i * np + i];
    }
    for (int i = np - 1; i >= 0; --i) {
      double v = B[i * m + c];
      for (int q = i + 1; q < np; ++q) v -= S[q * np + i] * B[q * m + c];
      B[i * m + c] = v / S[i * np + i];
    }
  }
}

}  // namespace

int cg_block_sorted(Plan* P, int m, const double* b, double* x, double tol, int max_iter,
                    int* iters, double* rel) {
  if (m < 1 || m > kMaxBlock) throw Error{GP_EINVAL, "block CG takes 1..16 right-hand sides"};
  const int64_t n = P->n;
  hipStream_t s = P->stream;
  DevBuf Rb, Pb, Qb, Zb, partb, Gb, cob, colb;
  Rb.alloc((size_t)m * n * sizeof(double), s);
  Pb.alloc((size_t)m * n * sizeof(double), s);
  Qb.alloc((size_t)m * n * sizeof(double), s);
  Zb.alloc((size_t)m * n * sizeof(double), s);
  partb.alloc((size_t)kRedBlocks * m * m * sizeof(double), s);
  Gb.alloc((size_t)m * m * sizeof(double), s);
  cob.alloc((size_t)2 * m * m * sizeof(double), s);
  colb.alloc(kMaxBlock * sizeof(int), s);
  double* R = Rb.as<double>();
  double* Pm = Pb.as<double>();
  double* Q = Qb.as<double>();
  double* Z = Zb.as<double>();
  const unsigned rows_blk = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
  const unsigned gram_blk = (unsigned)std::min<int64_t>((n + kGramRows - 1) / kGramRows, kRedBlocks);
  // G = U'V (nu x nv, row-major) on the host
  auto gram = [&](const double* U, int nu, const double* V, int nv, std::vector<double>& G) {
    hipLaunchKernelGGL(gram_partial, dim3(gram_blk), dim3(kRedThreads), 0, s, n, U, nu, V, nv,
                       partb.as<double>());
    hipLaunchKernelGGL(gram_final, dim3((nu * nv + 255) / 256), dim3(256), 0, s, (int)gram_blk,
                       nu * nv, partb.as<double>(), Gb.as<double>());
    GP_CHECK_LAUNCH();
    G.resize((size_t)nu * nv);
    GP_HIP(hipMemcpyAsync(G.data(), Gb.p, G.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    GP_HIP(hipStreamSynchronize(s));
  };
  // P = orth(Z): pivoted Cholesky QR of the unit-scaled columns that drops
  // directions below 1e-6 (deflation), then a second Cholesky QR pass of the
  // kept block for orthogonality.  Returns the block size.
  std::vector<int> cols;
  std::vector<double> T, G;
  auto apply = [&](const double* src, int np) {
    GP_HIP(hipMemcpyAsync(colb.p, cols.data(), np * sizeof(int), hipMemcpyHostToDevice, s));
    GP_HIP(hipMemcpyAsync(cob.p, T.data(), T.size() * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(block_orth, dim3(rows_blk), dim3(256), 0, s, n, np, colb.as<int>(),
                       cob.as<double>(), src, Pm);
    GP_CHECK_LAUNCH();
    GP_HIP(hipStreamSynchronize(s));  // cols and T are host buffers reused below
  };
  auto orth = [&](const double* Zs, int k) {
    gram(Zs, k, Zs, k, G);
    // scale the columns to unit length, so that dependence is judged by angle
    // (a column duplicating another leaves a Schur complement at rounding
    // level, ~1e-16 of its norm squared, far below the 1e-12 threshold)
    std::vector<double> sc(k);
    for (int j = 0; j < k; ++j) {
      const double g = G[(size_t)j * k + j];
      sc[j] = g > 0.0 ? 1.0 / std::sqrt(g) : 0.0;
    }
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) G[(size_t)i * k + j] *= sc[i] * sc[j];
    const int np = pivoted_chol_inv(k, G, 1e-6, cols, T);
    if (np == 0) return 0;
    for (int b = 0; b < np; ++b)
      for (int a = 0; a < np; ++a) T[(size_t)b * np + a] *= sc[cols[b]];
    apply(Zs, np);
    gram(Pm, np, Pm, np, G);
    std::vector<int> kept;
    const int np2 = pivoted_chol_inv(np, G, 1e-6, kept, T);
    cols = kept;
    if (np2 == 0) return 0;
    apply(Pm, np2);  // in place: each row is read whole before it is written
    return np2;
  };
  const unsigned mn = (unsigned)std::min<int64_t>(((int64_t)m * n + 255) / 256, 16384);
  hipLaunchKernelGGL(copy_vec, dim3(mn), dim3(256), 0, s, (int64_t)m * n, b, R);
  GP_CHECK_LAUNCH();
  std::vector<double> bb;
  gram(b, m, b, m, G);
  bb.resize(m);
  for (int j = 0; j < m; ++j) bb[j] = G[(size_t)j * m + j];
  std::vector<double> rr(bb);
  auto converged = [&]() {
    for (int j = 0; j < m; ++j)
      if (rr[j] > tol * tol * bb[j]) return false;
    return true;
  };
  int it = 0;
  int progress = 0;
  if (const char* e = std::getenv("GPNUFFT_PROGRESS")) progress = std::atoi(e);
  int np = converged() ? 0 : orth(R, m);
  std::vector<double> G1, G2, G3;
  auto upload = [&](const std::vector<double>& v) {
    GP_HIP(hipMemcpyAsync(cob.p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, s));
  };
  while (np > 0 && !converged() && it < max_iter) {
    matvec_multi_sorted(P, np, Pm, Q, 1);
    gram(Pm, np, Q, np, G1);  // P'AP
    gram(Pm, np, R, m, G2);   // P'R
    spd_solve(np, m, G1, G2);  // alpha
    upload(G2);
    hipLaunchKernelGGL(block_update_xr, dim3(rows_blk), dim3(256), 0, s, n, np, m,
                       cob.as<double>(), Pm, Q, x, R);
    GP_CHECK_LAUNCH();
    ++it;
    gram(R, m, R, m, G);
    for (int j = 0; j < m; ++j) rr[j] = G[(size_t)j * m + j];
    for (int j = 0; j < m; ++j)
      if (!std::isfinite(rr[j])) throw Error{GP_EDEVICE, "block CG breakdown: non-finite residual"};
    if (progress > 0 && it % progress == 0) {
      double worst = 0.0;
      for (int j = 0; j < m; ++j)
        if (bb[j] > 0) worst = std::max(worst, std::sqrt(rr[j] / bb[j]));
      std::fprintf(stderr, "[gpnufft] block cg it=%d block=%d worst_rel_res=%.3e\n", it, np, worst);
      std::fflush(stderr);
    }
    if (converged()) break;
    gram(Q, np, R, m, G3);  // Q'R with the new residual
    for (double& v : G3) v = -v;
    spd_solve(np, m, G1, G3);  // beta
    upload(G3);
    hipLaunchKernelGGL(block_update_z, dim3(rows_blk), dim3(256), 0, s, n, np, m,
                       cob.as<double>(), Pm, R, Z);
    GP_CHECK_LAUNCH();
    np = orth(Z, m);
  }
  for (int j = 0; j < m; ++j) {
    iters[j] = it;
    rel[j] = bb[j] > 0 ? std::sqrt(rr[j] / bb[j]) : 0.0;
  }
  return converged() ? GP_OK : GP_ENOCONV;
}

}  // namespace gp
