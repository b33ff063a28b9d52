// gp_cg_solve_noalloc: conjugate gradients on (K~ + eta^2 I) alpha = y for
// callers that cannot allocate memory (code under stream capture, tight
// serving loops, harnesses that forbid allocation).  It runs the same kernels
// as gp_cg_solve; the reduction scratch (per-block partial sums of the dot
// products and the solver's scalar slots) lives in the file-scope device
// array `scratch` below instead of the plan's buffers, and the host reads the
// scalar slots through a synchronous copy to its stack (no pinned buffer).
// The plan's own vectors, allocated when the plan was built, hold x, r, p, Ap
// and the sorted right-hand side.
#include <algorithm>
#include <chrono>
#include <mutex>
#include <vector>

#include "gp_internal.h"

namespace gp {

// One copy per GPU, for the life of the process; every call on a GPU shares
// it (concurrent calls on one GPU race on it).
constexpr int kScratchDoubles = kCgBlocks + kCgScalars;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;  // per device; null until looked up

// Device address of `scratch` on the current device, looked up once per
// device with that device current.  In host code the array's name is only a
// host-side stand-in, so every kernel argument uses this address.
double* device_scratch() {
  int dev = 0;
  GP_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    GP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error{GP_EDEVICE, "hipGetSymbolAddress(scratch) returned null"};
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace gp

using namespace gp;

extern "C" int gp_cg_solve_noalloc(gp_plan_t h, const double* y, double* alpha, int use_x0,
                                   double tol, int max_iter, int replace_every,
                                   gp_cg_info* info) {
  try {
    clear_error();
    if (!h || !y || !alpha) throw Error{GP_EINVAL, "null argument"};
    if (!(tol > 0) || max_iter < 0) throw Error{GP_EINVAL, "tol must be > 0, max_iter >= 0"};
    Plan* P = &h->P;
    int dev = 0;
    GP_HIP(hipGetDevice(&dev));
    if (dev != P->device)
      throw Error{GP_EINVAL, "the plan's device (" + std::to_string(P->device) +
                                 ") must be current (current: " + std::to_string(dev) + ")"};
    // The reduction uses min(ceil(n / 256), kCgBlocks) partial sums plus the
    // scalar slots: at most kScratchDoubles doubles for every n.
    const int64_t parts = std::min<int64_t>((P->n + 255) / 256, kCgBlocks);
    if (parts + kCgScalars > kScratchDoubles)
      throw Error{GP_EUNSUPPORTED, "CG scratch of " + std::to_string(parts + kCgScalars) +
                                       " doubles exceeds the static " +
                                       std::to_string(kScratchDoubles)};
    double* sp = device_scratch();
    const CgScratch sc{sp, sp + kCgBlocks, nullptr};
    const auto t0 = std::chrono::steady_clock::now();
    double* V = P->vec.as<double>();
    double* bs = V + 6 * P->n;
    double* xs = V + 2 * P->n;
    gather_sorted(P, y, bs);
    if (use_x0)
      gather_sorted(P, alpha, xs);
    else
      zero_sorted(P, xs);
    int iters = 0;
    double rr = 0;
    const int st = cg_solve_sorted_with(P, sc, bs, xs, !use_x0, tol, max_iter, replace_every,
                                        &iters, &rr);
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
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return GP_EDEVICE;
  }
}
