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
#include <cstring>
#include <limits>
#include <mutex>

#include <climits>

#include "gp_internal.h"

namespace gp {

namespace {
std::mutex& pinned_mu() {
  static std::mutex m;
  return m;
}
std::vector<double*>& pinned_free() {
  static std::vector<double*> v;  // held until the process ends
  return v;
}

// Once per device: keep released pool memory cached (the default threshold
// would hand it back to the driver at the next synchronisation).
hipMemPool_t device_pool() {
  static std::mutex mu;
  static std::vector<std::pair<int, hipMemPool_t>> pools;
  int dev = 0;
  GP_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  for (auto& q : pools)
    if (q.first == dev) return q.second;
  hipMemPool_t pool = nullptr;
  GP_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
  uint64_t keep = UINT64_MAX;
  GP_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
  pools.push_back({dev, pool});
  return pool;
}
}  // namespace

void DevBuf::alloc(size_t b, hipStream_t st) {
  release();
  if (b == 0) b = 256;
  hipMemPool_t pool = device_pool();
  hipError_t e = hipMallocAsync(&p, b, st);
  if (e != hipSuccess) {
    // hand the pool's cached memory back and try once more
    (void)hipGetLastError();
    (void)hipDeviceSynchronize();
    (void)hipMemPoolTrimTo(pool, 0);
    e = hipMallocAsync(&p, b, st);
  }
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    throw Error{GP_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed: " +
                               hipGetErrorString(e)};
  }
  bytes = b;
  s = st;
}

void DevBuf::release() {
  if (p) (void)hipFreeAsync(p, s);
  p = nullptr;
  bytes = 0;
  s = nullptr;
}

void retag_plan_stream(Plan* P, hipStream_t st) {
  Records& R = P->rec;
  DevBuf* bufs[] = {&R.perm, &R.cell, &R.pw, &R.bin_start, &R.sp_work, &R.sp_red, &R.in_work,
                    &R.in_work2, &R.part, &R.sub_off, &R.sub_list, &P->nodes_d, &P->bary_d,
                    &P->gtab, &P->etab, &P->vtd, &P->lr_off, &P->atab, &P->rowidx, &P->mode_tiles, &P->dec,
                    &P->tw[0], &P->tw[1], &P->tw[2], &P->tw4, &P->gridA, &P->gridB, &P->gridB2,
                    &P->gridC, &P->mA, &P->mB, &P->mB2, &P->mC, &P->vec, &P->cg_part, &P->cg_S};
  for (DevBuf* b : bufs)
    if (b->p) b->s = st;
}

double* pinned_scalars_get() {
  static_assert(kCgScalars > 0, "");
  {
    std::lock_guard<std::mutex> lk(pinned_mu());
    auto& fl = pinned_free();
    if (!fl.empty()) {
      double* h = fl.back();
      fl.pop_back();
      return h;
    }
  }
  double* h = nullptr;
  GP_HIP(hipHostMalloc((void**)&h, kCgScalars * sizeof(double), hipHostMallocDefault));
  return h;
}

void pinned_scalars_put(double* h) {
  if (!h) return;
  std::lock_guard<std::mutex> lk(pinned_mu());
  pinned_free().push_back(h);
}

namespace {

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

// ------------------------------------------------------------ bin sort ----
// Stable sort of the points by bin on the device, the order of a counting
// sort: by bin, and inside a bin by caller index.  The points are cut into
// chunks of consecutive indices; cnt[bin][chunk] counts them, its exclusive
// scan in bin-major order gives each (bin, chunk) its first sorted position,
// and one workgroup per chunk walks its points in batches of kSortBatch,
// sorts each batch by (bin, index) in LDS and places every run of equal bins
// after what earlier batches of the chunk placed there.
constexpr int kSortBatch = 256;

__global__ __launch_bounds__(kSortBatch) void sort_count_kernel(int64_t n, int64_t chunk, int64_t nch,
                                                                const int* __restrict__ bin_of,
                                                                int* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * kSortBatch + threadIdx.x;
  if (i >= n) return;
  atomicAdd(&cnt[(int64_t)bin_of[i] * nch + i / chunk], 1);
}

__global__ void bin_start_kernel(int64_t nbins, int64_t nch, int64_t n, const int64_t* __restrict__ off,
                                 int* __restrict__ bin_start) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nbins) bin_start[b] = (int)off[b * nch];
  if (b == nbins) bin_start[b] = (int)n;
}

__global__ __launch_bounds__(kSortBatch) void sort_place_kernel(int64_t n, int64_t chunk, int64_t nch,
                                                                const int* __restrict__ bin_of,
                                                                unsigned long long* __restrict__ off,
                                                                int* __restrict__ pos_of) {
  __shared__ int s_key[kSortBatch], s_idx[kSortBatch], s_gs[kSortBatch];
  __shared__ unsigned long long s_base[kSortBatch];
  const int t = threadIdx.x;
  const int64_t c = blockIdx.x;
  const int64_t lo = c * chunk, hi = min(n, lo + chunk);
  for (int64_t base = lo; base < hi; base += kSortBatch) {
    const int64_t i = base + t;
    __syncthreads();
    s_key[t] = i < hi ? bin_of[i] : INT_MAX;
    s_idx[t] = (int)(i - lo);  // unique within the chunk
    __syncthreads();
    // bitonic sort by (key, index), ascending
    for (int k = 2; k <= kSortBatch; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        const int u = t ^ j;
        if (u > t) {
          const bool up = (t & k) == 0;
          const int ka = s_key[t], kb = s_key[u], ia = s_idx[t], ib = s_idx[u];
          const bool gt = ka > kb || (ka == kb && ia > ib);
          if (gt == up) {
            s_key[t] = kb;
            s_key[u] = ka;
            s_idx[t] = ib;
            s_idx[u] = ia;
          }
        }
        __syncthreads();
      }
    }
    // first position of each run of equal keys (inclusive max-scan of heads)
    const int key = s_key[t];
    const bool head = t == 0 || s_key[t - 1] != key;
    s_gs[t] = head ? t : 0;
    __syncthreads();
    for (int d = 1; d < kSortBatch; d <<= 1) {
      const int v = t >= d ? s_gs[t - d] : 0;
      __syncthreads();
      s_gs[t] = max(s_gs[t], v);
      __syncthreads();
    }
    const int gs = s_gs[t];
    const bool tail = t == kSortBatch - 1 || s_key[t + 1] != key;
    if (tail && key != INT_MAX)
      s_base[gs] = atomicAdd(&off[(int64_t)key * nch + c], (unsigned long long)(t - gs + 1));
    __syncthreads();
    if (key != INT_MAX) pos_of[lo + s_idx[t]] = (int)(s_base[gs] + (unsigned long long)(t - gs));
  }
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
  for (int c = d * w + nkp; c < rs; ++c) row[c] = T(0);  // alignment padding
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
    R.in_work2.alloc(inw2.size() * sizeof(int), P->stream);
    GP_HIP(hipMemcpyAsync(R.in_work2.p, inw2.data(), inw2.size() * sizeof(int), hipMemcpyHostToDevice, s));
  }
  R.n_sp_work = (int64_t)spw.size() / 4;
  R.n_sp_red = (int64_t)spr.size() / 4;
  R.n_in_work = (int64_t)inw.size() / 4;
  R.n_slots = slots;
  R.sp_work.alloc(spw.size() * sizeof(int), P->stream);
  GP_HIP(hipMemcpyAsync(R.sp_work.p, spw.data(), spw.size() * sizeof(int), hipMemcpyHostToDevice, s));
  if (!spr.empty()) {
    R.sp_red.alloc(spr.size() * sizeof(int), P->stream);
    GP_HIP(hipMemcpyAsync(R.sp_red.p, spr.data(), spr.size() * sizeof(int), hipMemcpyHostToDevice, s));
    const int64_t tcells = (int64_t)P->tile[0] * P->tile[1] * P->tile[2];
    R.part.alloc((size_t)slots * tcells * slot_pairs(P) * cs, P->stream);
  }
  if (!inw.empty()) {
    R.in_work.alloc(inw.size() * sizeof(int), P->stream);
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
  bin_of.alloc(n * sizeof(int), P->stream);
  posd.alloc(n * sizeof(int), P->stream);
  cell_tmp.alloc(n * d * sizeof(int), P->stream);
  frac_tmp.alloc(n * d * sizeof(double), P->stream);
  sp_tmp.alloc(n * sizeof(double), P->stream);
  pf_tmp.alloc(n * sizeof(double), P->stream);
  bad.alloc(sizeof(int), P->stream);
  GP_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
  const int bs = 256;
  const unsigned nb = (unsigned)((n + bs - 1) / bs);
  hipLaunchKernelGGL(records_kernel, dim3(nb), dim3(bs), 0, s, a, pts, sig, l, bin_of.as<int>(),
                     cell_tmp.as<int>(), frac_tmp.as<double>(), sp_tmp.as<double>(),
                     pf_tmp.as<double>(), bad.as<int>());
  GP_CHECK_LAUNCH();
  // Stable sort by tile on the device: points keep their caller order inside
  // a tile, so every plan of the same input is identical.  The count matrix
  // has at most kSortCells entries (chunks of at least 1024 points).
  constexpr int64_t kSortCells = (int64_t)1 << 22;
  const int64_t nbins = P->n_bins;
  const int64_t nch = std::max<int64_t>(1, std::min<int64_t>((n + 1023) / 1024, kSortCells / nbins));
  const int64_t chunk = (n + nch - 1) / nch;
  R.n = n;
  // rows of 2-D plans that spread on sub-tiles are padded to 16 bytes (fp32:
  // 4 values), so the spreading kernel reads them as 16-byte vectors
  R.rs = d * P->w + P->nkp;
  if (d == 2 && spread_uses_sub_tiles(P)) R.rs = (R.rs + 3) / 4 * 4;
  R.perm.alloc(n * sizeof(int), P->stream);
  R.cell.alloc(n * d * sizeof(int), P->stream);
  R.pw.alloc((size_t)n * R.rs * tsz, P->stream);
  R.bin_start.alloc((P->n_bins + 1) * sizeof(int), P->stream);
  {
    DevBuf cnt, off;
    cnt.alloc((size_t)(nbins * nch) * sizeof(int), P->stream);
    off.alloc((size_t)(nbins * nch + 1) * sizeof(int64_t), P->stream);
    GP_HIP(hipMemsetAsync(cnt.p, 0, cnt.bytes, s));
    hipLaunchKernelGGL(sort_count_kernel, dim3((unsigned)((n + kSortBatch - 1) / kSortBatch)),
                       dim3(kSortBatch), 0, s, n, chunk, nch, bin_of.as<int>(), cnt.as<int>());
    GP_CHECK_LAUNCH();
    int64_t total = 0;
    exclusive_scan_counts(cnt.as<int>(), nbins * nch, off.as<int64_t>(), s, &total);
    if (total != n) throw Error{GP_EDEVICE, "internal: bin counts do not add up"};
    hipLaunchKernelGGL(bin_start_kernel, dim3((unsigned)((nbins + 1 + 255) / 256)), dim3(256), 0, s,
                       nbins, nch, n, off.as<int64_t>(), R.bin_start.as<int>());
    GP_CHECK_LAUNCH();
    hipLaunchKernelGGL(sort_place_kernel, dim3((unsigned)nch), dim3(kSortBatch), 0, s, n, chunk, nch,
                       bin_of.as<int>(), off.as<unsigned long long>(), posd.as<int>());
    GP_CHECK_LAUNCH();
    GP_HIP(hipStreamSynchronize(s));  // cnt and off are released here
  }
  int hbad = 0;
  std::vector<int> start(P->n_bins + 1, 0);
  GP_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  GP_HIP(hipMemcpyAsync(start.data(), R.bin_start.p, (P->n_bins + 1) * sizeof(int),
                        hipMemcpyDeviceToHost, s));
  GP_HIP(hipStreamSynchronize(s));
  if (out_of_box) *out_of_box = hbad;
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
  InputRanges rg;
  input_ranges(d, n, hx.data(), hs.data(), hl.data(), opts, &rg);
  map_box(P, rg);
  choose_params(P, d, nu, tol, rg.lmin, rg.lmax, opts);
  const int nf = P->nf[0];

  // ---- step 3 variant; radial rows of the precomputed tensor
  if (opts.step3 < 0 || opts.step3 > 2) throw Error{GP_EINVAL, "opts.step3 must be 0, 1 or 2"};
  P->step3 = opts.step3;
  if (opts.spread < 0 || opts.spread > 2) throw Error{GP_EINVAL, "opts.spread must be 0, 1 or 2"};
  P->spread_mode = opts.spread != GP_SPREAD_AUTO ? opts.spread : GP_SPREAD_OWNER;
  if (opts.interp < 0 || opts.interp > 2) throw Error{GP_EINVAL, "opts.interp must be 0, 1 or 2"};
  P->interp_mode = opts.interp;
  std::vector<double> svals;
  std::vector<int> rowmap;
  if (P->step3 != 1) {
    step3_rows(*P, svals, rowmap);
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
    szB = (int64_t)(P->na[1] + (P->na[1] & 1)) * (mc + (mc & 1));  // pair-interleaved (see fft_all)
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
  bytes += (size_t)n * (sizeof(int) * (1 + d) + ts * (d * P->w + P->nk + 1 + 3));
  bytes += (size_t)(P->n_bins + 1) * sizeof(int);
  bytes += work_list_bound_bytes(P, n, cs);
  bytes += spread_list_bound_bytes(P, n);
  if (P->step3 != 1)  // the low-rank rows (step3 = 2) hold at most the full row's size
    bytes += (size_t)P->a_rows * (P->nkp * (P->nkp + 1) / 2) * ts + rowmap.size() * sizeof(int) +
             (P->step3 == 2 ? (size_t)(P->a_rows + 1) * sizeof(int64_t) : 0) +
             (d == 2 ? (size_t)(P->M / kModeTileX + 1) * (P->M / kModeTileY + 1) * sizeof(int) : 0);
  else
    bytes += (size_t)P->nt_eff * P->nk * (P->M + 1) * ts * 2;
  bytes += (size_t)n * 8 * sizeof(double) + (kCgBlocks + kCgScalars) * sizeof(double);  // vectors
  bytes += (size_t)nf * cs * 2;
  P->device_bytes = bytes;
  if (bytes_out) *bytes_out = bytes;
  if (query_only) return GP_OK;
  if (opts.max_device_bytes > 0 && bytes > opts.max_device_bytes)
    throw Error{GP_ENOMEM, "plan needs " + std::to_string(bytes) + " device bytes, over the limit"};

  // ---- host tables: sigma nodes, t grid, step-3 terms, deconvolution
  StepTables tb;
  host_tables(P, &tb);
  const std::vector<double>& tvt = tb.tvt;

  auto upload = [&](DevBuf& buf, const std::vector<double>& v) {
    if (P->precision == GP_FP64) {
      buf.alloc(v.size() * sizeof(double), P->stream);
      GP_HIP(hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, s));
      GP_HIP(hipStreamSynchronize(s));
    } else {
      std::vector<float> f(v.begin(), v.end());
      buf.alloc(f.size() * sizeof(float), P->stream);
      GP_HIP(hipMemcpyAsync(buf.p, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, s));
      GP_HIP(hipStreamSynchronize(s));
    }
  };
  if (P->step3 == 1) {
    upload(P->gtab, tb.g0);
    upload(P->etab, tb.e1);
  } else {
    // precomputed tensor, one row per distinct |n|^2
    const std::vector<double>& tau = tb.ttau;
    const std::vector<double>& cst = tb.tcst;
    DevBuf dsv, dtau, dcst, dvt;
    auto up64 = [&](DevBuf& b, const std::vector<double>& v) {
      b.alloc(v.size() * sizeof(double), P->stream);
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
      P->atab.alloc((size_t)tot * ts, P->stream);
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
      full.alloc((size_t)tot * sizeof(double), P->stream);
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
      P->lr_off.alloc(off.size() * sizeof(int64_t), P->stream);
      GP_HIP(hipMemcpyAsync(P->lr_off.p, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
      upload(P->atab, rows);
    }
    if (d > 1) {
      P->rowidx.alloc(rowmap.size() * sizeof(int), P->stream);
      GP_HIP(hipMemcpyAsync(P->rowidx.p, rowmap.data(), rowmap.size() * sizeof(int),
                            hipMemcpyHostToDevice, s));
    }
    std::vector<int> order;  // read by the copy below until the stream is synchronised
    if (d == 2 && P->step3 == 0 && !P->fourstep) {
      // tiles of the orthant {0..M}^2 by the distance of their corner nearest the
      // origin (stable), so the rows of the table in use at any time form a band
      const int64_t ntx = P->M / kModeTileX + 1, nty = P->M / kModeTileY + 1;
      order.resize((size_t)(ntx * nty));
      std::vector<int64_t> key(order.size());
      for (int64_t t = 0; t < ntx * nty; ++t) {
        const int64_t x0 = (t % ntx) * kModeTileX, y0 = (t / ntx) * kModeTileY;
        order[(size_t)t] = (int)t;
        key[(size_t)t] = x0 * x0 + y0 * y0;
      }
      std::stable_sort(order.begin(), order.end(), [&](int u, int v) { return key[u] < key[v]; });
      P->mode_ntx = ntx;
      P->mode_tiles.alloc(order.size() * sizeof(int), P->stream);
      GP_HIP(hipMemcpyAsync(P->mode_tiles.p, order.data(), order.size() * sizeof(int),
                            hipMemcpyHostToDevice, s));
    }
    GP_HIP(hipStreamSynchronize(s));
  }
  upload(P->vtd, tvt);
  upload(P->dec, tb.dec);
  P->nodes_d.alloc(P->nk * sizeof(double), P->stream);
  P->bary_d.alloc(P->nk * sizeof(double), P->stream);
  GP_HIP(hipMemcpyAsync(P->nodes_d.p, P->sig_nodes.data(), P->nk * sizeof(double), hipMemcpyHostToDevice, s));
  GP_HIP(hipMemcpyAsync(P->bary_d.p, P->bary.data(), P->nk * sizeof(double), hipMemcpyHostToDevice, s));

  // FFT twiddles exp(-2 pi i k / L) for the pass lengths in use
  auto twiddles = [&](DevBuf& buf, int L) {
    std::vector<double> t;
    twiddle_table(L, t);
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
  build_spread_lists(P, P->rec);

  // ---- grids and vectors
  P->gridA.alloc((size_t)G * szA * cs, P->stream);
  P->gridB.alloc((size_t)G * szB * cs, P->stream);
  if (szB2) P->gridB2.alloc((size_t)G * szB2 * cs, P->stream);
  P->gridC.alloc((size_t)G * szC * cs, P->stream);
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
  P->vec.alloc((size_t)n * 8 * sizeof(double), P->stream);
  P->cg_part.alloc(kCgBlocks * sizeof(double), P->stream);
  P->cg_S.alloc(kCgScalars * sizeof(double), P->stream);
  P->cg_hS = pinned_scalars_get();
  GP_HIP(hipStreamSynchronize(s));
  return GP_OK;
}

}  // namespace gp
