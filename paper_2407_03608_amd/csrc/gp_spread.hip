// Type-1 spreading on sub-tiles (steps 1 and 2a of section 4.2):
// c_{k,i} = w_k(x_i) x_i (eq:c) spread onto the fine grids with the
// exponential-of-semicircle window, in d = 2 and 3.
//
// Owner-computes on sub-tiles of ST^d cells (ST = 8 in 2-D, 4 in 3-D) with one
// wavefront per sub-tile and one cell per lane.  The points whose window
// reaches a sub-tile are listed once per plan (in the order the sorted points
// are visited), so a matvec streams exactly the contributing points of each
// sub-tile, and the summation order of every cell is that list order (the
// result is bitwise reproducible; no atomics, no zero-fill pass, plain
// stores).  For each listed point the wavefront stages, per dimension, the ST
// window values that fall on the sub-tile's cells (zero where the window does
// not reach), so every lane adds psi_0 psi_1 (psi_2) x_i w_k to its cell
// without a test or a divergent branch.
#include <algorithm>
#include <limits>

#include "gp_internal.h"

namespace gp {
namespace {

template <typename T> struct V2;
template <> struct V2<double> { using type = double2; };
template <> struct V2<float> { using type = float2; };

constexpr int kSubThreads = 64;  // one wavefront per sub-tile
constexpr int kGCmax = 8;        // grid pairs per launch

// Sub-tile blk = bin * nsub + sub (sub-tiles of a bin consecutive, first
// dimension fastest): its first cell s0 and its bin's coordinates tcoord.
__device__ __forceinline__ void sub_tile_origin(const NuArgs& a, int D, int st, int64_t blk,
                                                int* s0, int* tcoord) {
  int nsub = 1;
  for (int r = 0; r < D; ++r) nsub *= a.tile[r] / st;  // st divides every tile side
  int64_t tb = blk / nsub;
  int sub = (int)(blk % nsub);
  for (int r = 0; r < 3; ++r) {
    s0[r] = 0;
    tcoord[r] = 0;
  }
  for (int r = 0; r < D; ++r) {
    const int per = a.tile[r] / st;
    tcoord[r] = (int)(tb % a.nbins[r]);
    tb /= a.nbins[r];
    s0[r] = tcoord[r] * a.tile[r] + (sub % per) * st;
    sub /= per;
  }
}

// Workgroups go to the 8 XCDs round-robin by id.  Sub-tiles are dealt to the
// XCDs in groups of `grp` consecutive ones (the sub-tiles of the bins that
// share cache lines of grid rows), so each group is written through one L2,
// while the groups still alternate between XCDs (clustered points keep every
// XCD equally busy).  The grid is padded to a multiple of 8 grp workgroups;
// the map is a bijection onto [0, gridDim.x) and ids >= the sub-tile count
// have no work.
__device__ __forceinline__ int64_t xcd_grouped(int64_t bid, int grp) {
  const int64_t x = bid % 8, k = bid / 8;
  return ((k / grp) * 8 + x) * grp + k % grp;
}

// Plan time, one wavefront per sub-tile: walk the concatenated source bins
// (the tile's bin and its lower neighbours within w-1 cells, first dimension
// fastest, without the bins none of whose points reach this sub-tile: along
// dimension r the points of the bin dq >= 1 tiles below start at most at
// t0 - (dq - 1) tile - 1, so their windows end before s0 when that
// start + w - 1 < s0), keep the points whose window reaches the sub-tile in
// every dimension, and either count them (FILL = false) or write them at
// list[off[blk] ..] in visiting order (FILL = true): {sorted index, first
// window cell relative to s0 - (w - 1), 8 bits per dimension}.
template <int D, bool FILL>
__global__ __launch_bounds__(kSubThreads) void spread_list_build_kernel(
    NuArgs a, int st, const int* __restrict__ cell, const int* __restrict__ bin_start,
    int* __restrict__ cnt, const int64_t* __restrict__ off, int2* __restrict__ list) {
  extern __shared__ int ismem[];
  const int64_t blk = blockIdx.x;
  int s0[3], tcoord[3];
  sub_tile_origin(a, D, st, blk, s0, tcoord);
  const int w = a.w;
  int nsrc_tot = 1;
  for (int r = 0; r < D; ++r) nsrc_tot *= a.nsrc;
  int* s_sb0 = ismem;              // [nsrc_tot]
  int* s_soff = s_sb0 + nsrc_tot;  // [nsrc_tot + 1]
  for (int sb = threadIdx.x; sb < nsrc_tot; sb += kSubThreads) {
    int64_t b = 0, mul = 1;
    bool ok = true;
    int q = sb;
    for (int r = 0; r < D; ++r) {
      const int dq = q % a.nsrc;
      const int br = tcoord[r] - dq;
      q /= a.nsrc;
      if (br < 0) ok = false;
      if (dq > 0 && tcoord[r] * a.tile[r] - (dq - 1) * a.tile[r] - 1 + w - 1 < s0[r]) ok = false;
      b += (int64_t)br * mul;
      mul *= a.nbins[r];
    }
    const int b0 = ok ? bin_start[b] : 0;
    s_sb0[sb] = b0;
    s_soff[sb + 1] = ok ? bin_start[b + 1] - b0 : 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s_soff[0] = 0;
    for (int sb = 0; sb < nsrc_tot; ++sb) s_soff[sb + 1] += s_soff[sb];
  }
  __syncthreads();
  const int seq_hi = s_soff[nsrc_tot];
  int64_t count = 0;
  const int64_t o = FILL ? off[blk] : 0;
  for (int base = 0; base < seq_hi; base += kSubThreads) {
    const int qpos = base + (int)threadIdx.x;
    bool keep = qpos < seq_hi;
    int idx = 0, cw = 0;
    if (keep) {
      int sb = 0;
      while (qpos >= s_soff[sb + 1]) ++sb;
      idx = s_sb0[sb] + (qpos - s_soff[sb]);
      int cr[3];
      for (int r = 0; r < D; ++r) cr[r] = cell[r * a.n + idx];
      for (int r = 0; r < D; ++r) {
        keep = keep & (cr[r] + w - 1 >= s0[r]) & (cr[r] < s0[r] + st);
        cw |= (cr[r] - s0[r] + w - 1) << (8 * r);
      }
    }
    const unsigned long long m = __ballot(keep);
    if (FILL && keep) list[o + count + __popcll(m & ((1ull << threadIdx.x) - 1ull))] = int2{idx, cw};
    count += __popcll(m);
  }
  if (!FILL && threadIdx.x == 0) cnt[blk] = (int)count;
}

// One wavefront per sub-tile of ST^D cells, one cell per lane.  Batches of up
// to 64 listed points are staged in LDS, per point: for each dimension r the
// ST window values psi_r(cell - first cell) on the sub-tile's cells along r
// (zero outside the window; dimension 0 multiplied by x_i), then the chunk's
// 2 GC weights w_k (16-byte aligned, read as vectors).  A lane adds
// ((psi_0 x) psi_1) psi_2 w_k to its cell for every staged point, four points
// per step (the batch is padded to a multiple of four with zero entries).
// In 2-D (latency-bound: about 17 points per sub-tile) the point rows are read
// as 16-byte vectors, kStageVec per lane in flight, and each value is put in
// its slot (0.27 -> 0.24 ms at d=2 N=1e6); in 3-D (bound by VALU issue) each
// lane fetches the slot values it stores, kStageChunk loads in flight (the
// vector form measured 3.65 against 3.19 ms at d=3 N=1e7).
constexpr int kStageVec = 8;
constexpr int kStageChunk = 4;
template <typename T, int D, int ST, int GC>
__global__ __launch_bounds__(kSubThreads) void spread_list_kernel(
    NuArgs a, int grp, int64_t nsub, const double* __restrict__ x, const T* __restrict__ pw,
    int rs, const int64_t* __restrict__ off, const int2* __restrict__ list,
    typename V2<T>::type* __restrict__ grid) {
  using V = typename V2<T>::type;
  constexpr int NW = D * ST;                     // staged window values per point
  constexpr int SW = (NW + 3) / 4 * 4;           // first weight (aligned)
  constexpr int SS = (SW + 2 * GC + 3) / 4 * 4;  // staged values per point
  constexpr int NG = 2 * GC;
  __shared__ __align__(16) T s_v[kSubThreads * SS];
  __shared__ int s_cw[kSubThreads], s_map[kSubThreads];
  __shared__ T s_x[kSubThreads];
  static_assert(sizeof(T) == 4, "sub-tile spreading reads fp32 rows as 16-byte vectors");

  const int64_t blk = xcd_grouped(blockIdx.x, grp);
  if (blk >= nsub) return;
  int s0[3], tcoord[3];
  sub_tile_origin(a, D, ST, blk, s0, tcoord);
  const int t = threadIdx.x;
  const int lx = t % ST, ly = (t / ST) % ST, lz = D > 2 ? (t / (ST * ST)) % ST : 0;
  const bool mine = t < (D > 2 ? ST * ST * ST : ST * ST);
  V acc[GC];
#pragma unroll
  for (int g = 0; g < GC; ++g) acc[g] = V{T(0), T(0)};
  const int w = a.w;
  const int wko = D * w + 2 * a.g0;
  const char* pwb = reinterpret_cast<const char*>(pw);
  const int64_t lo = off[blk], hi = off[blk + 1];
  for (int64_t base = lo; base < hi; base += kSubThreads) {
    const int np = (int)min((int64_t)kSubThreads, hi - base);
    const int np4 = (np + 3) & ~3;
    if constexpr (D == 2) {
      __syncthreads();
      if (t < np) {
        const int2 ent = list[base + t];
        s_map[t] = ent.x;
        s_cw[t] = ent.y;
        s_x[t] = (T)x[ent.x];
      }
      // window slots the point's window does not reach stay zero; padding
      // entries (np .. np4) are zero throughout
      for (int e = t; e < np * NW; e += kSubThreads) s_v[(e / NW) * SS + e % NW] = T(0);
      for (int e = np * SS + t; e < np4 * SS; e += kSubThreads) s_v[e] = T(0);
      __syncthreads();
      // the rows as 16-byte vectors (rows are padded to a multiple of 4
      // values), kStageVec per lane issued together; each value goes to the slot
      // of the sub-tile cell it weights (dimension 0 times x_i) or, for the
      // chunk's weights, to its place after the window slots
      const int R4 = rs / 4, nv = np * R4;
      const float4* __restrict__ pw4 = reinterpret_cast<const float4*>(pw);
      for (int e0 = 0; e0 < nv; e0 += kSubThreads * kStageVec) {
        float4 v[kStageVec];
#pragma unroll
        for (int j = 0; j < kStageVec; ++j) {
          const int e = e0 + t + kSubThreads * j;
          if (e < nv) v[j] = pw4[(int64_t)s_map[e / R4] * R4 + e % R4];
        }
#pragma unroll
        for (int j = 0; j < kStageVec; ++j) {
          const int e = e0 + t + kSubThreads * j;
          if (e >= nv) continue;
          const int p = e / R4, c0 = (e % R4) * 4;
          const int cw = s_cw[p];
          const T xp = s_x[p];
          int r = c0 / w, q = c0 - r * w;
          const float vals[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int c = c0 + u;
            if (c < D * w) {
              const int l = q + ((cw >> (8 * r)) & 255) - (w - 1);  // cell s0 + l along r
              if (l >= 0 && l < ST) s_v[p * SS + r * ST + l] = r == 0 ? (T)vals[u] * xp : (T)vals[u];
            } else if (c >= wko && c < wko + NG) {
              s_v[p * SS + SW + c - wko] = (T)vals[u];
            }
            if (++q == w) {
              q = 0;
              ++r;
            }
          }
        }
      }
      __syncthreads();
    } else {
      __syncthreads();
      if (t < np) {
        const int2 ent = list[base + t];
        s_map[t] = ent.x;
        s_cw[t] = ent.y;
      }
      __syncthreads();
      // x of the lane's own point, loaded with the staging loads
      T xv = T(0);
      if (t < np) xv = (T)x[s_map[t]];
      // Items per lane: NW window items (e = p NW + r ST + l, e = t + 64 k) then
      // NG weight items (e = p NG + c, e = t + 64 (k - NW)).  Offsets into pw
      // are 32-bit (point sets whose rows exceed 4 GiB spread whole tiles).
#pragma unroll 1
      for (int k0 = 0; k0 < NW + NG; k0 += kStageChunk) {
        T vals[kStageChunk];
        int dst[kStageChunk];
#pragma unroll
        for (int j = 0; j < kStageChunk; ++j) {
          const int k = k0 + j;
          vals[j] = T(0);
          dst[j] = -1;
          if (k < NW) {
            const int e = t + kSubThreads * k;
            if (e < np * NW) {
              const int p = e / NW, rem = e % NW, r = rem / ST, l = rem % ST;
              const int q = l + w - 1 - ((s_cw[p] >> (8 * r)) & 255);  // window index of cell s0 + l
              dst[j] = p * SS + rem;
              if (q >= 0 && q < w)
                vals[j] = *reinterpret_cast<const T*>(
                    pwb + (uint32_t)(s_map[p] * rs + r * w + q) * (uint32_t)sizeof(T));
            }
          } else if (k < NW + NG) {
            const int e = t + kSubThreads * (k - NW);
            if (e < np * NG) {
              const int p = e / NG, c = e % NG;
              dst[j] = p * SS + SW + c;
              vals[j] = *reinterpret_cast<const T*>(
                  pwb + (uint32_t)(s_map[p] * rs + wko + c) * (uint32_t)sizeof(T));
            }
          }
        }
#pragma unroll
        for (int j = 0; j < kStageChunk; ++j)
          if (dst[j] >= 0) s_v[dst[j]] = vals[j];
      }
      __syncthreads();
      // dimension-0 window values times x_i; padding entries all zero
      if (t < np) {
#pragma unroll
        for (int l = 0; l < ST; ++l) s_v[t * SS + l] *= xv;
      } else if (t < np4) {
#pragma unroll
        for (int c = 0; c < SS; ++c) s_v[t * SS + c] = T(0);
      }
      __syncthreads();
    }
    for (int p = 0; p < np4; p += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const T* pv = s_v + (p + u) * SS;
        T v = pv[lx] * pv[ST + ly];
        if (D > 2) v *= pv[2 * ST + lz];
        const V* pg = reinterpret_cast<const V*>(pv + SW);
#pragma unroll
        for (int g = 0; g < GC; ++g) {
          const V wk = pg[g];
          acc[g].x += v * wk.x;
          acc[g].y += v * wk.y;
        }
      }
    }
  }
  if (!mine) return;
  const int64_t gi = a.grid_off + (int64_t)(s0[0] + lx) * a.gstride[0] +
                     (int64_t)(s0[1] + ly) * a.gstride[1] + (int64_t)(s0[2] + lz) * a.gstride[2];
#pragma unroll
  for (int g = 0; g < GC; ++g) grid[(int64_t)(a.g0 + g) * a.pair_stride + gi] = acc[g];
}

// ------------------------------------------------------------------ scan ----
// Exclusive prefix sum of counts into int64 offsets; 1024 elements per
// workgroup (4 per thread), the workgroup totals scanned the same way and
// added back.
constexpr int kScanThreads = 256, kScanPer = 4, kScanBlock = kScanThreads * kScanPer;
template <typename In>
__global__ __launch_bounds__(kScanThreads) void scan_block_kernel(const In* __restrict__ in, int64_t n,
                                                                  int64_t* __restrict__ out,
                                                                  int64_t* __restrict__ sums) {
  __shared__ int64_t s[kScanThreads];
  const int64_t b0 = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  int64_t v[kScanPer], tsum = 0;
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = b0 + k < n ? (int64_t)in[b0 + k] : 0;
    tsum += v[k];
  }
  s[threadIdx.x] = tsum;
  __syncthreads();
  for (int d = 1; d < kScanThreads; d *= 2) {
    const int64_t add = (int)threadIdx.x >= d ? s[threadIdx.x - d] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t run = s[threadIdx.x] - tsum;  // exclusive prefix of this thread
  for (int k = 0; k < kScanPer; ++k) {
    if (b0 + k < n) out[b0 + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = s[threadIdx.x];
}
__global__ __launch_bounds__(kScanThreads) void scan_add_kernel(int64_t* __restrict__ out, int64_t n,
                                                                const int64_t* __restrict__ offs) {
  const int64_t i = (int64_t)blockIdx.x * kScanThreads + threadIdx.x;
  if (i < n) out[i] += offs[i / kScanBlock];
}

// out[0..n) = exclusive prefix sums of in[0..n); *total = their sum (read back
// once at the end; plan time only).
template <typename In>
void exclusive_scan(const In* in, int64_t n, int64_t* out, hipStream_t s, int64_t* total) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  DevBuf sums, soff;
  sums.alloc((size_t)std::max<int64_t>(nb, 1) * sizeof(int64_t), s);
  if (n > 0) {
    hipLaunchKernelGGL((scan_block_kernel<In>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n,
                       out, sums.as<int64_t>());
    GP_CHECK_LAUNCH();
  }
  if (nb > 1) {
    soff.alloc((size_t)nb * sizeof(int64_t), s);
    int64_t sub_total = 0;
    exclusive_scan<int64_t>(sums.as<int64_t>(), nb, soff.as<int64_t>(), s, &sub_total);
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)((n + kScanThreads - 1) / kScanThreads)),
                       dim3(kScanThreads), 0, s, out, n, soff.as<int64_t>());
    GP_CHECK_LAUNCH();
    *total = sub_total;
    GP_HIP(hipStreamSynchronize(s));  // sums and soff are released on return
    return;
  }
  int64_t tv = 0;
  if (n > 0) GP_HIP(hipMemcpyAsync(&tv, sums.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  GP_HIP(hipStreamSynchronize(s));
  *total = tv;
}

// Runs CALL(GCV) with GCV the compile-time pair count equal to gc (1..8).
#define GP_SUB_GC_SWITCH(gc, CALL) \
  switch (gc) {                    \
    case 1: CALL(1); break;        \
    case 2: CALL(2); break;        \
    case 3: CALL(3); break;        \
    case 4: CALL(4); break;        \
    case 5: CALL(5); break;        \
    case 6: CALL(6); break;        \
    case 7: CALL(7); break;        \
    default: CALL(8); break;       \
  }

template <typename T, int D, int ST>
void launch_sub(Plan* P, const Records& R, const double* xs) {
  PhaseScope ps(P, PH_SPREAD);
  NuArgs a = nu_args(P, R);
  const int gc = std::min(kGCmax, P->npair);
  const int nch = (P->npair + gc - 1) / gc;
  // groups: the sub-tiles of one bin, or of two bins along dimension 0 in 3-D
  // (whose 8-cell rows of fp32 pairs are half a 128-byte line)
  int grp = 1;
  for (int r = 0; r < D; ++r) grp *= P->tile[r] / ST;
  if (D == 3 && P->nbins[0] % 2 == 0) grp *= 2;
  const int64_t nblk = (R.n_sub + 8 * grp - 1) / (8 * grp) * (8 * grp);
  auto* grid = static_cast<typename V2<T>::type*>(grid_a_current(P));
  for (int ch = 0; ch < nch; ++ch) {
    a.g0 = ch * gc;
    a.gc = std::min(gc, P->npair - a.g0);
#define GP_LAUNCH_SUB(GCV)                                                                         \
  hipLaunchKernelGGL((spread_list_kernel<T, D, ST, GCV>), dim3((unsigned)nblk), dim3(kSubThreads), \
                     0, P->stream, a, grp, R.n_sub, xs, R.pw.as<T>(), R.rs, R.sub_off.as<int64_t>(), \
                     R.sub_list.as<int2>(), grid)
    GP_SUB_GC_SWITCH(a.gc, GP_LAUNCH_SUB)
#undef GP_LAUNCH_SUB
    GP_CHECK_LAUNCH();
  }
}

template <typename T>
void launch_sub_t(Plan* P, const Records& R, const double* xs) {
  const int st = R.sub_st;
  if (P->d == 2 && st == 8) return launch_sub<T, 2, 8>(P, R, xs);
  if (P->d == 2 && st == 4) return launch_sub<T, 2, 4>(P, R, xs);
  if (P->d == 3 && st == 4) return launch_sub<T, 3, 4>(P, R, xs);
  if (P->d == 3 && st == 2) return launch_sub<T, 3, 2>(P, R, xs);
  throw Error{GP_EDEVICE, "internal: sub-tile side not compiled"};
}

}  // namespace

int spread_sub_side(const Plan* P) {
  if (P->spread_mode == GP_SPREAD_LDS_ATOMIC || P->d < 2 || P->precision != GP_FP32_BULK) return 0;
  int st = P->d == 2 ? 8 : 4;
  for (int r = 0; r < P->d; ++r) st = std::min(st, P->tile[r]);
  // compiled sides: 8, 4 in 2-D; 4, 2 in 3-D (smaller tiles spread whole tiles)
  if (st < (P->d == 2 ? 4 : 2)) return 0;
  return st;
}

size_t spread_list_bound_bytes(const Plan* P, int64_t n) {
  const int st = spread_sub_side(P);
  if (st == 0) return 0;
  int64_t per_point = 1, nsub = P->n_bins;
  for (int r = 0; r < P->d; ++r) {
    per_point *= (P->w - 2 + st) / st + 1;  // sub-tiles one window spans, at most
    nsub *= P->tile[r] / st;
  }
  return (size_t)n * per_point * sizeof(int2) + (size_t)(2 * nsub + 1) * sizeof(int64_t);
}

// The exact source lists of sub-tile spreading, built on the device from the
// sorted points: count per sub-tile, scan, fill (both passes visit the points
// in the same order, so the lists and every later sum are deterministic).
void build_spread_lists(Plan* P, Records& R) {
  R.n_sub = 0;
  const int st = spread_sub_side(P);
  if (st == 0) return;
  // the kernel addresses the point rows with 32-bit byte offsets; larger point
  // sets spread whole tiles
  const size_t ts = P->precision == GP_FP64 ? 8 : 4;
  if ((size_t)R.n * (size_t)R.rs * ts >= ((size_t)1 << 32)) return;
  hipStream_t s = P->stream;
  for (int r = 0; r < P->d; ++r)
    if (P->tile[r] % st != 0) throw Error{GP_EDEVICE, "internal: sub-tile does not divide the tile"};
  int64_t nsub = P->n_bins;
  for (int r = 0; r < P->d; ++r) nsub *= P->tile[r] / st;
  if (nsub > (int64_t)std::numeric_limits<int>::max() / 2) throw Error{GP_ENOMEM, "too many sub-tiles"};
  NuArgs a = nu_args(P, R);
  int nsrc_tot = 1;
  for (int r = 0; r < P->d; ++r) nsrc_tot *= P->nsrc;
  const size_t smem = (2 * (size_t)nsrc_tot + 1) * sizeof(int);
  DevBuf cnt;
  cnt.alloc((size_t)nsub * sizeof(int), P->stream);
  R.sub_off.alloc((size_t)(nsub + 1) * sizeof(int64_t), P->stream);
  if (P->d == 2)
    hipLaunchKernelGGL((spread_list_build_kernel<2, false>), dim3((unsigned)nsub), dim3(kSubThreads), smem,
                       s, a, st, R.cell.as<int>(), R.bin_start.as<int>(), cnt.as<int>(), nullptr, nullptr);
  else
    hipLaunchKernelGGL((spread_list_build_kernel<3, false>), dim3((unsigned)nsub), dim3(kSubThreads), smem,
                       s, a, st, R.cell.as<int>(), R.bin_start.as<int>(), cnt.as<int>(), nullptr, nullptr);
  GP_CHECK_LAUNCH();
  int64_t total = 0;
  exclusive_scan<int>(cnt.as<int>(), nsub, R.sub_off.as<int64_t>(), s, &total);
  GP_HIP(hipMemcpyAsync(R.sub_off.as<int64_t>() + nsub, &total, sizeof(int64_t), hipMemcpyHostToDevice, s));
  const size_t bound = spread_list_bound_bytes(P, R.n);
  if ((size_t)total * sizeof(int2) > bound) throw Error{GP_EDEVICE, "internal: sub-tile lists over their bound"};
  R.sub_list.alloc((size_t)std::max<int64_t>(total, 1) * sizeof(int2), P->stream);
  if (P->d == 2)
    hipLaunchKernelGGL((spread_list_build_kernel<2, true>), dim3((unsigned)nsub), dim3(kSubThreads), smem,
                       s, a, st, R.cell.as<int>(), R.bin_start.as<int>(), nullptr,
                       R.sub_off.as<int64_t>(), R.sub_list.as<int2>());
  else
    hipLaunchKernelGGL((spread_list_build_kernel<3, true>), dim3((unsigned)nsub), dim3(kSubThreads), smem,
                       s, a, st, R.cell.as<int>(), R.bin_start.as<int>(), nullptr,
                       R.sub_off.as<int64_t>(), R.sub_list.as<int2>());
  GP_CHECK_LAUNCH();
  GP_HIP(hipStreamSynchronize(s));  // &total is a host stack value
  R.n_sub = nsub;
  R.sub_st = st;
}

void exclusive_scan_counts(const int* in, int64_t n, int64_t* out, hipStream_t s, int64_t* total) {
  exclusive_scan<int>(in, n, out, s, total);
}

void spread_sub_launch(Plan* P, const Records& R, const double* xs) {
  if (R.n_sub <= 0) throw Error{GP_EDEVICE, "internal: sub-tile lists missing"};
  if (P->precision != GP_FP32_BULK || (P->d == 2 && R.rs % 4 != 0))
    throw Error{GP_EDEVICE, "internal: sub-tile spreading needs fp32 rows (padded to 16 bytes in 2-D)"};
  launch_sub_t<float>(P, R, xs);
}

}  // namespace gp
