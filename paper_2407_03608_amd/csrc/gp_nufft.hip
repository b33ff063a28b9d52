// The matvec y = K~ x of section 4.2 on gfx950.
//
//  step 1+2a  spread_kernel   c_{k,i} = w_k(x_i) x_i (eq:c) spread onto the fine
//                             grids with the exponential-of-semicircle window
//  step 2b    fft passes      forward FFT of every grid (pruned)
//  step 3     mode_kernel     a_k'[n] = sum_j v~_j G^_k'j[n] sum_k G^_kj[n] b_k[n]
//                             with the window deconvolution folded in
//  step 4a    fft passes      inverse FFT (pruned)
//  step 4b+5  interp_kernel   beta_{k,i} by interpolation, y_i = sum_k w_k(x_i) beta_{k,i}
//                             (+ eta^2 x_i)
//
// Real grids travel in complex pairs: grid 2g is the real part and grid 2g+1
// the imaginary part of complex grid g, so every FFT is complex-to-complex and
// the mode kernel separates the two spectra with b(n) = (Z(n) + conj Z(-n))/2.
//
// Spreading is a gather: each workgroup owns one tile (or sub-tile) of the
// active fine grid, collects every point whose window reaches it (the points
// are bin-sorted by the tile of their first window cell, so the sources are
// the 2^d (or more) neighbouring bins), and each thread sums the contributions
// to the cells it owns in registers (owner-computes: no atomics, a fixed
// summation order) before writing them with plain coalesced stores.  No global
// atomics and no zero-fill pass.  An LDS-atomic variant (per-(point, row)
// items) is kept as an option.
#include <algorithm>
#include <climits>
#include <cmath>
#include <limits>
#include <mutex>

#include "gp_internal.h"

namespace gp {

void mix_modes_fp64(Plan* P);
void mix_modes_fp32(Plan* P);
static void mix_modes(Plan* P) {
  if (P->precision == GP_FP64)
    mix_modes_fp64(P);
  else
    mix_modes_fp32(P);
}

namespace {

template <typename T> struct V2;
template <> struct V2<double> { using type = double2; };
template <> struct V2<float> { using type = float2; };

constexpr int kThreads = 256;
constexpr int kPB = 64;      // points staged per batch
constexpr int kGC = 8;       // max complex grids per chunk
constexpr int kRG = 4;       // interpolation row groups per (point, grid pair)


// Points are staged in LDS in batches of kPB: the first window cell per
// dimension, the point's row of window values and weights (padded to an odd
// stride so that lanes reading different points hit different banks) and x_i.
__host__ __device__ constexpr int lds_stride(int rs) { return rs | 1; }

// ---------------------------------------------------------- spread (owner) ----
// Owner-computes variant: each thread owns CPT cells of the tile and, for every
// staged source point, adds its contribution to the grid pairs of the chunk in
// registers when the point's window covers the cell.  No atomics, so the
// summation order (and the result) is fixed.
//
// A crowded tile is split into chunks of its source points (work item
// {tile, lo, hi, slot}); each chunk writes a partial tile to `part`, and
// spread_reduce_kernel adds the partials in slot order.
template <typename T, int D, int CPT, int GC>
__global__ __launch_bounds__(kThreads) void spread_owner_kernel(
    NuArgs a, const double* __restrict__ x, const int* __restrict__ cell,
    const T* __restrict__ pw, int rs, const int* __restrict__ bin_start,
    const int4* __restrict__ work, typename V2<T>::type* __restrict__ part,
    typename V2<T>::type* __restrict__ grid) {
  using V = typename V2<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tc0 = a.tile[0], tc1 = D > 1 ? a.tile[1] : 1;
  const int ls = lds_stride(rs);
  T* s_rec = reinterpret_cast<T*>(smem);          // [kPB][ls]
  T* s_x = s_rec + kPB * ls;                      // [kPB]
  int* s_cell = reinterpret_cast<int*>(s_x + kPB);  // [kPB][D]
  int* s_map = s_cell + kPB * D;                    // [kPB] staged point -> sorted index
  int* s_np = s_map + kPB;                          // staged count

  // no work list: one item per tile, all of its sources, written to the grid
  const int4 wk = work ? work[blockIdx.x] : make_int4((int)blockIdx.x, 0, INT_MAX, -1);
  const int src_lo = wk.y, src_hi = wk.z, slot = wk.w;
  int tcoord[3] = {0, 0, 0}, t0[3] = {0, 0, 0};
  {
    int64_t tb = wk.x;
    for (int r = 0; r < D; ++r) {
      tcoord[r] = (int)(tb % a.nbins[r]);
      tb /= a.nbins[r];
      t0[r] = tcoord[r] * a.tile[r];
    }
  }
  // my cells (absolute active-box coordinates)
  const int tcells = tc0 * tc1 * (D > 2 ? a.tile[2] : 1);
  int cx[CPT], cy[CPT], cz[CPT];
  bool mine[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    int l = threadIdx.x + c * kThreads;
    mine[c] = l < tcells;
    if (!mine[c]) l = 0;
    cx[c] = t0[0] + l % tc0;
    l /= tc0;
    cy[c] = D > 1 ? t0[1] + l % tc1 : 0;
    cz[c] = D > 2 ? t0[2] + l / tc1 : 0;
  }
  V acc[CPT][GC];
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int g = 0; g < GC; ++g) acc[c][g] = V{T(0), T(0)};

  const int w = a.w;
  const int wko = D * w + 2 * a.g0;
  int nsrc_tot = 1;
  for (int r = 0; r < D; ++r) nsrc_tot *= a.nsrc;
  // The tile's source sequence: its source bins in order (offset q along each
  // dimension, first dimension fastest; bins before the grid start skipped),
  // concatenated.  Thread sb < nsrc_tot records bin sb's range and the
  // dimensions along which it lies before the tile.
  int* s_sb0 = s_np + 1;                  // [nsrc_tot] first sorted index
  int* s_soff = s_sb0 + nsrc_tot;         // [nsrc_tot + 1] offsets in the sequence
  int* s_smask = s_soff + nsrc_tot + 1;   // [nsrc_tot] offset-dimension mask
  for (int sb = threadIdx.x; sb < nsrc_tot; sb += kThreads) {
    int64_t bin = 0, mul = 1;
    bool ok = true;
    int q = sb, mask = 0;
    for (int r = 0; r < D; ++r) {
      const int dq = q % a.nsrc;
      const int br = tcoord[r] - dq;
      q /= a.nsrc;
      if (dq) mask |= 1 << r;
      if (br < 0) ok = false;
      bin += (int64_t)br * mul;
      mul *= a.nbins[r];
    }
    const int b0 = ok ? bin_start[bin] : 0;
    s_sb0[sb] = b0;
    s_soff[sb + 1] = ok ? bin_start[bin + 1] - b0 : 0;  // count, summed below
    s_smask[sb] = mask;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    s_soff[0] = 0;
    for (int sb = 0; sb < nsrc_tot; ++sb) s_soff[sb + 1] += s_soff[sb];
  }
  __syncthreads();
  const int seq_lo = max(src_lo, 0), seq_hi = min(src_hi, s_soff[nsrc_tot]);
  // Windows of kPB consecutive candidates of the sequence.  Along a dimension
  // where a candidate's bin lies before the tile, the point reaches the tile
  // only if the last cell of its window does: wave 0 filters each window and
  // compacts the survivors (ballot), so only they are staged and tested by
  // every thread.  The order of the survivors is the sequence order.
  for (int base = seq_lo; base < seq_hi; base += kPB) {
    {
      const int nc = min(kPB, seq_hi - base);
      __syncthreads();
      if (threadIdx.x < kPB) {  // wave 0 (kPB is the wavefront size)
        bool keep = (int)threadIdx.x < nc;
        int idx = 0;
        if (keep) {
          const int qpos = base + threadIdx.x;
          int sb = 0;
          while (qpos >= s_soff[sb + 1]) ++sb;
          idx = s_sb0[sb] + (qpos - s_soff[sb]);
          const int mask = s_smask[sb];
          if (mask)
            for (int r = 0; r < D; ++r)
              if ((mask >> r) & 1) keep = keep && cell[r * a.n + idx] + w - 1 >= t0[r];
        }
        const unsigned long long m = __ballot(keep);
        if (keep) s_map[__popcll(m & ((1ull << threadIdx.x) - 1ull))] = idx;
        if (threadIdx.x == 0) *s_np = __popcll(m);
      }
      __syncthreads();
      const int np = *s_np;
      if (np == 0) continue;
      for (int e = threadIdx.x; e < np * rs; e += kThreads) {
        const int p = e / rs, c = e - p * rs;
        s_rec[p * ls + c] = pw[(int64_t)s_map[p] * rs + c];
      }
      if (threadIdx.x < np) {
        const int i = s_map[threadIdx.x];
        s_x[threadIdx.x] = (T)x[i];
        for (int r = 0; r < D; ++r) s_cell[threadIdx.x * D + r] = cell[r * a.n + i];
      }
      __syncthreads();
      for (int p = 0; p < np; ++p) {
        const T* pr = s_rec + p * ls;
        const int s0 = s_cell[p * D];
        const int s1 = D > 1 ? s_cell[p * D + 1] : 0;
        const int s2 = D > 2 ? s_cell[p * D + 2] : 0;
        const T xa = s_x[p];
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          const unsigned d0 = (unsigned)(cx[c] - s0);
          const unsigned d1 = (unsigned)(cy[c] - s1);
          const unsigned d2 = (unsigned)(cz[c] - s2);
          bool hit = d0 < (unsigned)w;
          if (D > 1) hit = hit && d1 < (unsigned)w;
          if (D > 2) hit = hit && d2 < (unsigned)w;
          if (hit) {
            T v = pr[d0] * xa;
            if (D > 1) v *= pr[w + d1];
            if (D > 2) v *= pr[2 * w + d2];
#pragma unroll
            for (int g = 0; g < GC; ++g) {
              acc[c][g].x += v * pr[wko + 2 * g];
              acc[c][g].y += v * pr[wko + 2 * g + 1];
            }
          }
        }
      }
    }
  }
  // write my cells (the tile, or this chunk's partial tile, is exclusively owned)
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    if (!mine[c]) continue;
    if (slot >= 0) {
      const int l = threadIdx.x + c * kThreads;
#pragma unroll
      for (int g = 0; g < GC; ++g) part[((int64_t)slot * a.slot_pairs + g) * tcells + l] = acc[c][g];
      continue;
    }
    const int64_t gi = a.grid_off + (int64_t)cx[c] * a.gstride[0] + (int64_t)cy[c] * a.gstride[1] +
                       (int64_t)cz[c] * a.gstride[2];
#pragma unroll
    for (int g = 0; g < GC; ++g) grid[(int64_t)(a.g0 + g) * a.pair_stride + gi] = acc[c][g];
  }
}

// Tiles split into chunks: grid tile = sum of the chunks' partial tiles, added
// in chunk order.  One workgroup per split tile ({tile, slot0, count}).
template <typename T, int D>
__global__ __launch_bounds__(kThreads) void spread_reduce_kernel(
    NuArgs a, const int4* __restrict__ red, const typename V2<T>::type* __restrict__ part,
    typename V2<T>::type* __restrict__ grid) {
  using V = typename V2<T>::type;
  const int4 wk = red[blockIdx.x];
  const int tc0 = a.tile[0], tc1 = D > 1 ? a.tile[1] : 1;
  const int tcells = tc0 * tc1 * (D > 2 ? a.tile[2] : 1);
  int t0[3] = {0, 0, 0};
  {
    int64_t tb = wk.x;
    for (int r = 0; r < D; ++r) {
      t0[r] = (int)(tb % a.nbins[r]) * a.tile[r];
      tb /= a.nbins[r];
    }
  }
  for (int e = threadIdx.x; e < a.gc * tcells; e += kThreads) {
    const int g = e / tcells, l = e - g * tcells;
    V v = V{T(0), T(0)};
    for (int j = 0; j < wk.z; ++j) {
      const V u = part[((int64_t)(wk.y + j) * a.slot_pairs + g) * tcells + l];
      v.x += u.x;
      v.y += u.y;
    }
    const int c0 = t0[0] + l % tc0;
    const int c1 = D > 1 ? t0[1] + (l / tc0) % tc1 : 0;
    const int c2 = D > 2 ? t0[2] + l / (tc0 * tc1) : 0;
    const int64_t gi = a.grid_off + (int64_t)c0 * a.gstride[0] + (int64_t)c1 * a.gstride[1] +
                       (int64_t)c2 * a.gstride[2];
    grid[(int64_t)(a.g0 + g) * a.pair_stride + gi] = v;
  }
}

// ---------------------------------------------------------------- spread ----
// One workgroup per tile of the active grid and chunk of complex grids.  The
// sources are the bins whose points' windows can reach the tile (nsrc per
// dimension).  Work items are (point, window row, grid pair); each adds its
// row of w cells into the LDS tile with LDS atomics.
template <typename T, int D>
__global__ __launch_bounds__(kThreads) void spread_kernel(
    NuArgs a, const double* __restrict__ x, const int* __restrict__ cell,
    const T* __restrict__ pw, int rs, const int* __restrict__ bin_start,
    typename V2<T>::type* __restrict__ grid) {
  using V = typename V2<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tc0 = a.tile[0], tc1 = D > 1 ? a.tile[1] : 1, tc2 = D > 2 ? a.tile[2] : 1;
  const int tcells = tc0 * tc1 * tc2;
  const int ls = lds_stride(rs);
  V* acc = reinterpret_cast<V*>(smem);
  T* s_rec = reinterpret_cast<T*>(acc + (size_t)a.gc * tcells);  // [kPB][ls]
  T* s_x = s_rec + kPB * ls;                                      // [kPB]
  int* s_cell = reinterpret_cast<int*>(s_x + kPB);                // [kPB][D]

  int tcoord[3] = {0, 0, 0}, t0[3] = {0, 0, 0};
  {
    int64_t tb = blockIdx.x;
    for (int r = 0; r < D; ++r) {
      tcoord[r] = (int)(tb % a.nbins[r]);
      tb /= a.nbins[r];
      t0[r] = tcoord[r] * a.tile[r];
    }
  }
  for (int e = threadIdx.x; e < a.gc * tcells; e += kThreads) acc[e] = V{T(0), T(0)};

  const int w = a.w;
  const int wko = D * w + 2 * a.g0;  // offset of w_{2 g0} in a row
  int nsrc_tot = 1;
  for (int r = 0; r < D; ++r) nsrc_tot *= a.nsrc;
  int rows = 1;
  for (int r = 1; r < D; ++r) rows *= w;

  for (int sb = 0; sb < nsrc_tot; ++sb) {
    int64_t bin = 0, mul = 1;
    bool ok = true;
    int q = sb;
    for (int r = 0; r < D; ++r) {
      int br = tcoord[r] - (q % a.nsrc);
      q /= a.nsrc;
      if (br < 0) ok = false;
      bin += (int64_t)br * mul;
      mul *= a.nbins[r];
    }
    if (!ok) continue;
    const int p0 = bin_start[bin], p1 = bin_start[bin + 1];
    for (int pb = p0; pb < p1; pb += kPB) {
      const int np = min(kPB, p1 - pb);
      __syncthreads();  // previous batch (or the tile clear) done
      for (int e = threadIdx.x; e < np * rs; e += kThreads) {
        const int p = e / rs;
        s_rec[p * ls + (e - p * rs)] = pw[(int64_t)pb * rs + e];
      }
      if (threadIdx.x < np) {
        s_x[threadIdx.x] = (T)x[pb + threadIdx.x];
        for (int r = 0; r < D; ++r) s_cell[threadIdx.x * D + r] = cell[r * a.n + pb + threadIdx.x];
      }
      __syncthreads();
      const int nitems = np * rows * a.gc;
      for (int it = threadIdx.x; it < nitems; it += kThreads) {
        const int p = it % np;
        const int rest = it / np;
        const int row = rest % rows;
        const int g = rest / rows;
        const T* pr = s_rec + p * ls;
        int loc1 = 0, loc2 = 0;
        T wv = T(1);
        bool inside = true;
        if (D > 1) {
          const int q1 = row % w;
          loc1 = s_cell[p * D + 1] + q1 - t0[1];
          inside = inside && loc1 >= 0 && loc1 < tc1;
          wv *= pr[w + q1];
        }
        if (D > 2) {
          const int q2 = row / w;
          loc2 = s_cell[p * D + 2] + q2 - t0[2];
          inside = inside && loc2 >= 0 && loc2 < tc2;
          wv *= pr[2 * w + q2];
        }
        if (!inside) continue;
        const T xa = s_x[p];
        const T c0 = pr[wko + 2 * g] * xa * wv, c1 = pr[wko + 2 * g + 1] * xa * wv;
        const int base0 = s_cell[p * D] - t0[0];
        V* accg = acc + (size_t)g * tcells + (loc2 * tc1 + loc1) * tc0;
        const int qa = max(0, -base0), qb = min(w, tc0 - base0);
        for (int q0 = qa; q0 < qb; ++q0) {
          const T v = pr[q0];
          atomicAdd(&accg[base0 + q0].x, c0 * v);
          atomicAdd(&accg[base0 + q0].y, c1 * v);
        }
      }
    }
  }
  __syncthreads();
  // write the tile (exclusively owned: plain stores)
  for (int e = threadIdx.x; e < a.gc * tcells; e += kThreads) {
    const int g = e / tcells;
    int c = e - g * tcells;
    const int l0 = c % tc0;
    c /= tc0;
    const int l1 = c % tc1;
    const int l2 = c / tc1;
    const int64_t gi = a.grid_off + (int64_t)(t0[0] + l0) * a.gstride[0] +
                       (int64_t)(t0[1] + l1) * a.gstride[1] + (int64_t)(t0[2] + l2) * a.gstride[2];
    grid[(int64_t)(a.g0 + g) * a.pair_stride + gi] = acc[e];
  }
}

// ------------------------------------------------------- interp (gather) ----
// One thread per point: sums its w^d window of every grid pair straight from
// the cache hierarchy (points are bin-sorted, so neighbouring threads read
// overlapping windows) and forms sum_k w_k beta_k (+ eta^2 x_i).
template <typename T, int D, int WT>
__global__ __launch_bounds__(kThreads) void interp_gather_kernel(
    NuArgs a, const typename V2<T>::type* __restrict__ grid, const int* __restrict__ cell,
    const T* __restrict__ pw, int rs, const double* __restrict__ x, double* __restrict__ y) {
  using V = typename V2<T>::type;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= a.n) return;
  const int w = a.w;
  const T* pr = pw + i * rs;
  T p0[WT], p1[WT], p2[WT];
#pragma unroll
  for (int q = 0; q < WT; ++q) {
    p0[q] = q < w ? pr[q] : T(0);
    p1[q] = (D > 1 && q < w) ? pr[w + q] : T(0);
    p2[q] = (D > 2 && q < w) ? pr[2 * w + q] : T(0);
  }
  const int64_t base = a.grid_off + (int64_t)cell[i] * a.gstride[0] +
                       (D > 1 ? (int64_t)cell[a.n + i] * a.gstride[1] : 0) +
                       (D > 2 ? (int64_t)cell[2 * a.n + i] * a.gstride[2] : 0);
  double out = a.add_noise ? a.eta2 * x[i] : 0.0;
  const int n1 = D > 1 ? w : 1, n2 = D > 2 ? w : 1;
  for (int g = 0; g < a.npair; ++g) {
    const V* gp = grid + (int64_t)g * a.pair_stride + base;
    T sx = 0, sy = 0;
    for (int q2 = 0; q2 < n2; ++q2) {
      for (int q1 = 0; q1 < n1; ++q1) {
        T wv = T(1);
        if (D > 1) wv = p1[q1];
        if (D > 2) wv *= p2[q2];
        const V* row = gp + (D > 1 ? (int64_t)q1 * a.gstride[1] : 0) + (D > 2 ? (int64_t)q2 * a.gstride[2] : 0);
        T rx = 0, ry = 0;
#pragma unroll
        for (int q0 = 0; q0 < WT; ++q0) {
          if (q0 < w) {
            const V v = row[q0];
            rx += p0[q0] * v.x;
            ry += p0[q0] * v.y;
          }
        }
        sx += wv * rx;
        sy += wv * ry;
      }
    }
    out += (double)pr[D * w + 2 * g] * (double)sx + (double)pr[D * w + 2 * g + 1] * (double)sy;
  }
  y[i] = out;
}

// ---------------------------------------------------------------- interp ----
// One workgroup per bin.  For each chunk of complex grids the bin's tile plus
// its (w-1) halo is staged in LDS; every (point, grid pair) item sums its
// window and adds w_2g beta_2g + w_2g+1 beta_2g+1 to the point's accumulator.
template <typename T, int D>
__global__ __launch_bounds__(kThreads) void interp_kernel(
    NuArgs a, const typename V2<T>::type* __restrict__ grid, const int* __restrict__ cell,
    const T* __restrict__ pw, int rs, const int4* __restrict__ work,
    const double* __restrict__ x, double* __restrict__ y) {
  using V = typename V2<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  const int w = a.w;
  const int pc0 = a.tile[0] + w - 1;
  const int pc1 = D > 1 ? a.tile[1] + w - 1 : 1;
  const int pc2 = D > 2 ? a.tile[2] + w - 1 : 1;
  // tile rows padded to an odd number of cells: the RG lanes of one item group
  // read RG consecutive rows, which then fall in different LDS banks
  const int ps0 = pc0 | 1;
  const int pcells = ps0 * pc1 * pc2;
  const int ls = lds_stride(rs);
  V* tileA = reinterpret_cast<V*>(smem);                                  // [gc][pcells]
  T* s_rec = reinterpret_cast<T*>(tileA + (size_t)a.gc * pcells);         // [kPB][ls]
  // per-(point, grid pair) partial sums, reduced in a fixed order
  double* s_part = reinterpret_cast<double*>(s_rec + kPB * ls);  // [kPB][kGC] (8-B aligned)
  int* s_cell = reinterpret_cast<int*>(s_part + kPB * kGC);      // [kPB][D]

  const int4 wk = work[blockIdx.x];  // {bin, p_lo, p_hi}: one chunk of the bin's points
  const int p0 = wk.y, p1 = wk.z;
  int t0[3] = {0, 0, 0};
  {
    int64_t tb = wk.x;
    for (int r = 0; r < D; ++r) {
      t0[r] = (int)(tb % a.nbins[r]) * a.tile[r];
      tb /= a.nbins[r];
    }
  }
  const int ucells = pc0 * pc1 * pc2;
  for (int e = threadIdx.x; e < a.gc * ucells; e += kThreads) {
    const int g = e / ucells;
    int c = e - g * ucells;
    const int l0 = c % pc0;
    c /= pc0;
    const int l1 = c % pc1;
    const int l2 = c / pc1;
    V v = V{T(0), T(0)};
    const int c0 = t0[0] + l0, c1 = t0[1] + l1, c2 = t0[2] + l2;
    if (c0 < a.na[0] && (D < 2 || c1 < a.na[1]) && (D < 3 || c2 < a.na[2]))
      v = grid[(int64_t)(a.g0 + g) * a.pair_stride + a.grid_off + (int64_t)c0 * a.gstride[0] +
               (int64_t)c1 * a.gstride[1] + (int64_t)c2 * a.gstride[2]];
    tileA[(size_t)g * pcells + (l2 * pc1 + l1) * ps0 + l0] = v;
  }
  const int wko = D * w + 2 * a.g0;
  int cellsw = 1;
  for (int r = 1; r < D; ++r) cellsw *= w;
  // row groups per item: a power of two, so that a group is RG adjacent lanes
  const int RG = cellsw >= kRG ? kRG : (cellsw >= 2 ? 2 : 1);
  for (int pb = p0; pb < p1; pb += kPB) {
    const int np = min(kPB, p1 - pb);
    __syncthreads();
    for (int e = threadIdx.x; e < np * rs; e += kThreads) {
      const int p = e / rs;
      s_rec[p * ls + (e - p * rs)] = pw[(int64_t)pb * rs + e];
    }
    if (threadIdx.x < np)
      for (int r = 0; r < D; ++r) s_cell[threadIdx.x * D + r] = cell[r * a.n + pb + threadIdx.x] - t0[r];
    __syncthreads();
    // items: (row group, point, grid pair) with the row group fastest; a row
    // group takes window rows rg, rg + RG, ... and the RG lanes of an item
    // combine their shares of w_2g beta_2g + w_2g+1 beta_2g+1 by xor shuffles
    // (kThreads and nitems are multiples of RG, so a group is all active or
    // all inactive)
    const int nitems = np * a.gc * RG;
    for (int it = threadIdx.x; it < nitems; it += kThreads) {
      const int rg = it % RG;
      const int rest = it / RG;
      const int p = rest % np;
      const int g = rest / np;
      const T* pr = s_rec + p * ls;
      double part = 0.0;
      for (int row = rg; row < cellsw; row += RG) {
        T wv = T(1);
        int off = s_cell[p * D];
        if (D > 1) {
          const int q1 = row % w;
          wv *= pr[w + q1];
          off += (s_cell[p * D + 1] + q1) * ps0;
        }
        if (D > 2) {
          const int q2 = row / w;
          wv *= pr[2 * w + q2];
          off += (s_cell[p * D + 2] + q2) * ps0 * pc1;
        }
        const V* tr = tileA + (size_t)g * pcells + off;
        T rx = 0, ry = 0;
        for (int q0 = 0; q0 < w; ++q0) {
          const T ps = pr[q0];
          const V gv = tr[q0];
          rx += ps * gv.x;
          ry += ps * gv.y;
        }
        part += (double)wv * ((double)pr[wko + 2 * g] * (double)rx + (double)pr[wko + 2 * g + 1] * (double)ry);
      }
      if (RG >= 2) part += __shfl_xor(part, 1);
      if (RG >= 4) part += __shfl_xor(part, 2);
      if (rg == 0) s_part[p * kGC + g] = part;
    }
    __syncthreads();
    if (threadIdx.x < np) {
      const int p = threadIdx.x;
      double sum = 0.0;
      for (int g = 0; g < a.gc; ++g) sum += s_part[p * kGC + g];
      const int64_t i = pb + p;
      const double base = a.first_chunk ? (a.add_noise ? a.eta2 * x[i] : 0.0) : y[i];
      y[i] = base + sum;
    }
  }
}

// ------------------------------------------------- interp (2x2 super-tile) ----
// d = 2, 3.  One workgroup per chunk of the points of a 2x2(x1) block of bins: the
// block's cells plus the (w-1) halo are staged in LDS for one grid pair at a
// time (halo overhead (2t+w-1)^2/(2t)^2 instead of (t+w-1)^2/t^2 per bin), the
// points' rows are staged once, and each thread keeps its items' partial sums
// over all pairs in registers.  Items are (row group, point), row group
// fastest; the RG lanes of a point combine by xor shuffles at the end, so the
// order of every sum is fixed.  The next pair's tile is loaded into registers
// while the current pair is computed (the kernel is otherwise latency-bound:
// 1.71 -> 0.88 ms at d=2 N=1e6 fp64 on the 8192^2 grid).
// Points staged per batch: 128 for fp32 grids (in 3-D the 2x2x1 block of
// 20 x 20 x 12 cells at w = 5 and the rows then take 49 KB, three workgroups
// per CU: d=3 N=1e7 3.19 -> 2.71 ms against 320 points per batch at 80 KB,
// although the block is staged more often); 64 for fp64 grids, whose rows of
// 38 doubles per point would otherwise hold two workgroups per CU (d=2 N=1e6:
// three, with the block staged about twice as often, 0.79 -> 0.70 ms).
template <int D, typename T>
constexpr int kPB2 = sizeof(T) == 8 ? 64 : 128;

// tile cells per thread kept in flight by the pipelined variant (a d=3 block
// of 2x2x1 bins of 8^3 cells with w = 5 has 20 x 20 x 12 = 4800 cells)
template <int D>
constexpr int kTE = D > 2 ? 20 : 8;

// W > 0: the window width as a compile-time constant (inner loops unrolled);
// W = 0 reads it from the arguments.
template <typename T, bool PIPE, int D, int W>
__global__ __launch_bounds__(kThreads) void interp_super_kernel(
    NuArgs a, const typename V2<T>::type* __restrict__ grid, const int* __restrict__ cell,
    const T* __restrict__ pw, int rs, const int* __restrict__ bin_start,
    const int4* __restrict__ work, const double* __restrict__ x, double* __restrict__ y,
    int64_t nwork, int grp) {
  using V = typename V2<T>::type;
  constexpr int PB = kPB2<D, T>;
  constexpr int NI = (PB * kRG + kThreads - 1) / kThreads;  // items per thread
  extern __shared__ __align__(16) unsigned char smem[];
  const int w = W > 0 ? W : a.w;
  // blocks of 2 x 2 (x 1) bins: the first two dimensions doubled
  const int st0 = 2 * a.tile[0], st1 = 2 * a.tile[1], st2 = D > 2 ? a.tile[2] : 1;
  const int pc0 = st0 + w - 1, pc1 = st1 + w - 1, pc2 = D > 2 ? st2 + w - 1 : 1;
  const int ps0 = pc0 | 1;  // odd row stride: the RG lanes of a point hit different banks
  const int ls = lds_stride(rs);
  V* tile = reinterpret_cast<V*>(smem);                              // [pc2][pc1][ps0]
  T* s_rec = reinterpret_cast<T*>(tile + (size_t)ps0 * pc1 * pc2);   // [PB][ls]
  int* s_cell = reinterpret_cast<int*>(s_rec + PB * ls);           // [PB][D]
  int* s_idx = s_cell + D * PB;                                     // [PB] sorted index

  // block -> work item: groups of grp consecutive items per XCD (blocks go to
  // the XCDs round-robin); the grid is padded to a multiple of 8 grp
  int64_t item = blockIdx.x;
  if (grp > 0) {
    const int64_t xx = item % 8, k = item / 8;
    item = ((k / grp) * 8 + xx) * grp + k % grp;
    if (item >= nwork) return;
  }
  const int4 wk = work[item];
  const int nsb0 = (a.nbins[0] + 1) / 2, nsb1 = (a.nbins[1] + 1) / 2;
  const int sx = wk.x % nsb0, sy = (wk.x / nsb0) % nsb1, sz = D > 2 ? wk.x / (nsb0 * nsb1) : 0;
  const int t00 = sx * st0, t01 = sy * st1, t02 = sz * st2;
  const int bx0 = 2 * sx, bx1 = min(2 * sx + 1, a.nbins[0] - 1);
  int r_lo[2] = {0, 0}, r_len0 = 0;
  for (int q = 0; q < 2; ++q) {
    const int by = 2 * sy + q;
    if (by >= a.nbins[1]) break;
    const int64_t rowbin = ((int64_t)sz * a.nbins[1] + by) * a.nbins[0];
    r_lo[q] = bin_start[rowbin + bx0];
    if (q == 0) r_len0 = bin_start[rowbin + bx1 + 1] - r_lo[0];
  }
  const int cellsw = D > 2 ? w * w : w;  // window rows per point
  const int RG = cellsw >= kRG ? kRG : (cellsw >= 2 ? 2 : 1);  // power of two; kThreads % RG == 0
  const int wko = D * w;
  for (int pos = wk.y; pos < wk.z; pos += PB) {
    const int np = min(PB, wk.z - pos);
    __syncthreads();
    for (int e = threadIdx.x; e < np; e += kThreads) {
      const int q = pos + e;
      const int idx = q < r_len0 ? r_lo[0] + q : r_lo[1] + (q - r_len0);
      s_idx[e] = idx;
      s_cell[D * e] = cell[idx] - t00;
      s_cell[D * e + 1] = cell[a.n + idx] - t01;
      if (D > 2) s_cell[D * e + 2] = cell[2 * a.n + idx] - t02;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < np * rs; e += kThreads) {
      const int p = e / rs, c = e - p * rs;
      s_rec[p * ls + c] = pw[(int64_t)s_idx[p] * rs + c];
    }
    double part[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) part[k] = 0.0;
    const int nitems = np * RG;
    const int ucells = pc0 * pc1 * pc2;
    // PIPE: the next pair's tile is loaded into registers while this pair is
    // computed, and stored to LDS after the barrier (ucells <= kTE kThreads)
    V nxt[PIPE ? kTE<D> : 1];
    auto load_tile = [&](int g) {
#pragma unroll
      for (int j = 0; j < (PIPE ? kTE<D> : 1); ++j) {
        const int e = threadIdx.x + j * kThreads;
        V v = V{T(0), T(0)};
        if (e < ucells) {
          const int l12 = e / pc0, l0 = e - l12 * pc0;
          const int l1 = D > 2 ? l12 % pc1 : l12, l2 = D > 2 ? l12 / pc1 : 0;
          const int c0 = t00 + l0, c1 = t01 + l1, c2 = t02 + l2;
          if (c0 < a.na[0] && c1 < a.na[1] && (D < 3 || c2 < a.na[2]))
            v = grid[(int64_t)g * a.pair_stride + a.grid_off + (int64_t)c0 * a.gstride[0] +
                     (int64_t)c1 * a.gstride[1] + (D > 2 ? (int64_t)c2 * a.gstride[2] : 0)];
        }
        nxt[j] = v;
      }
    };
    if (PIPE) load_tile(0);
    for (int g = 0; g < a.npair; ++g) {
      __syncthreads();  // records staged / previous pair's tile no longer read
      if (PIPE) {
#pragma unroll
        for (int j = 0; j < (PIPE ? kTE<D> : 1); ++j) {
          const int e = threadIdx.x + j * kThreads;
          if (e < ucells) {
            const int l12 = e / pc0, l0 = e - l12 * pc0;
            tile[l12 * ps0 + l0] = nxt[j];
          }
        }
        if (g + 1 < a.npair) load_tile(g + 1);
      } else {
        // cell (l0, l1, l2) of the thread's e, stepped by kThreads = s12 rows + s0 cells
        const int s12 = kThreads / pc0, s0 = kThreads - s12 * pc0;
        int l0 = threadIdx.x % pc0, l1 = threadIdx.x / pc0, l2 = 0;
        while (l1 >= pc1) { l1 -= pc1; ++l2; }
        for (int e = threadIdx.x; e < ucells; e += kThreads) {
          const int c0 = t00 + l0, c1 = t01 + l1, c2 = t02 + l2;
          V v = V{T(0), T(0)};
          if (c0 < a.na[0] && c1 < a.na[1] && (D < 3 || c2 < a.na[2]))
            v = grid[(int64_t)g * a.pair_stride + a.grid_off + (int64_t)c0 * a.gstride[0] +
                     (int64_t)c1 * a.gstride[1] + (D > 2 ? (int64_t)c2 * a.gstride[2] : 0)];
          tile[(l2 * pc1 + l1) * ps0 + l0] = v;
          l0 += s0;
          l1 += s12;
          if (l0 >= pc0) { l0 -= pc0; ++l1; }
          while (l1 >= pc1) { l1 -= pc1; ++l2; }
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        const int it = threadIdx.x + k * kThreads;
        if (it < nitems) {
          const int rg = it % RG, p = it / RG;
          const T* pr = s_rec + p * ls;
          const int o0 = s_cell[D * p], o1 = s_cell[D * p + 1], o2 = D > 2 ? s_cell[D * p + 2] : 0;
          // beta_2g, beta_2g+1 over this item's window rows, then weighted in fp64
          T sx = 0, sy = 0;
          // window row (q1, q2) of row index q2 w + q1, stepped by RG < w
          int q1 = D > 2 ? (rg < w ? rg : rg - w) : rg, q2 = D > 2 && rg >= w ? 1 : 0;
          for (int row = rg; row < cellsw; row += RG) {
            const V* tr = tile + ((o2 + q2) * pc1 + (o1 + q1)) * ps0 + o0;
            T rx = 0, ry = 0;
            if constexpr (W > 0) {
#pragma unroll
              for (int q0 = 0; q0 < W; ++q0) {
                const T ps = pr[q0];
                const V gv = tr[q0];
                rx += ps * gv.x;
                ry += ps * gv.y;
              }
            } else {
              for (int q0 = 0; q0 < w; ++q0) {
                const T ps = pr[q0];
                const V gv = tr[q0];
                rx += ps * gv.x;
                ry += ps * gv.y;
              }
            }
            const T wv = D > 2 ? pr[w + q1] * pr[2 * w + q2] : pr[w + row];
            sx += wv * rx;
            sy += wv * ry;
            q1 += RG;
            if (D > 2) {
              while (q1 >= w) { q1 -= w; ++q2; }
            }
          }
          part[k] += (double)pr[wko + 2 * g] * (double)sx + (double)pr[wko + 2 * g + 1] * (double)sy;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const int it = threadIdx.x + k * kThreads;  // a lane group is all in or all out
      double v = part[k];
      if (RG >= 2) v += __shfl_xor(v, 1);
      if (RG >= 4) v += __shfl_xor(v, 2);
      if (it < nitems && it % RG == 0) {
        const int i = s_idx[it / RG];
        y[i] = (a.add_noise ? a.eta2 * x[i] : 0.0) + v;
      }
    }
  }
}

__global__ void gather_kernel(int64_t n, const int* __restrict__ perm, const double* __restrict__ u,
                              double* __restrict__ s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) s[i] = u[perm[i]];
}
__global__ void scatter_kernel(int64_t n, const int* __restrict__ perm, const double* __restrict__ s,
                               double* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) u[perm[i]] = s[i];
}

// ------------------------------------------------------------- launchers ----
template <typename T>
size_t spread_smem(const Plan* P, int gc, int rs) {
  size_t tcells = (size_t)P->tile[0] * P->tile[1] * P->tile[2];
  return gc * tcells * sizeof(typename V2<T>::type) + kPB * (lds_stride(rs) + 1) * sizeof(T) +
         kPB * P->d * sizeof(int) + 16;
}
template <typename T>
size_t interp_smem(const Plan* P, int gc, int rs) {
  size_t pc = (size_t)((P->tile[0] + P->w - 1) | 1);
  for (int r = 1; r < P->d; ++r) pc *= (size_t)(P->tile[r] + P->w - 1);
  return gc * pc * sizeof(typename V2<T>::type) + (kPB * lds_stride(rs) + 1) * sizeof(T) +
         kPB * kGC * sizeof(double) + kPB * P->d * sizeof(int) + 16;
}

// Runs CALL(GCV) with GCV the compile-time pair count equal to gc (1..kGC).
#define GP_GC_SWITCH(gc, CALL)                                  \
  switch (gc) {                                                 \
    case 1: CALL(1); break;                                     \
    case 2: CALL(2); break;                                     \
    case 3: CALL(3); break;                                     \
    case 4: CALL(4); break;                                     \
    case 5: CALL(5); break;                                     \
    case 6: CALL(6); break;                                     \
    case 7: CALL(7); break;                                     \
    default: CALL(8); break;                                    \
  }

constexpr size_t kSmemCap = 64 * 1024;


// Grid A (spread output, interpolation input) of the current vector set.
template <typename V>
V* cur_gridA(const Plan* P) {
  const int64_t set = (int64_t)P->npair * P->grid_elems[0];
  return static_cast<V*>(P->gv.A) + P->gv.cur * set;
}
// The 1-D four-step leaves the inverse transform in grid C.
template <typename V>
V* cur_interp_grid(const Plan* P) {
  if (!P->fourstep) return cur_gridA<V>(P);
  const int64_t set = (int64_t)P->npair * P->grid_elems[3];
  return static_cast<V*>(P->gv.C) + P->gv.cur * set;
}

template <typename T>
size_t spread_owner_smem(const Plan* P, int rs) {
  static_assert(kPB == 64, "the spread pre-filter compacts one batch per wavefront");
  int nsrc_tot = 1;
  for (int r = 0; r < P->d; ++r) nsrc_tot *= P->nsrc;
  return kPB * (lds_stride(rs) + 1) * sizeof(T) + (kPB * P->d + kPB + 1) * sizeof(int) +
         (3 * (size_t)nsrc_tot + 1) * sizeof(int) + 16;
}

template <typename T, int D, int CPT>
void launch_spread_owner(Plan* P, const Records& R, const double* xs) {
  PhaseScope ps(P, PH_SPREAD);
  NuArgs a = nu_args(P, R);
  const int gc = std::min(kGC, P->npair);
  const int nch = (P->npair + gc - 1) / gc;
  for (int ch = 0; ch < nch; ++ch) {
    a.g0 = ch * gc;
    a.gc = std::min(gc, P->npair - a.g0);
#define GP_LAUNCH_OWNER(GCV)                                                                   \
  hipLaunchKernelGGL((spread_owner_kernel<T, D, CPT, GCV>), dim3((unsigned)R.n_sp_work),         \
                     dim3(kThreads), spread_owner_smem<T>(P, R.rs), P->stream, a, xs,            \
                     R.cell.as<int>(), R.pw.as<T>(), R.rs, R.bin_start.as<int>(),                \
                     R.n_sp_red > 0 ? R.sp_work.as<int4>() : nullptr,                            \
                     R.part.as<typename V2<T>::type>(), cur_gridA<typename V2<T>::type>(P))
    GP_GC_SWITCH(a.gc, GP_LAUNCH_OWNER)
#undef GP_LAUNCH_OWNER
    GP_CHECK_LAUNCH();
    if (R.n_sp_red > 0) {
      hipLaunchKernelGGL((spread_reduce_kernel<T, D>), dim3((unsigned)R.n_sp_red), dim3(kThreads), 0,
                         P->stream, a, R.sp_red.as<int4>(), R.part.as<typename V2<T>::type>(),
                         cur_gridA<typename V2<T>::type>(P));
      GP_CHECK_LAUNCH();
    }
  }
}

template <typename T, int D>
void launch_spread(Plan* P, const Records& R, const double* xs) {
  PhaseScope ps(P, PH_SPREAD);
  NuArgs a = nu_args(P, R);
  int gc = std::min(kGC, P->npair);
  while (gc > 1 && spread_smem<T>(P, gc, R.rs) > kSmemCap) --gc;
  const int nch = (P->npair + gc - 1) / gc;
  for (int ch = 0; ch < nch; ++ch) {
    a.g0 = ch * gc;
    a.gc = std::min(gc, P->npair - a.g0);
    hipLaunchKernelGGL((spread_kernel<T, D>), dim3((unsigned)P->n_bins), dim3(kThreads),
                       spread_smem<T>(P, a.gc, R.rs), P->stream, a, xs, R.cell.as<int>(),
                       R.pw.as<T>(), R.rs, R.bin_start.as<int>(),
                       cur_gridA<typename V2<T>::type>(P));
    GP_CHECK_LAUNCH();
  }
}

// Dynamic LDS above 64 KB needs an explicit opt-in for each kernel (each
// instantiation: kernels of one signature are distinct functions).
constexpr size_t kSmemBig = 150 * 1024;
template <typename K>
void allow_big_lds(K kernel) {
  static std::mutex mu;
  static std::vector<const void*> done;
  const void* f = reinterpret_cast<const void*>(kernel);
  std::lock_guard<std::mutex> lk(mu);
  if (std::find(done.begin(), done.end(), f) != done.end()) return;
  GP_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmemBig));
  done.push_back(f);
}
// The 2x2(x1)-bin interpolation takes up to 80 KB: two workgroups per CU.
constexpr size_t kSmemSuper = 80 * 1024;

template <typename T, int D>
void launch_interp(Plan* P, const Records& R, const double* xs, double* ys, int add_noise) {
  PhaseScope ps(P, PH_INTERP);
  NuArgs a = nu_args(P, R);
  a.add_noise = add_noise;
  allow_big_lds(interp_kernel<T, D>);
  int gc = std::min(kGC, P->npair);
  while (gc > 1 && interp_smem<T>(P, gc, R.rs) > kSmemCap) --gc;
  const int nch = (P->npair + gc - 1) / gc;
  // the 1-D four-step inverse leaves the grid in C (see fft_all)
  const auto* gptr = cur_interp_grid<typename V2<T>::type>(P);
  for (int ch = 0; ch < nch; ++ch) {
    a.g0 = ch * gc;
    a.gc = std::min(gc, P->npair - a.g0);
    a.first_chunk = ch == 0;
    if (R.n_in_work == 0) break;
    hipLaunchKernelGGL((interp_kernel<T, D>), dim3((unsigned)R.n_in_work), dim3(kThreads),
                       interp_smem<T>(P, a.gc, R.rs), P->stream, a,
                       gptr, R.cell.as<int>(), R.pw.as<T>(), R.rs,
                       R.in_work.as<int4>(), xs, ys);
    GP_CHECK_LAUNCH();
  }
}

template <typename T>
void spread_dispatch(Plan* P, const Records& R, const double* xs) {
  const int tcells = P->tile[0] * P->tile[1] * P->tile[2];
  const int mode = P->spread_mode;
  // d >= 2: one wavefront per sub-tile from the point set's per-sub-tile lists
  if (spread_uses_sub_tiles(P) && R.n_sub > 0) {
    spread_sub_launch(P, R, xs);
    return;
  }
  if (mode != GP_SPREAD_LDS_ATOMIC && tcells <= 2 * kThreads) {
    const bool two = tcells > kThreads;
    if (P->d == 1) two ? launch_spread_owner<T, 1, 2>(P, R, xs) : launch_spread_owner<T, 1, 1>(P, R, xs);
    else if (P->d == 2) two ? launch_spread_owner<T, 2, 2>(P, R, xs) : launch_spread_owner<T, 2, 1>(P, R, xs);
    else two ? launch_spread_owner<T, 3, 2>(P, R, xs) : launch_spread_owner<T, 3, 1>(P, R, xs);
    return;
  }
  if (P->d == 1) launch_spread<T, 1>(P, R, xs);
  else if (P->d == 2) launch_spread<T, 2>(P, R, xs);
  else launch_spread<T, 3>(P, R, xs);
}

template <typename T, int D, int WT>
void launch_interp_gather(Plan* P, const Records& R, const double* xs, double* ys, int add_noise) {
  PhaseScope ps(P, PH_INTERP);
  NuArgs a = nu_args(P, R);
  a.add_noise = add_noise;
  hipLaunchKernelGGL((interp_gather_kernel<T, D, WT>), dim3((unsigned)((R.n + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, P->stream, a, cur_interp_grid<typename V2<T>::type>(P), R.cell.as<int>(),
                     R.pw.as<T>(), R.rs, xs, ys);
  GP_CHECK_LAUNCH();
}

template <typename T>
size_t interp_super_smem(const Plan* P, int rs) {
  const size_t pc0 = (size_t)(2 * P->tile[0] + P->w - 1), pc1 = (size_t)(2 * P->tile[1] + P->w - 1);
  const size_t pc2 = P->d > 2 ? (size_t)(P->tile[2] + P->w - 1) : 1;
  return (pc0 | 1) * pc1 * pc2 * sizeof(typename V2<T>::type) +
         (size_t)(P->d > 2 ? kPB2<3, T> : kPB2<2, T>) * (lds_stride(rs) * sizeof(T) + (P->d + 1) * sizeof(int)) + 16;
}

template <typename T>
void launch_interp_super(Plan* P, const Records& R, const double* xs, double* ys, int add_noise) {
  PhaseScope ps(P, PH_INTERP);
  NuArgs a = nu_args(P, R);
  a.add_noise = add_noise;
  if (R.n_in_work2 == 0) return;
  const int ucells = (2 * P->tile[0] + P->w - 1) * (2 * P->tile[1] + P->w - 1) *
                     (P->d > 2 ? P->tile[2] + P->w - 1 : 1);
  // software-pipelined tile loads when a pair's tile fits kTE cells per thread
  const bool pipe = ucells <= (P->d > 2 ? kTE<3> : kTE<2>) * kThreads;
  // compile-time window widths of the common plans (fp32 at tol 1e-4: 5 in
  // 3-D, 7 in 2-D at the automatic oversampling; fp64 at 1e-8 in 2-D: 12)
  auto pick = [&](auto d2, auto d3) { return P->d == 2 ? d2 : d3; };
  auto kern = pipe ? (P->w == 5    ? pick(interp_super_kernel<T, true, 2, 5>, interp_super_kernel<T, true, 3, 5>)
                      : P->w == 7  ? pick(interp_super_kernel<T, true, 2, 7>, interp_super_kernel<T, true, 3, 7>)
                      : P->w == 12 ? pick(interp_super_kernel<T, true, 2, 12>, interp_super_kernel<T, true, 3, 12>)
                                   : pick(interp_super_kernel<T, true, 2, 0>, interp_super_kernel<T, true, 3, 0>))
                   : pick(interp_super_kernel<T, false, 2, 0>, interp_super_kernel<T, false, 3, 0>);
  if (interp_super_smem<T>(P, R.rs) > kSmemCap) allow_big_lds(kern);
  // work items (2x2 bin blocks in raster order) are dealt to the 8 XCDs in
  // groups of 16 consecutive ones, so neighbouring blocks, whose halos
  // overlap, read them through one L2 (d=3 N=1e7: 3.50 -> 3.20 ms)
  constexpr int grp = 16;
  const int64_t nw = R.n_in_work2;
  const int64_t nblk = grp > 0 ? (nw + 8 * grp - 1) / (8 * grp) * (8 * grp) : nw;
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(kThreads),
                     interp_super_smem<T>(P, R.rs), P->stream, a,
                     cur_gridA<typename V2<T>::type>(P), R.cell.as<int>(), R.pw.as<T>(), R.rs,
                     R.bin_start.as<int>(), R.in_work2.as<int4>(), xs, ys, nw, grp);
  GP_CHECK_LAUNCH();
}

template <typename T>
void interp_dispatch(Plan* P, const Records& R, const double* xs, double* ys, int add_noise) {
  if (P->interp_mode == 0 && P->d >= 2 && interp_super_smem<T>(P, R.rs) <= kSmemSuper) {
    launch_interp_super<T>(P, R, xs, ys, add_noise);
    return;
  }
  if (P->interp_mode == 1) {  // cache-gather variant
    const bool big = P->w > 8;
#define GP_IG(DD) big ? launch_interp_gather<T, DD, 16>(P, R, xs, ys, add_noise) \
                      : launch_interp_gather<T, DD, 8>(P, R, xs, ys, add_noise)
    if (P->d == 1) GP_IG(1);
    else if (P->d == 2) GP_IG(2);
    else GP_IG(3);
#undef GP_IG
    return;
  }
  if (P->d == 1) launch_interp<T, 1>(P, R, xs, ys, add_noise);
  else if (P->d == 2) launch_interp<T, 2>(P, R, xs, ys, add_noise);
  else launch_interp<T, 3>(P, R, xs, ys, add_noise);
}

// Forward (sign -1) FFT of every grid pair: active box -> truncated modes.
// Inverse (sign +1): truncated modes -> active box.
void fft_all(Plan* P, int sign) {
  const int fp64 = P->precision == GP_FP64;
  // every set of the current grid view: the sets are consecutive, so they
  // transform as one batch of nsets * npair pairs
  const int64_t G = (int64_t)P->npair * P->gv.nsets, mc = P->mcount;
  const int d = P->d;
  const int nf = P->nf[0];
  hipStream_t s = P->stream;
  void* A = P->gv.A;
  void* B = P->gv.B;
  void* B2 = P->gv.B2;
  void* C = P->gv.C;
  FftPass q;
  q.sign = sign;
  // phase of a pass over dimension r
  auto run = [&](int r, const FftPass& ps_, const void* in, void* out, const void* twp) {
    PhaseScope sc(P, sign < 0 ? PH_FFT_FWD0 + r : PH_FFT_INV2 + (2 - r));
    fft_pass(fp64, ps_, in, out, twp, s);
  };
  if (d == 1 && P->fourstep) {
    const int L1 = P->L1, L2 = P->L2;
    FftPass y;  // over l2 (stride L1)
    y.L = L2; y.n_outer = G; y.inner = L1; y.in_os = nf; y.out_os = nf;
    y.n_in = L2; y.in_start = 0; y.n_out = L2; y.out_start = 0; y.sign = sign;
    FftPass x;  // over l1 (contiguous), four-step twiddle
    x.L = L1; x.n_outer = G * L2; x.inner = 1; x.in_os = L1; x.out_os = L1;
    x.n_in = L1; x.in_start = 0; x.n_out = L1; x.out_start = 0; x.sign = sign;
    x.tw4 = P->tw4.p; x.L4 = nf;
    if (sign < 0) {
      run(1, y, A, B, P->tw[1].p);
      x.tw4_at_load = 1;
      run(0, x, B, C, P->tw[0].p);
    } else {
      // the inverse result goes to C, not A: A keeps zeros outside the active
      // box (the spread writes only inside it) for the next forward pass
      x.tw4_at_load = 0;
      run(0, x, C, B, P->tw[0].p);
      run(1, y, B, C, P->tw[1].p);
    }
    return;
  }
  const void* tw = P->tw[0].p;
  if (d == 1) {
    q.L = nf; q.n_outer = G; q.inner = 1;
    if (sign < 0) {
      q.in_os = P->na[0]; q.n_in = P->na[0]; q.in_start = P->lo[0];
      q.out_os = mc; q.n_out = (int)mc; q.out_start = (int)-P->M;
      run(0, q, A, C, tw);
    } else {
      q.in_os = mc; q.n_in = (int)mc; q.in_start = (int)-P->M;
      q.out_os = P->na[0]; q.n_out = P->na[0]; q.out_start = P->lo[0];
      run(0, q, C, A, tw);
    }
    return;
  }
  if (d == 2) {
    // The modes are stored transposed, C[g][k0][k1], so that each strided
    // (column) pass writes whole sequences contiguously:
    //   forward: rows A[g][y][x] -> B; columns of B -> C[g][k0][k1]
    //   inverse: rows C[g][k0][.] -> B; columns of B -> A[g][y][x]
    // fp32 grids hold pairs of sequences interleaved in B, B[g][y/2][k0][y%2]
    // (forward) and B[g][k0/2][y][k0%2] (inverse): the column pass then reads
    // 2 x 2 elements contiguously, and the row pass, which transforms two
    // adjacent rows per workgroup, writes contiguously (fp32 FFT 1.24 ->
    // 1.16 ms per matvec at d=2 N=1e6).  fp64 grids keep B[g][y][k0] and
    // B[g][k0][y]: their two-row workgroups hold half the waves per CU
    // (5.26 -> 5.58 ms interleaved).
    // The mode kernel is symmetric in the two axes (it depends on |n|^2 and
    // on the same deconvolution factor per axis), so it runs on C unchanged.
    // B holds (na1 and mc rounded up to even) na1e x mce elements per pair.
    const int64_t na0 = P->na[0], na1 = P->na[1], mce = mc + (mc & 1), na1e = na1 + (na1 & 1);
    const bool ilv = !fp64;
    const int64_t bstride = ilv ? na1e * mce : na1 * mc;  // elements of B per grid pair
    FftPass r0;  // rows: two adjacent ones per workgroup when interleaved
    r0.L = nf; r0.sign = sign; r0.n_outer = G; r0.in_es = 1;
    if (ilv) { r0.out_cp = 2; r0.out_cs1 = 1; r0.out_es = 2; } else { r0.out_es = 1; }
    FftPass c1;  // strided sequences, contiguous output
    c1.L = nf; c1.sign = sign; c1.n_outer = G; c1.out_es = 1;
    if (ilv) { c1.in_cs = 2; c1.in_ip = 2; c1.in_es1 = 1; } else { c1.in_cs = 1; }
    if (sign < 0) {
      r0.inner = na1; r0.in_os = na1 * na0; r0.in_cs = na0;
      r0.n_in = (int)na0; r0.in_start = P->lo[0];
      r0.out_os = bstride; r0.out_cs = 2 * mce;
      r0.n_out = (int)mc; r0.out_start = (int)-P->M;
      if (!ilv) {  // one contiguous row per transform
        r0.inner = 1; r0.n_outer = G * na1; r0.in_os = na0; r0.in_cs = 0;
        r0.out_os = mc; r0.out_cs = 0;
      }
      run(0, r0, A, B, tw);
      c1.inner = mc; c1.in_os = bstride; c1.in_es = ilv ? 2 * mce : mc;
      c1.n_in = (int)na1; c1.in_start = P->lo[1];
      c1.out_os = mc * mc; c1.out_cs = mc;
      c1.n_out = (int)mc; c1.out_start = (int)-P->M;
      run(1, c1, B, C, tw);
    } else {
      r0.inner = mc; r0.in_os = mc * mc; r0.in_cs = mc;
      r0.n_in = (int)mc; r0.in_start = (int)-P->M;
      r0.out_os = bstride; r0.out_cs = 2 * na1;
      r0.n_out = (int)na1; r0.out_start = P->lo[1];
      if (!ilv) {
        r0.inner = 1; r0.n_outer = G * mc; r0.in_os = mc; r0.in_cs = 0;
        r0.out_os = na1; r0.out_cs = 0;
      }
      run(1, r0, C, B, tw);
      c1.inner = na1; c1.in_os = bstride; c1.in_es = ilv ? 2 * na1 : na1;
      c1.n_in = (int)mc; c1.in_start = (int)-P->M;
      c1.out_os = na1 * na0; c1.out_cs = na0;
      c1.n_out = (int)na0; c1.out_start = P->lo[0];
      run(0, c1, B, A, tw);
    }
    return;
  }
  // d = 3: dimension-0 pass (contiguous) between A [.., na0] and B [.., mc]
  FftPass x;
  x.L = nf; x.inner = 1; x.sign = sign;
  x.n_outer = G * P->na[1] * (d > 2 ? P->na[2] : 1);
  // dimension-1 pass between B [G][na2][na1][mc] and B2/C [G][na2][mc][mc]
  FftPass y;
  y.L = nf; y.inner = mc; y.sign = sign;
  y.n_outer = G * (d > 2 ? P->na[2] : 1);
  if (sign < 0) {
    x.in_os = P->na[0]; x.n_in = P->na[0]; x.in_start = P->lo[0];
    x.out_os = mc; x.n_out = (int)mc; x.out_start = (int)-P->M;
    run(0, x, A, B, tw);
    y.in_os = P->na[1] * mc; y.n_in = P->na[1]; y.in_start = P->lo[1];
    y.out_os = mc * mc; y.n_out = (int)mc; y.out_start = (int)-P->M;
    if (d == 2) {
      run(1, y, B, C, tw);
    } else {
      run(1, y, B, B2, tw);
      FftPass z;
      z.L = nf; z.inner = mc * mc; z.sign = sign; z.n_outer = G;
      z.in_os = P->na[2] * mc * mc; z.n_in = P->na[2]; z.in_start = P->lo[2];
      z.out_os = mc * mc * mc; z.n_out = (int)mc; z.out_start = (int)-P->M;
      run(2, z, B2, C, tw);
    }
  } else {
    if (d == 3) {
      FftPass z;
      z.L = nf; z.inner = mc * mc; z.sign = sign; z.n_outer = G;
      z.in_os = mc * mc * mc; z.n_in = (int)mc; z.in_start = (int)-P->M;
      z.out_os = P->na[2] * mc * mc; z.n_out = P->na[2]; z.out_start = P->lo[2];
      run(2, z, C, B2, tw);
    }
    y.in_os = mc * mc; y.n_in = (int)mc; y.in_start = (int)-P->M;
    y.out_os = P->na[1] * mc; y.n_out = P->na[1]; y.out_start = P->lo[1];
    run(1, y, d == 2 ? C : B2, B, tw);
    x.in_os = mc; x.n_in = (int)mc; x.in_start = (int)-P->M;
    x.out_os = P->na[0]; x.n_out = P->na[0]; x.out_start = P->lo[0];
    run(0, x, B, A, tw);
  }
}

template <typename T>
void forward_and_mix(Plan* P, const Records& R, const double* xs) {
  spread_dispatch<T>(P, R, xs);
  fft_all(P, -1);
  mix_modes(P);
  fft_all(P, +1);
}

}  // namespace

// Kernel arguments for the point set R (training points or targets) of plan P.
NuArgs nu_args(const Plan* P, const Records& R) {
  NuArgs a;
  a.n = R.n;
  a.nk = P->nk;
  a.npair = P->npair;
  a.w = P->w;
  a.beta = P->beta;
  for (int r = 0; r < 3; ++r) {
    a.tile[r] = P->tile[r];
    a.nbins[r] = P->nbins[r];
    a.na[r] = P->na[r];
  }
  a.gstride[0] = 1;
  a.gstride[1] = P->d > 1 ? P->na[0] : 0;
  a.gstride[2] = P->d > 2 ? (int64_t)P->na[0] * P->na[1] : 0;
  if (P->d == 1) {
    a.pair_stride = P->fourstep ? P->nf[0] : P->na[0];
    a.grid_off = P->fourstep ? P->lo[0] : 0;
  } else {
    a.pair_stride = (int64_t)P->na[0] * P->na[1] * P->na[2];
    a.grid_off = 0;
  }
  a.nsrc = P->nsrc;
  a.slot_pairs = std::min(kGC, P->npair);
  a.g0 = 0;
  a.gc = 0;
  a.eta2 = P->eta * P->eta;
  a.add_noise = 0;
  a.first_chunk = 1;
  return a;
}

void* grid_a_current(const Plan* P) {
  const size_t cs = P->precision == GP_FP64 ? 16 : 8;
  return static_cast<char*>(P->gv.A) + (size_t)P->gv.cur * P->npair * P->grid_elems[0] * cs;
}

void matvec_sorted(Plan* P, const double* xs, double* ys, int add_noise) {
  if (P->precision == GP_FP64) {
    forward_and_mix<double>(P, P->rec, xs);
    interp_dispatch<double>(P, P->rec, xs, ys, add_noise);
  } else {
    forward_and_mix<float>(P, P->rec, xs);
    interp_dispatch<float>(P, P->rec, xs, ys, add_noise);
  }
}

int multi_capacity(Plan* P, int want) {
  if (want <= P->m_cap) return want;
  const size_t cs = P->precision == GP_FP64 ? 16 : 8;
  const size_t per = (size_t)P->npair *
                     (P->grid_elems[0] + P->grid_elems[1] + P->grid_elems[2] + P->grid_elems[3]) * cs;
  size_t free_b = 0, total_b = 0;
  GP_HIP(hipMemGetInfo(&free_b, &total_b));
  const size_t fit = per > 0 ? (free_b / 2) / per : (size_t)want;
  return (int)std::max<size_t>(1, std::min<size_t>((size_t)want, fit));
}

static void ensure_multi(Plan* P, int m) {
  if (m <= P->m_cap) return;
  const size_t cs = P->precision == GP_FP64 ? 16 : 8;
  const size_t G = (size_t)P->npair * m;
  P->mA.alloc(G * P->grid_elems[0] * cs, P->stream);
  P->mB.alloc(G * P->grid_elems[1] * cs, P->stream);
  if (P->grid_elems[2]) P->mB2.alloc(G * P->grid_elems[2] * cs, P->stream);
  P->mC.alloc(G * P->grid_elems[3] * cs, P->stream);
  // the 1-D four-step keeps zeros in A outside the active box (see fft_all)
  if (P->fourstep) GP_HIP(hipMemsetAsync(P->mA.p, 0, P->mA.bytes, P->stream));
  P->m_cap = m;
}

void matvec_multi_sorted(Plan* P, int m, const double* xs, double* ys, int add_noise) {
  if (m < 1) return;
  ensure_multi(P, m);
  const Plan::GridView own = P->gv;
  P->gv.A = P->mA.p;
  P->gv.B = P->mB.p;
  P->gv.B2 = P->mB2.p;
  P->gv.C = P->mC.p;
  P->gv.nsets = m;
  try {
    const int64_t n = P->n;
    for (int j = 0; j < m; ++j) {
      P->gv.cur = j;
      if (P->precision == GP_FP64) spread_dispatch<double>(P, P->rec, xs + j * n);
      else spread_dispatch<float>(P, P->rec, xs + j * n);
    }
    fft_all(P, -1);
    mix_modes(P);
    fft_all(P, +1);
    for (int j = 0; j < m; ++j) {
      P->gv.cur = j;
      if (P->precision == GP_FP64) interp_dispatch<double>(P, P->rec, xs + j * n, ys + j * n, add_noise);
      else interp_dispatch<float>(P, P->rec, xs + j * n, ys + j * n, add_noise);
    }
  } catch (...) {
    P->gv = own;
    throw;
  }
  P->gv = own;
}

void posterior_sorted(Plan* P, const double* xs, int64_t m, const double* tpts,
                      const double* tsig, const double* tl, double* mu) {
  Records T;
  int oob = 0;
  build_records_into(P, m, tpts, tsig, tl, T, &oob);
  if (oob) throw Error{GP_ERANGE, "posterior target outside the plan's box"};
  DevBuf tmp;
  tmp.alloc(m * sizeof(double), P->stream);
  if (P->precision == GP_FP64) {
    forward_and_mix<double>(P, P->rec, xs);
    interp_dispatch<double>(P, T, nullptr, tmp.as<double>(), 0);
  } else {
    forward_and_mix<float>(P, P->rec, xs);
    interp_dispatch<float>(P, T, nullptr, tmp.as<double>(), 0);
  }
  hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, P->stream,
                     m, T.perm.as<int>(), tmp.as<double>(), mu);
  GP_CHECK_LAUNCH();
  GP_HIP(hipStreamSynchronize(P->stream));
}

// Grids for the points of R weighted by xs (sorted order of R): spread,
// forward FFT, mode mixing, inverse FFT.  interp_from_grid then evaluates the
// result at the points of another record set of the same plan.
void forward_from(Plan* P, const Records& R, const double* xs) {
  if (P->precision == GP_FP64)
    forward_and_mix<double>(P, R, xs);
  else
    forward_and_mix<float>(P, R, xs);
}
void interp_from_grid(Plan* P, const Records& R, double* ys) {
  if (P->precision == GP_FP64)
    interp_dispatch<double>(P, R, nullptr, ys, 0);
  else
    interp_dispatch<float>(P, R, nullptr, ys, 0);
}

void gather_sorted(Plan* P, const double* xu, double* xs) {
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((P->n + 255) / 256)), dim3(256), 0, P->stream,
                     P->n, P->rec.perm.as<int>(), xu, xs);
  GP_CHECK_LAUNCH();
}

void scatter_user(Plan* P, const double* xs, double* xu) {
  hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((P->n + 255) / 256)), dim3(256), 0,
                     P->stream, P->n, P->rec.perm.as<int>(), xs, xu);
  GP_CHECK_LAUNCH();
}

}  // namespace gp
