// Step 3 of section 4.2: mixing of the Fourier coefficients of the N_sigma+1
// grids at every mode of the grid {-M..M}^d (rem:step3).  Two variants:
// the precomputed tensor A_k'k stored per distinct |n|^2 (default) and the
// direct sum over the t nodes.  Both fold the window deconvolution in.
#include "gp_internal.h"

namespace gp {
namespace {

template <typename T> struct V2;
template <> struct V2<double> { using type = double2; };
template <> struct V2<float> { using type = float2; };

constexpr int kThreads = 256;

// ------------------------------------------------------------------ mode ----
struct ModeArgs {
  int d;
  int64_t M, mc, F;       // mc = 2M+1, F = mc^d
  int nk, npair, nt;
  int64_t pair_stride;
  int fourstep;
  int64_t nf, L1, L2;
};

__device__ __forceinline__ int64_t mode_store(const ModeArgs& a, int64_t f, const int64_t* nv) {
  if (!a.fourstep) return f;
  int64_t k = nv[0] % a.nf;
  if (k < 0) k += a.nf;
  return (k % a.L2) * a.L1 + (k / a.L2);
}

// Each thread owns a mode pair (n, -n) of every complex grid: it unpacks the two
// real spectra b_2g, b_2g+1, deconvolves, applies
//   a_k'[n] = sum_j v~_j G^_k'j[n] sum_k G^_kj[n] b_k[n]     (step 3, rem:step3 direct)
// re-deconvolves and packs the result back in place.
template <typename T, int NK>
__global__ __launch_bounds__(kThreads) void mode_kernel(
    ModeArgs a, typename V2<T>::type* __restrict__ C, const T* __restrict__ gtab,
    const T* __restrict__ etab, const T* __restrict__ vt, const T* __restrict__ dec) {
  using V = typename V2<T>::type;
  const int64_t f = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t half = (a.F + 1) / 2;
  if (f >= half) return;
  const int64_t fc = a.F - 1 - f;
  int64_t nv[3] = {0, 0, 0}, nvc[3] = {0, 0, 0};
  int64_t an[3] = {0, 0, 0};
  {
    int64_t q = f;
    for (int r = 0; r < a.d; ++r) {
      nv[r] = q % a.mc - a.M;
      q /= a.mc;
      nvc[r] = -nv[r];
      an[r] = nv[r] < 0 ? -nv[r] : nv[r];
    }
  }
  const int64_t M1 = a.M + 1;
  T D = T(1);
  for (int r = 0; r < a.d; ++r) D *= dec[r * M1 + an[r]];
  const int64_t s0 = mode_store(a, f, nv), s1 = mode_store(a, fc, nvc);
  V b[NK], acc[NK];
#pragma unroll
  for (int g = 0; g < NK / 2; ++g) {
    V z = V{T(0), T(0)}, zc = V{T(0), T(0)};
    if (g < a.npair) {
      z = C[g * a.pair_stride + s0];
      zc = C[g * a.pair_stride + s1];
    }
    b[2 * g] = V{T(0.5) * (z.x + zc.x) * D, T(0.5) * (z.y - zc.y) * D};
    b[2 * g + 1] = V{T(0.5) * (z.y + zc.y) * D, T(-0.5) * (z.x - zc.x) * D};
    acc[2 * g] = V{T(0), T(0)};
    acc[2 * g + 1] = V{T(0), T(0)};
  }
  const int nk = a.nk;
  for (int j = 0; j < a.nt; ++j) {
    const T* g0 = gtab + ((int64_t)j * nk) * M1 + an[0];
    const T* e1 = etab + ((int64_t)j * nk) * M1 + an[1];
    const T* e2 = etab + ((int64_t)j * nk) * M1 + an[2];
    T gk[NK];
    V s = V{T(0), T(0)};
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      T g = T(0);
      if (k < nk) {
        g = g0[k * M1];
        if (a.d > 1) g *= e1[k * M1];
        if (a.d > 2) g *= e2[k * M1];
      }
      gk[k] = g;
      s.x += g * b[k].x;
      s.y += g * b[k].y;
    }
    const T v = vt[j];
    s.x *= v;
    s.y *= v;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      acc[k].x += gk[k] * s.x;
      acc[k].y += gk[k] * s.y;
    }
  }
#pragma unroll
  for (int g = 0; g < NK / 2; ++g) {
    if (g >= a.npair) break;
    const V p = V{acc[2 * g].x * D, acc[2 * g].y * D};
    const V q = V{acc[2 * g + 1].x * D, acc[2 * g + 1].y * D};
    C[g * a.pair_stride + s0] = V{p.x - q.y, p.y + q.x};
    if (s1 != s0) C[g * a.pair_stride + s1] = V{p.x + q.y, -p.y + q.x};
  }
}

// Step 3 with the precomputed tensor of rem:step3.  A_k'k[n] depends on n only
// through |n|^2, so it is stored once per distinct |n|^2 (upper triangle, nkp
// wide).  Each thread owns the orthant point (|n_0|, .., |n_d-1|) and the up to
// 2^(d-1) conjugate pairs (s*n, -s*n) of sign patterns s that share its row.
struct RadialArgs {
  int d;
  int64_t M, mc, Q;       // Q = (M+1)^d orthant points
  int npair;
  int64_t pair_stride;
  int fourstep;
  int64_t nf, L1, L2;
  int nsets;              // vector sets (consecutive, set_stride elements apart)
  int64_t set_stride;
  const int* tiles;       // 2-D: the block -> orthant tile order (null: linear in q)
  int64_t ntx;            // tiles along n_0
};
static_assert(kModeTileX * kModeTileY == kThreads, "one orthant tile per block");

__device__ __forceinline__ int64_t radial_store(const RadialArgs& a, const int64_t* nv) {
  if (!a.fourstep) {
    int64_t f = 0, mul = 1;
    for (int r = 0; r < a.d; ++r) {
      f += (nv[r] + a.M) * mul;
      mul *= a.mc;
    }
    return f;
  }
  int64_t k = nv[0] % a.nf;
  if (k < 0) k += a.nf;
  return (k % a.L2) * a.L1 + (k / a.L2);
}

template <typename T, int NK>
__global__ __launch_bounds__(kThreads) void mode_radial_kernel(
    RadialArgs a, typename V2<T>::type* __restrict__ C, const T* __restrict__ Atab,
    const int* __restrict__ rowidx, const T* __restrict__ dec) {
  using V = typename V2<T>::type;
  constexpr int NP = NK * (NK + 1) / 2;
  const int64_t M1 = a.M + 1;
  int64_t an[3] = {0, 0, 0};
  if (a.tiles) {
    const int64_t t = a.tiles[blockIdx.x];
    an[0] = (t % a.ntx) * kModeTileX + threadIdx.x % kModeTileX;
    an[1] = (t / a.ntx) * kModeTileY + threadIdx.x / kModeTileX;
    if (an[0] > a.M || an[1] > a.M) return;
  } else {
    const int64_t tid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (tid >= a.Q) return;
    int64_t q = tid;
    for (int r = 0; r < a.d; ++r) {
      an[r] = q % M1;
      q /= M1;
    }
  }
  const int64_t s2 = an[0] * an[0] + an[1] * an[1] + an[2] * an[2];
  const int64_t row = a.d == 1 ? an[0] : (int64_t)rowidx[s2];
  const T* Ar = Atab + row * NP;
  T D = T(1);
  for (int r = 0; r < a.d; ++r) D *= dec[r * M1 + an[r]];
  int first_nz = -1;
  for (int r = 0; r < a.d; ++r)
    if (an[r] != 0) {
      first_nz = r;
      break;
    }
  // Sign patterns are processed two at a time so that one pass over the row of
  // A serves both (the row is the dominant read of this kernel); the vector
  // sets of a multi-vector application reuse the row from the caches.
  const int npat = 1 << (a.d - 1);
  for (int set = 0; set < a.nsets; ++set)
  for (int pg = 0; pg < npat; pg += 2) {
    V* __restrict__ Cs = C + set * a.set_stride;
    bool keep[2];
    int64_t st0[2], st1[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int pat = pg + h;
      keep[h] = pat < npat;
      int64_t nv[3] = {0, 0, 0}, nvc[3] = {0, 0, 0};
      for (int r = 0; r < a.d; ++r) {
        const int neg = r == 0 ? 0 : ((pat >> (r - 1)) & 1);
        if (neg && (an[r] == 0 || r == first_nz)) keep[h] = false;  // duplicate pattern
        nv[r] = neg ? -an[r] : an[r];
        nvc[r] = -nv[r];
      }
      st0[h] = keep[h] ? radial_store(a, nv) : 0;
      st1[h] = keep[h] ? radial_store(a, nvc) : 0;
    }
    if (!keep[0] && !keep[1]) continue;
    V b[2][NK];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int g = 0; g < NK / 2; ++g) {
        V z = V{T(0), T(0)}, zc = V{T(0), T(0)};
        if (keep[h] && g < a.npair) {
          z = Cs[g * a.pair_stride + st0[h]];
          zc = Cs[g * a.pair_stride + st1[h]];
        }
        b[h][2 * g] = V{T(0.5) * (z.x + zc.x) * D, T(0.5) * (z.y - zc.y) * D};
        b[h][2 * g + 1] = V{T(0.5) * (z.y + zc.y) * D, T(-0.5) * (z.x - zc.x) * D};
      }
    V acc[2][NK];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < NK; ++k) acc[h][k] = V{T(0), T(0)};
    int p = 0;
#pragma unroll
    for (int k1 = 0; k1 < NK; ++k1) {
#pragma unroll
      for (int k2 = k1; k2 < NK; ++k2) {
        const T av = Ar[p++];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          acc[h][k1].x += av * b[h][k2].x;
          acc[h][k1].y += av * b[h][k2].y;
          if (k2 != k1) {
            acc[h][k2].x += av * b[h][k1].x;
            acc[h][k2].y += av * b[h][k1].y;
          }
        }
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (!keep[h]) continue;
#pragma unroll
      for (int g = 0; g < NK / 2; ++g) {
        if (g >= a.npair) break;
        const V pp = V{acc[h][2 * g].x * D, acc[h][2 * g].y * D};
        const V qq = V{acc[h][2 * g + 1].x * D, acc[h][2 * g + 1].y * D};
        Cs[g * a.pair_stride + st0[h]] = V{pp.x - qq.y, pp.y + qq.x};
        if (st1[h] != st0[h]) Cs[g * a.pair_stride + st1[h]] = V{pp.x + qq.y, -pp.y + qq.x};
      }
    }
  }
}

// d = 2: one thread per (orthant point, sign pattern), the two patterns of a
// point on adjacent lanes, so each reads the same row of A in the same load
// instruction (one fetch) while holding half the registers of a thread that
// owns both patterns.  Two blocks per orthant tile (two of its rows each).
template <typename T, int NK>
__global__ __launch_bounds__(kThreads) void mode_radial2_kernel(
    RadialArgs a, typename V2<T>::type* __restrict__ C, const T* __restrict__ Atab,
    const int* __restrict__ rowidx, const T* __restrict__ dec) {
  using V = typename V2<T>::type;
  constexpr int NP = NK * (NK + 1) / 2;
  const int h = (int)(threadIdx.x & 1);
  const int lp = (int)(threadIdx.x >> 1);
  const int64_t M1 = a.M + 1;
  int64_t an0, an1;
  if (a.tiles) {
    const int64_t t = a.tiles[blockIdx.x >> 1];
    an0 = (t % a.ntx) * kModeTileX + lp % kModeTileX;
    an1 = (t / a.ntx) * kModeTileY + (kModeTileY / 2) * (blockIdx.x & 1) + lp / kModeTileX;
    if (an0 > a.M || an1 > a.M) return;
  } else {
    const int64_t q = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 1;
    if (q >= a.Q) return;
    an0 = q % M1;
    an1 = q / M1;
  }
  const T* Ar = Atab + (int64_t)rowidx[an0 * an0 + an1 * an1] * NP;
  const T D = dec[an0] * dec[M1 + an1];
  // pattern 1 negates n_1; it repeats pattern 0 when n_0 = 0 or n_1 = 0
  if (h == 1 && (an0 == 0 || an1 == 0)) return;
  const int64_t n1 = h ? -an1 : an1;
  const int64_t st0 = (an0 + a.M) + (n1 + a.M) * a.mc;
  const int64_t st1 = (-an0 + a.M) + (-n1 + a.M) * a.mc;
  for (int set = 0; set < a.nsets; ++set) {
    V* __restrict__ Cs = C + set * a.set_stride;
    V b[NK];
#pragma unroll
    for (int g = 0; g < NK / 2; ++g) {
      V z = V{T(0), T(0)}, zc = V{T(0), T(0)};
      if (g < a.npair) {
        z = Cs[g * a.pair_stride + st0];
        zc = Cs[g * a.pair_stride + st1];
      }
      b[2 * g] = V{T(0.5) * (z.x + zc.x) * D, T(0.5) * (z.y - zc.y) * D};
      b[2 * g + 1] = V{T(0.5) * (z.y + zc.y) * D, T(-0.5) * (z.x - zc.x) * D};
    }
    V acc[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) acc[k] = V{T(0), T(0)};
    int p = 0;
#pragma unroll
    for (int k1 = 0; k1 < NK; ++k1) {
#pragma unroll
      for (int k2 = k1; k2 < NK; ++k2) {
        const T av = Ar[p++];
        acc[k1].x += av * b[k2].x;
        acc[k1].y += av * b[k2].y;
        if (k2 != k1) {
          acc[k2].x += av * b[k1].x;
          acc[k2].y += av * b[k1].y;
        }
      }
    }
#pragma unroll
    for (int g = 0; g < NK / 2; ++g) {
      if (g >= a.npair) break;
      const V pp = V{acc[2 * g].x * D, acc[2 * g].y * D};
      const V qq = V{acc[2 * g + 1].x * D, acc[2 * g + 1].y * D};
      Cs[g * a.pair_stride + st0] = V{pp.x - qq.y, pp.y + qq.x};
      if (st1 != st0) Cs[g * a.pair_stride + st1] = V{pp.x + qq.y, -pp.y + qq.x};
    }
  }
}

// Step 3 with the rows of A in low-rank form (rem:step3, last paragraph):
// A(|n|^2) ~ sum_a R_a R_a', rank_r = (off[r+1] - off[r]) / NK factors of NK
// entries each.  a = R (R' b): 2 rank NK multiply-adds per complex value
// instead of NK^2.  Orthant points and sign patterns as in mode_radial_kernel.
template <typename T, int NK>
__global__ __launch_bounds__(kThreads) void mode_lowrank_kernel(
    RadialArgs a, typename V2<T>::type* __restrict__ C, const T* __restrict__ Rtab,
    const int64_t* __restrict__ off, const int* __restrict__ rowidx, const T* __restrict__ dec) {
  using V = typename V2<T>::type;
  const int64_t tid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (tid >= a.Q) return;
  const int64_t M1 = a.M + 1;
  int64_t an[3] = {0, 0, 0};
  {
    int64_t q = tid;
    for (int r = 0; r < a.d; ++r) {
      an[r] = q % M1;
      q /= M1;
    }
  }
  const int64_t s2 = an[0] * an[0] + an[1] * an[1] + an[2] * an[2];
  const int64_t row = a.d == 1 ? an[0] : (int64_t)rowidx[s2];
  const T* Rr = Rtab + off[row];
  const int rank = (int)((off[row + 1] - off[row]) / NK);
  T D = T(1);
  for (int r = 0; r < a.d; ++r) D *= dec[r * M1 + an[r]];
  int first_nz = -1;
  for (int r = 0; r < a.d; ++r)
    if (an[r] != 0) {
      first_nz = r;
      break;
    }
  const int npat = 1 << (a.d - 1);
  for (int set = 0; set < a.nsets; ++set)
  for (int pg = 0; pg < npat; pg += 2) {
    V* __restrict__ Cs = C + set * a.set_stride;
    bool keep[2];
    int64_t st0[2], st1[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int pat = pg + h;
      keep[h] = pat < npat;
      int64_t nv[3] = {0, 0, 0}, nvc[3] = {0, 0, 0};
      for (int r = 0; r < a.d; ++r) {
        const int neg = r == 0 ? 0 : ((pat >> (r - 1)) & 1);
        if (neg && (an[r] == 0 || r == first_nz)) keep[h] = false;
        nv[r] = neg ? -an[r] : an[r];
        nvc[r] = -nv[r];
      }
      st0[h] = keep[h] ? radial_store(a, nv) : 0;
      st1[h] = keep[h] ? radial_store(a, nvc) : 0;
    }
    if (!keep[0] && !keep[1]) continue;
    V b[2][NK];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int g = 0; g < NK / 2; ++g) {
        V z = V{T(0), T(0)}, zc = V{T(0), T(0)};
        if (keep[h] && g < a.npair) {
          z = Cs[g * a.pair_stride + st0[h]];
          zc = Cs[g * a.pair_stride + st1[h]];
        }
        b[h][2 * g] = V{T(0.5) * (z.x + zc.x) * D, T(0.5) * (z.y - zc.y) * D};
        b[h][2 * g + 1] = V{T(0.5) * (z.y + zc.y) * D, T(-0.5) * (z.x - zc.x) * D};
      }
    V acc[2][NK];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < NK; ++k) acc[h][k] = V{T(0), T(0)};
    for (int f = 0; f < rank; ++f) {
      const T* ra = Rr + (int64_t)f * NK;
      T rv[NK];
#pragma unroll
      for (int k = 0; k < NK; ++k) rv[k] = ra[k];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        V t = V{T(0), T(0)};
#pragma unroll
        for (int k = 0; k < NK; ++k) {
          t.x += rv[k] * b[h][k].x;
          t.y += rv[k] * b[h][k].y;
        }
#pragma unroll
        for (int k = 0; k < NK; ++k) {
          acc[h][k].x += rv[k] * t.x;
          acc[h][k].y += rv[k] * t.y;
        }
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (!keep[h]) continue;
#pragma unroll
      for (int g = 0; g < NK / 2; ++g) {
        if (g >= a.npair) break;
        const V pp = V{acc[h][2 * g].x * D, acc[h][2 * g].y * D};
        const V qq = V{acc[h][2 * g + 1].x * D, acc[h][2 * g + 1].y * D};
        Cs[g * a.pair_stride + st0[h]] = V{pp.x - qq.y, pp.y + qq.x};
        if (st1[h] != st0[h]) Cs[g * a.pair_stride + st1[h]] = V{pp.x + qq.y, -pp.y + qq.x};
      }
    }
  }
}

// d = 1: the M+1 orthant points are too few to fill the chip one per thread,
// so each point takes a group of NK lanes: lane j forms b_j, computes row j
// of A b (terms in the order k = 0..NK-1, as the per-thread kernel adds them),
// and lanes g < npair write the conjugate pair (n, -n) of grid g.
template <typename T, int NK>
__global__ __launch_bounds__(kThreads) void mode_radial_1d_kernel(
    RadialArgs a, typename V2<T>::type* __restrict__ C, const T* __restrict__ Atab,
    const T* __restrict__ dec) {
  using V = typename V2<T>::type;
  constexpr int NP = NK * (NK + 1) / 2;
  constexpr int PPB = kThreads / NK;  // points per workgroup
  __shared__ V sb[PPB][NK];
  __shared__ V sa[PPB][NK];
  const int lp = threadIdx.x / NK, j = threadIdx.x % NK;
  const int64_t n0 = (int64_t)blockIdx.x * PPB + lp;
  const bool act = lp < PPB && n0 <= a.M;
  int64_t st0 = 0, st1 = 0;
  T D = T(0);
  if (act) {
    int64_t nv[3] = {n0, 0, 0}, nvc[3] = {-n0, 0, 0};
    st0 = radial_store(a, nv);
    st1 = radial_store(a, nvc);
    D = dec[n0];
    const int g = j / 2;
    V z = V{T(0), T(0)}, zc = V{T(0), T(0)};
    if (g < a.npair) {
      z = C[g * a.pair_stride + st0];
      zc = C[g * a.pair_stride + st1];
    }
    sb[lp][j] = (j & 1) ? V{T(0.5) * (z.y + zc.y) * D, T(-0.5) * (z.x - zc.x) * D}
                        : V{T(0.5) * (z.x + zc.x) * D, T(0.5) * (z.y - zc.y) * D};
  }
  __syncthreads();
  if (act) {
    const T* Ar = Atab + n0 * NP;
    V acc = V{T(0), T(0)};
#pragma unroll 8
    for (int k = 0; k < NK; ++k) {
      const int lo = min(j, k), hi = max(j, k);
      const T av = Ar[lo * NK - lo * (lo - 1) / 2 + (hi - lo)];
      acc.x += av * sb[lp][k].x;
      acc.y += av * sb[lp][k].y;
    }
    sa[lp][j] = acc;
  }
  __syncthreads();
  if (act && j < a.npair) {
    const V pp = V{sa[lp][2 * j].x * D, sa[lp][2 * j].y * D};
    const V qq = V{sa[lp][2 * j + 1].x * D, sa[lp][2 * j + 1].y * D};
    C[j * a.pair_stride + st0] = V{pp.x - qq.y, pp.y + qq.x};
    if (st1 != st0) C[j * a.pair_stride + st1] = V{pp.x + qq.y, -pp.y + qq.x};
  }
}

// 1-D four-step: zero the spectrum outside {-M..M} before the inverse transform.
template <typename T>
__global__ void zero_band_kernel(typename V2<T>::type* C, int64_t nf, int64_t L1, int64_t L2,
                                 int64_t M, int npair) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nf * npair) return;
  const int64_t idx = e % nf;
  const int64_t k2 = idx / L1, k1 = idx % L1;
  const int64_t k = k2 + L2 * k1;
  const int64_t n = k <= nf / 2 ? k : k - nf;
  if (n > M || n < -M) C[e] = typename V2<T>::type{T(0), T(0)};
}

template <typename T, int NK>
void launch_mode_nk(Plan* P) {
  PhaseScope ps(P, PH_MODE);
  ModeArgs a;
  a.d = P->d;
  a.M = P->M;
  a.mc = P->mcount;
  a.F = 1;
  for (int r = 0; r < P->d; ++r) a.F *= a.mc;
  a.nk = P->nk;
  a.npair = P->npair;
  a.nt = P->nt_eff;
  a.fourstep = P->fourstep;
  a.nf = P->nf[0];
  a.L1 = P->L1;
  a.L2 = P->L2;
  a.pair_stride = P->fourstep ? P->nf[0] : a.F;
  const int64_t half = (a.F + 1) / 2;
  for (int set = 0; set < P->gv.nsets; ++set) {
    hipLaunchKernelGGL((mode_kernel<T, NK>), dim3((unsigned)((half + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, P->stream, a,
                       static_cast<typename V2<T>::type*>(P->gv.C) + set * P->npair * a.pair_stride,
                       P->gtab.as<T>(), P->etab.as<T>(), P->vtd.as<T>(), P->dec.as<T>());
    GP_CHECK_LAUNCH();
  }
}

template <typename T, int NK>
void launch_radial_nk(Plan* P) {
  PhaseScope ps(P, PH_MODE);
  RadialArgs a;
  a.d = P->d;
  a.M = P->M;
  a.mc = P->mcount;
  a.Q = 1;
  for (int r = 0; r < P->d; ++r) a.Q *= (P->M + 1);
  a.npair = P->npair;
  a.fourstep = P->fourstep;
  a.nf = P->nf[0];
  a.L1 = P->L1;
  a.L2 = P->L2;
  int64_t F = 1;
  for (int r = 0; r < P->d; ++r) F *= a.mc;
  a.pair_stride = P->fourstep ? P->nf[0] : F;
  a.nsets = P->gv.nsets;
  a.set_stride = P->npair * a.pair_stride;
  a.tiles = nullptr;
  a.ntx = 0;
  auto* C = static_cast<typename V2<T>::type*>(P->gv.C);
  if (P->step3 == 2) {
    hipLaunchKernelGGL((mode_lowrank_kernel<T, NK>), dim3((unsigned)((a.Q + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, P->stream, a, C, P->atab.as<T>(), P->lr_off.as<int64_t>(),
                       P->d > 1 ? P->rowidx.as<int>() : nullptr, P->dec.as<T>());
    GP_CHECK_LAUNCH();
    return;
  }
  if (P->d == 1) {
    constexpr int PPB = kThreads / NK;
    for (int set = 0; set < a.nsets; ++set) {
      hipLaunchKernelGGL((mode_radial_1d_kernel<T, NK>), dim3((unsigned)((a.Q + PPB - 1) / PPB)),
                         dim3(kThreads), 0, P->stream, a, C + set * a.set_stride,
                         P->atab.as<T>(), P->dec.as<T>());
      GP_CHECK_LAUNCH();
    }
    return;
  }
  // fp64: 1.52 -> 1.43 ms at d=2 N=1e6; fp32 unchanged (0.37 ms), kept on
  // the two-pattern kernel
  // 2-D: orthant tiles nearest the origin first (the table rows in use then
  // form a band that stays in the caches)
  int64_t nblk = (a.Q + kThreads - 1) / kThreads;
  if (P->d == 2 && P->mode_tiles.p) {
    a.tiles = P->mode_tiles.as<int>();
    a.ntx = P->mode_ntx;
    nblk = P->mode_ntx * (P->M / kModeTileY + 1);
  }
  if (P->d == 2 && !a.fourstep && sizeof(T) == 8) {
    hipLaunchKernelGGL((mode_radial2_kernel<T, NK>), dim3((unsigned)(a.tiles ? 2 * nblk : (2 * a.Q + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, P->stream, a, C, P->atab.as<T>(), P->rowidx.as<int>(),
                       P->dec.as<T>());
    GP_CHECK_LAUNCH();
    return;
  }
  hipLaunchKernelGGL((mode_radial_kernel<T, NK>), dim3((unsigned)nblk),
                     dim3(kThreads), 0, P->stream, a, C,
                     P->atab.as<T>(), P->d > 1 ? P->rowidx.as<int>() : nullptr, P->dec.as<T>());
  GP_CHECK_LAUNCH();
}

template <typename T>
void launch_mode(Plan* P) {
  const int nk2 = 2 * P->npair;
  if (P->step3 != 1) {
    switch (nk2) {
#define GP_R(N) case N: launch_radial_nk<T, N>(P); return;
      GP_R(2) GP_R(4) GP_R(6) GP_R(8) GP_R(10) GP_R(12) GP_R(14) GP_R(16) GP_R(18) GP_R(20)
      GP_R(22) GP_R(24) GP_R(26) GP_R(28) GP_R(30) GP_R(32) GP_R(34) GP_R(36) GP_R(38) GP_R(40)
      GP_R(42) GP_R(44) GP_R(46) GP_R(48)
#undef GP_R
      default:
        throw Error{GP_EUNSUPPORTED, "too many Chebyshev nodes"};
    }
  }
  switch (nk2) {
#define GP_M(N) case N: launch_mode_nk<T, N>(P); break;
    GP_M(2) GP_M(4) GP_M(6) GP_M(8) GP_M(10) GP_M(12) GP_M(14) GP_M(16) GP_M(18) GP_M(20)
    GP_M(22) GP_M(24) GP_M(26) GP_M(28) GP_M(30) GP_M(32) GP_M(34) GP_M(36) GP_M(38) GP_M(40)
    GP_M(42) GP_M(44) GP_M(46) GP_M(48)
#undef GP_M
    default:
      throw Error{GP_EUNSUPPORTED, "too many Chebyshev nodes"};
  }
}

}  // namespace

// Compiled twice (GP_MODE_FP64 = 1 / 0) so the two precisions build in parallel.
#if GP_MODE_FP64
#define GP_MODE_T double
#define GP_MIX_FN mix_modes_fp64
#else
#define GP_MODE_T float
#define GP_MIX_FN mix_modes_fp32
#endif

void GP_MIX_FN(Plan* P) {
  using T = GP_MODE_T;
  launch_mode<T>(P);
  if (P->fourstep) {
    const int npairs = P->npair * P->gv.nsets;
    const int64_t tot = (int64_t)P->nf[0] * npairs;
    hipLaunchKernelGGL(zero_band_kernel<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                       P->stream, static_cast<typename V2<T>::type*>(P->gv.C), (int64_t)P->nf[0],
                       (int64_t)P->L1, (int64_t)P->L2, P->M, npairs);
    GP_CHECK_LAUNCH();
  }
}

}  // namespace gp
