// Batched, pruned 1-D FFT passes for gfx950 (Stockham autosort).
//
// Steps 2 and 4 of the matvec (section 4.2) transform every fine grid along
// each axis in turn.  A workgroup transforms B sequences of length L.  Each
// thread keeps EPT elements in registers for the whole transform: the first
// radix stage loads its inputs straight from HBM (only the non-zero input
// window; everything else is zero), the last stage stores straight to HBM
// (only the output window later steps read), and the stages in between
// exchange data through LDS one real component at a time (a padded buffer of
// L + L/32 reals per sequence).  Radices go up to 32 (24 for lengths 3*2^k):
// an 8192-point transform is three stages with 32 elements per thread
// (32*32*8) and four with 16 (16*16*16*2); a 6144-point one with 24 elements
// per thread is four (24*8*8*4).
// Pruning both windows keeps the empty border of the oversampled grid (points
// fill a fraction 2*Delta-omega of the period) and the discarded high
// frequencies out of HBM.
#include "gp_internal.h"

namespace gp {
namespace {

template <typename T> struct V2;
template <> struct V2<double> { using type = double2; };
template <> struct V2<float> { using type = float2; };

template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
// multiply by s*i (s = +-1)
template <typename V> __device__ __forceinline__ V cmuli(V a, int s) {
  return s > 0 ? V{-a.y, a.x} : V{a.y, -a.x};
}

// y_q = sum_m x_m exp(s 2 pi i q m / r), in place.
template <typename T, typename V, int R> struct Dft;

template <typename T, typename V> struct Dft<T, V, 2> {
  __device__ __forceinline__ static void run(V* x, int) {
    V a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};
template <typename T, typename V> struct Dft<T, V, 3> {
  __device__ __forceinline__ static void run(V* x, int s) {
    const T h = T(0.86602540378443864676372317075294);  // sqrt(3)/2
    V t = cadd(x[1], x[2]);
    V u = csub(x[1], x[2]);
    V a = V{x[0].x - T(0.5) * t.x, x[0].y - T(0.5) * t.y};
    V b = cmuli(V{h * u.x, h * u.y}, s);
    x[0] = cadd(x[0], t);
    x[1] = cadd(a, b);
    x[2] = csub(a, b);
  }
};
template <typename T, typename V> struct Dft<T, V, 4> {
  __device__ __forceinline__ static void run(V* x, int s) {
    V a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
    V c = cadd(x[1], x[3]), e = cmuli(csub(x[1], x[3]), s);
    x[0] = cadd(a, c);
    x[2] = csub(a, c);
    x[1] = cadd(b, e);
    x[3] = csub(b, e);
  }
};
template <typename T, typename V> struct Dft<T, V, 8> {
  __device__ __forceinline__ static void run(V* x, int s) {
    V ev[4] = {x[0], x[2], x[4], x[6]};
    V od[4] = {x[1], x[3], x[5], x[7]};
    Dft<T, V, 4>::run(ev, s);
    Dft<T, V, 4>::run(od, s);
    const T r = T(0.70710678118654752440084436210485);
    // w^q = exp(s 2 pi i q / 8), q = 0..3
    V w1 = V{r, T(s) * r};
    V w3 = V{-r, T(s) * r};
    V o0 = od[0];
    V o1 = cmul(od[1], w1);
    V o2 = cmuli(od[2], s);
    V o3 = cmul(od[3], w3);
    x[0] = cadd(ev[0], o0);
    x[4] = csub(ev[0], o0);
    x[1] = cadd(ev[1], o1);
    x[5] = csub(ev[1], o1);
    x[2] = cadd(ev[2], o2);
    x[6] = csub(ev[2], o2);
    x[3] = cadd(ev[3], o3);
    x[7] = csub(ev[3], o3);
  }
};

// ------------------------------------------------------------ constants ----
constexpr double kPiC = 3.14159265358979323846264338327950288;
__host__ __device__ constexpr double taylor_sin(double r) {
  double t = r, s = r;
  for (int i = 1; i < 14; ++i) {
    t *= -r * r / ((2.0 * i) * (2.0 * i + 1.0));
    s += t;
  }
  return s;
}
__host__ __device__ constexpr double taylor_cos(double r) {
  double t = 1, s = 1;
  for (int i = 1; i < 14; ++i) {
    t *= -r * r / ((2.0 * i - 1.0) * (2.0 * i));
    s += t;
  }
  return s;
}
// cos(2 pi a / b), reduced to |angle - n pi/2| <= pi/4 before the series
__host__ __device__ constexpr double cos2pi(int a, int b) {
  a = ((a % b) + b) % b;
  const int n = (8 * a + b) / (2 * b);
  const double r = kPiC * (4.0 * a - (double)n * b) / (2.0 * b);
  return (n & 3) == 0 ? taylor_cos(r) : (n & 3) == 1 ? -taylor_sin(r) : (n & 3) == 2 ? -taylor_cos(r) : taylor_sin(r);
}
__host__ __device__ constexpr double sin2pi(int a, int b) { return cos2pi(4 * a - b, 4 * b); }

// ------------------------------------------------------- small DFTs ----
// y_q = sum_m x_m exp(s 2 pi i q m / R), in place; composite sizes split as
// R = R1 * R2 (m = m2 R1 + m1, q = q1 R2 + q2) with compile-time twiddles.
template <typename T, typename V, int R> struct Dft;

template <typename T, typename V, int R1, int R2, int I>
__device__ __forceinline__ void comp_twiddle(V* z, int s) {
  if constexpr (I < R1 * R2) {
    constexpr int m1 = I / R2, q2 = I % R2;
    if constexpr ((m1 * q2) % (R1 * R2) != 0) {
      constexpr double c = cos2pi(m1 * q2, R1 * R2), sn = sin2pi(m1 * q2, R1 * R2);
      z[I] = cmul(z[I], V{T(c), T(s) * T(sn)});
    }
    comp_twiddle<T, V, R1, R2, I + 1>(z, s);
  }
}

template <typename T, typename V, int R1, int R2> struct DftComp {
  __device__ __forceinline__ static void run(V* x, int s) {
    V z[R1 * R2];
#pragma unroll
    for (int m1 = 0; m1 < R1; ++m1) {
      V t[R2];
#pragma unroll
      for (int m2 = 0; m2 < R2; ++m2) t[m2] = x[m2 * R1 + m1];
      Dft<T, V, R2>::run(t, s);
#pragma unroll
      for (int q2 = 0; q2 < R2; ++q2) z[m1 * R2 + q2] = t[q2];
    }
    comp_twiddle<T, V, R1, R2, 0>(z, s);
#pragma unroll
    for (int q2 = 0; q2 < R2; ++q2) {
      V t[R1];
#pragma unroll
      for (int m1 = 0; m1 < R1; ++m1) t[m1] = z[m1 * R2 + q2];
      Dft<T, V, R1>::run(t, s);
#pragma unroll
      for (int q1 = 0; q1 < R1; ++q1) x[q1 * R2 + q2] = t[q1];
    }
  }
};
template <typename T, typename V> struct Dft<T, V, 16> : DftComp<T, V, 4, 4> {};
template <typename T, typename V> struct Dft<T, V, 32> : DftComp<T, V, 8, 4> {};
template <typename T, typename V> struct Dft<T, V, 24> : DftComp<T, V, 8, 3> {};

constexpr int next_radix(int rem, int ept) {
  return (rem % 32 == 0 && ept % 32 == 0)   ? 32
         : (rem % 24 == 0 && ept % 24 == 0) ? 24
         : (rem % 16 == 0 && ept % 16 == 0) ? 16
         : (rem % 8 == 0 && ept % 8 == 0)   ? 8
         : (rem % 4 == 0 && ept % 4 == 0)   ? 4
         : (rem % 2 == 0 && ept % 2 == 0)   ? 2
         : (rem % 3 == 0 && ept % 3 == 0)   ? 3
                                            : 0;
}

__device__ __forceinline__ int lpad(int p) { return p + (p >> 5); }

// offset of element i of a sequence: (i / ip) es + (i % ip) es1, ip = 1 << ips
__device__ __forceinline__ int64_t elem_off(int i, int ips, int64_t es, int64_t es1) {
  return (int64_t)(i >> ips) * es + (int64_t)(i & ((1 << ips) - 1)) * es1;
}

// Buffer-addressed element access (the default for passes without four-step
// twiddles): a workgroup-uniform buffer resource at the lowest line start of
// the workgroup, 32-bit byte offsets per element, and an offset past the
// resource's range for elements outside the pruning window (the load returns
// zero, the store is dropped), so the window tests cost no branches and the
// addresses no 64-bit arithmetic.  The host enables it only where every offset
// a workgroup forms fits below kBufRange.
constexpr unsigned kBufRange = 0x7fffffffu;
constexpr unsigned kBufOut = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)kBufRange,
                                           0x00020000);
}
__device__ __forceinline__ float2 buf_load(__amdgpu_buffer_rsrc_t r, unsigned off, float2*) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ double2 buf_load(__amdgpu_buffer_rsrc_t r, unsigned off, double2*) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}
__device__ __forceinline__ void buf_store(float2 v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  using U = __attribute__((ext_vector_type(2))) unsigned;
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U, v), r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_store(double2 v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  using U = __attribute__((ext_vector_type(4))) unsigned;
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U, v), r, (int)off, 0, 0);
}

struct KParams {
  int64_t ntrans, inner, in_os, out_os, in_es, in_cs, out_es, out_cs;
  int64_t in_cs1, in_es1, out_cs1, out_es1;
  int in_cps, in_ips, out_cps, out_ips;  // log2 of the interleave factors (0 or 1)
  int n_in, in_start, n_out, out_start, sign;
  int64_t L4, tw4_mod;
  int tw4_at_load;
};

// Stage with sub-transform length Ls and radix R on the registers v:
// butterfly j = jt + TPT u (u < EPT/R), k = j mod Ls, inputs v[u R + m] =
// X[j + m L/R], twiddle exp(s 2 pi i k m / (Ls R)) (one table load, powers by
// recurrence), outputs Y[(j - k) R + k + q Ls].  Then either exchange through
// LDS into the next stage's inputs or, on the last stage, store.
template <typename T, typename V, int L, int EPT, int Ls, bool BUF>
__device__ __forceinline__ void stages(V (&v)[EPT], T* __restrict__ buf, int jt,
                                       const V* __restrict__ tw, int s, bool act, V* dst,
                                       int64_t dstride, const KParams& p, const V* tw4,
                                       int64_t row4, __amdgpu_buffer_rsrc_t orsrc, int odl) {
  constexpr int TPT = L / EPT;
  constexpr int R = next_radix(L / Ls, EPT);
  static_assert(R > 0, "unsupported FFT length");
  constexpr int NB = EPT / R;
  if constexpr (Ls > 1) {
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int j = jt + TPT * u;
      const int k = j % Ls;
      V base = tw[k * (L / (Ls * R))];
      if (s > 0) base.y = -base.y;
      V wm = base;
#pragma unroll
      for (int m = 1; m < R; ++m) {
        v[u * R + m] = cmul(v[u * R + m], wm);
        if (m + 1 < R) wm = cmul(wm, base);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NB; ++u) Dft<T, V, R>::run(v + u * R, s);
  if constexpr (Ls * R < L) {
    constexpr int R2 = next_radix(L / (Ls * R), EPT);
    static_assert(R2 > 0, "unsupported FFT length");
    constexpr int NB2 = EPT / R2;
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int j = jt + TPT * u;
        const int k = j % Ls;
#pragma unroll
        for (int q = 0; q < R; ++q) buf[lpad((j - k) * R + k + q * Ls)] = comp ? v[u * R + q].y : v[u * R + q].x;
      }
      __syncthreads();
      // the read index is jt plus a compile-time c; where c is a multiple of
      // 32, lpad(jt + c) = lpad(jt) + c + c/32, an immediate offset
      const int rb = lpad(jt);
#pragma unroll
      for (int u = 0; u < NB2; ++u) {
        const int j = jt + TPT * u;
#pragma unroll
        for (int m = 0; m < R2; ++m) {
          const int c = TPT * u + m * (L / R2);
          const T val = (TPT % 32 == 0 && (L / R2) % 32 == 0) ? buf[rb + c + (c >> 5)]
                                                             : buf[lpad(j + m * (L / R2))];
          if (comp) v[u * R2 + m].y = val; else v[u * R2 + m].x = val;
        }
      }
      __syncthreads();
    }
    stages<T, V, L, EPT, Ls * R, BUF>(v, buf, jt, tw, s, act, dst, dstride, p, tw4, row4, orsrc,
                                      odl);
  } else {
    // last stage: k = j, outputs at j + q L/R
    if (!act) return;
    if constexpr (BUF) {
      const int pm = (1 << p.out_ips) - 1;
      const int oes = (int)dstride, oes1 = (int)p.out_es1;
      const int i0 = jt - p.out_start;
#pragma unroll
      for (int u = 0; u < NB; ++u)
#pragma unroll
        for (int q = 0; q < R; ++q) {
          int i = i0 + TPT * u + q * (L / R);
          i = i < 0 ? i + L : i;
          const int off = odl + (i >> p.out_ips) * oes + (i & pm) * oes1;
          buf_store(v[u * R + q], orsrc, i < p.n_out ? (unsigned)off * (unsigned)sizeof(V) : kBufOut);
        }
      return;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int j = jt + TPT * u;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int pos = j + q * (L / R);
        int i = pos - p.out_start;
        if (i < 0) i += L;
        if (i < p.n_out) {
          V val = v[u * R + q];
          if (tw4 != nullptr && !p.tw4_at_load) {
            V wv = tw4[((int64_t)pos * row4) % p.L4];
            if (s > 0) wv.y = -wv.y;
            val = cmul(val, wv);
          }
          dst[elem_off(i, p.out_ips, dstride, p.out_es1)] = val;
        }
      }
    }
  }
}

// Waves per SIMD that the LDS buffer allows (160 KB per CU, four SIMDs),
// passed to the compiler as its register budget for the long transforms:
// more registers than that occupancy leaves would keep LDS idle.  Capped
// where the elements held per thread need more registers than the budget.
constexpr int fft_waves(int L, int EPT, int B, int tb) {
  if (L < 1536) return 1;
  const int lds = B * (L + L / 32) * tb;
  const int wgs = (160 * 1024) / lds;
  const int w = wgs * ((B * (L / EPT) + 63) / 64) / 4;
  const int need = EPT * 2 * tb / 4 + 48;  // registers of the elements and the temporaries
  const int wr = 512 / need;
  const int m = w < wr ? w : wr;
  return m < 1 ? 1 : (m > 8 ? 8 : m);
}

template <typename T, int L, int EPT, int B, bool BUF, int S>
__global__ __launch_bounds__(B*(L / EPT), fft_waves(L, EPT, B, (int)sizeof(T))) void fft_pass_kernel(
    const typename V2<T>::type* __restrict__ in, typename V2<T>::type* __restrict__ out,
    const typename V2<T>::type* __restrict__ tw, const typename V2<T>::type* __restrict__ tw4,
    KParams p) {
  using V = typename V2<T>::type;
  constexpr int TPT = L / EPT;
  constexpr int LP = L + L / 32;
  __shared__ T buf[B * LP];
  // Workgroups go to the 8 XCDs round-robin by id.  For strided (column)
  // passes, give each XCD a contiguous range of transforms so neighbouring
  // columns, which share cache lines, run on the same XCD (same L2).
  int64_t bid = blockIdx.x;
  if (p.inner > 1) {
    const int64_t nb = gridDim.x, q = nb / 8, r = nb % 8;
    const int64_t x = bid % 8, slot = bid / 8;
    bid = x < r ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
  }
  int b, jt;
  if (p.inner == 1) {
    b = threadIdx.x / TPT;
    jt = threadIdx.x % TPT;
  } else {
    b = threadIdx.x % B;
    jt = threadIdx.x / B;
  }
  const int64_t t = bid * B + b;
  const bool act = t < p.ntrans;
  const int64_t o = act ? t / p.inner : 0, c = act ? t - o * p.inner : 0;
  const V* src = in + o * p.in_os + (c >> p.in_cps) * p.in_cs + (c & ((1 << p.in_cps) - 1)) * p.in_cs1;
  V* dst = out + o * p.out_os + (c >> p.out_cps) * p.out_cs + (c & ((1 << p.out_cps) - 1)) * p.out_cs1;
  const int64_t row4 = tw4 != nullptr ? o % p.tw4_mod : 0;
  constexpr int R1 = next_radix(L, EPT);
  constexpr int NB1 = EPT / R1;
  V v[EPT];
  __amdgpu_buffer_rsrc_t orsrc = buf_rsrc(out);
  int odl = 0;
  if constexpr (BUF) {
    // line starts are non-decreasing in the transform index (checked on the
    // host), so the workgroup's first line is its lowest
    const int64_t t0 = bid * B;
    const int64_t o0 = t0 / p.inner, c0 = t0 - o0 * p.inner;
    const V* ib = in + o0 * p.in_os + (c0 >> p.in_cps) * p.in_cs + (c0 & ((1 << p.in_cps) - 1)) * p.in_cs1;
    V* ob = out + o0 * p.out_os + (c0 >> p.out_cps) * p.out_cs + (c0 & ((1 << p.out_cps) - 1)) * p.out_cs1;
    const __amdgpu_buffer_rsrc_t irsrc = buf_rsrc(ib);
    orsrc = buf_rsrc(ob);
    const int idl = (int)(src - ib);
    odl = (int)(dst - ob);
    const int pm = (1 << p.in_ips) - 1;
    const int ies = (int)p.in_es, ies1 = (int)p.in_es1;
    const int i0 = jt - p.in_start;
#pragma unroll
    for (int u = 0; u < NB1; ++u)
#pragma unroll
      for (int m = 0; m < R1; ++m) {
        int i = i0 + TPT * u + m * (L / R1);
        i = i < 0 ? i + L : i;
        const int off = idl + (i >> p.in_ips) * ies + (i & pm) * ies1;
        v[u * R1 + m] = buf_load(irsrc, act && i < p.n_in ? (unsigned)off * (unsigned)sizeof(V) : kBufOut,
                                 (V*)nullptr);
      }
  } else
#pragma unroll
  for (int u = 0; u < NB1; ++u) {
    const int j = jt + TPT * u;
#pragma unroll
    for (int m = 0; m < R1; ++m) {
      const int pos = j + m * (L / R1);
      int i = pos - p.in_start;
      if (i < 0) i += L;
      V val = V{T(0), T(0)};
      if (act && i < p.n_in) {
        val = src[elem_off(i, p.in_ips, p.in_es, p.in_es1)];
        if (tw4 != nullptr && p.tw4_at_load) {
          V wv = tw4[((int64_t)pos * row4) % p.L4];
          if (S > 0) wv.y = -wv.y;
          val = cmul(val, wv);
        }
      }
      v[u * R1 + m] = val;
    }
  }
  stages<T, V, L, EPT, 1, BUF>(v, buf + b * LP, jt, tw, S, act, dst, p.out_es, p, tw4, row4,
                               orsrc, odl);
}

constexpr int ept_for(int L) { return (L % 3 == 0) ? (L < 24 ? L : 24) : (L < 32 ? L : 32); }
constexpr int batch_for(int L, int elem_bytes) {
  int tpt = L / ept_for(L);
  int b = 256 / tpt;
  if (b < 1) b = 1;
  int cap = (80 * 1024) / ((L + L / 32) * elem_bytes);
  if (cap < 1) cap = 1;
  return b < cap ? b : cap;
}

// Whether workgroups of B consecutive transforms can use buffer addressing:
// no four-step twiddles, non-negative strides, line starts non-decreasing in
// the transform index (so a workgroup's first line is its lowest), and every
// byte offset from a workgroup's first line below kBufRange.
bool buf_fits(const KParams& p, const FftPass& q, int B, int64_t vb) {
  if (q.tw4 != nullptr) return false;
  auto side = [&](int64_t os, int64_t cs, int64_t cs1, int cps, int64_t es, int64_t es1, int ips,
                  int n) {
    if (os < 0 || cs < 0 || cs1 < 0 || es < 0 || es1 < 0) return false;
    // largest start difference between the first and the last of B
    // consecutive transforms: k steps to the next outer index (each at most
    // os) and at most B - 1 steps within one (each at most cs)
    int64_t span = (int64_t)(B - 1) * os;
    if (p.inner > 1) {
      if (cps && cs1 > cs) return false;
      const int64_t cmax = ((p.inner - 1) >> cps) * cs + (cps ? cs1 : 0);
      if (os < cmax && p.ntrans > p.inner) return false;
      const int64_t k = (B - 1 + p.inner - 1) / p.inner;
      span = k * os + (int64_t)(B - 1) * cs;
    }
    const int64_t emax = n > 0 ? ((int64_t)(n - 1) >> ips) * es + (ips ? es1 : 0) : 0;
    return (span + emax + 1) * vb < (int64_t)kBufRange - 64;
  };
  return side(p.in_os, p.in_cs, p.in_cs1, p.in_cps, p.in_es, p.in_es1, p.in_ips, p.n_in) &&
         side(p.out_os, p.out_cs, p.out_cs1, p.out_cps, p.out_es, p.out_es1, p.out_ips, p.n_out);
}

template <typename T, int L, int EPT, int B>
void launch_kernel(bool buf, int64_t nblk, const KParams& p, const void* in, void* out,
                   const void* tw, const void* tw4, hipStream_t s) {
  using V = typename V2<T>::type;
  if (nblk <= 0) return;
  const dim3 g((unsigned)nblk), t(B * (L / EPT));
  const V *i = static_cast<const V*>(in), *w = static_cast<const V*>(tw), *w4 = static_cast<const V*>(tw4);
  V* o = static_cast<V*>(out);
  if (buf && p.sign < 0)
    hipLaunchKernelGGL((fft_pass_kernel<T, L, EPT, B, true, -1>), g, t, 0, s, i, o, w, w4, p);
  else if (buf)
    hipLaunchKernelGGL((fft_pass_kernel<T, L, EPT, B, true, 1>), g, t, 0, s, i, o, w, w4, p);
  else if (p.sign < 0)
    hipLaunchKernelGGL((fft_pass_kernel<T, L, EPT, B, false, -1>), g, t, 0, s, i, o, w, w4, p);
  else
    hipLaunchKernelGGL((fft_pass_kernel<T, L, EPT, B, false, 1>), g, t, 0, s, i, o, w, w4, p);
  GP_CHECK_LAUNCH();
}

template <typename T, int L>
void launch_len(const FftPass& q, const void* in, void* out, const void* tw, hipStream_t s) {
  using V = typename V2<T>::type;
  constexpr int EPT = ept_for(L);
  constexpr int B = batch_for(L, (int)sizeof(T));
  KParams p;
  p.ntrans = q.n_outer * q.inner;
  p.inner = q.inner;
  p.in_os = q.in_os;
  p.out_os = q.out_os;
  p.in_es = q.in_es ? q.in_es : q.inner;
  p.in_cs = q.in_cs ? q.in_cs : 1;
  p.out_es = q.out_es ? q.out_es : q.inner;
  p.out_cs = q.out_cs ? q.out_cs : 1;
  p.in_cs1 = q.in_cs1;
  p.in_es1 = q.in_es1;
  p.out_cs1 = q.out_cs1;
  p.out_es1 = q.out_es1;
  p.in_cps = q.in_cp == 2;
  p.in_ips = q.in_ip == 2;
  p.out_cps = q.out_cp == 2;
  p.out_ips = q.out_ip == 2;
  p.n_in = q.n_in;
  p.in_start = ((q.in_start % L) + L) % L;
  p.n_out = q.n_out;
  p.out_start = ((q.out_start % L) + L) % L;
  p.sign = q.sign;
  p.L4 = q.L4 > 0 ? q.L4 : 1;
  p.tw4_mod = q.L4 > 0 ? (q.L4 / L) : 1;
  p.tw4_at_load = q.tw4_at_load;
  // 8192-point passes.  Rows (and fp64 columns): 16 elements per thread, 512
  // threads, half the VGPRs of 32 per thread, so twice the waves per CU to
  // cover the memory latency.  fp32 columns: four adjacent columns per
  // workgroup (1024 threads, 32 elements each), so each quad of lanes reads 32
  // contiguous bytes; the column passes are bound by cache-line requests per
  // byte, and this wins (0.81 -> 0.72 ms) even though the 128-VGPR budget of a
  // 1024-thread workgroup spills a few registers.
  const int64_t vb = (int64_t)sizeof(V);
  if constexpr (L == 8192) {
    if constexpr (sizeof(T) == 4) {
      if (q.inner > 1) {
        launch_kernel<T, L, 32, 4>(buf_fits(p, q, 4, vb), (p.ntrans + 3) / 4, p, in, out, tw, q.tw4, s);
        return;
      }
    }
    launch_kernel<T, L, 16, 1>(buf_fits(p, q, 1, vb), p.ntrans, p, in, out, tw, q.tw4, s);
  } else {
    // Long strided (column) fp32 transforms: two columns per workgroup, so
    // pairs of adjacent lanes read adjacent elements of one cache line.  fp64
    // ones stay one per workgroup (two per workgroup: 1.56 against 1.47 ms for
    // the forward column pass at d=2 N=1e6 with contiguous output).
    if constexpr (B == 1 && L >= 6144) {
      if (q.inner > 1 && sizeof(T) == 4) {
        launch_kernel<T, L, EPT, 2>(buf_fits(p, q, 2, vb), (p.ntrans + 1) / 2, p, in, out, tw, q.tw4, s);
        return;
      }
    }
    launch_kernel<T, L, EPT, B>(buf_fits(p, q, B, vb), (p.ntrans + B - 1) / B, p, in, out, tw, q.tw4, s);
  }
}

template <typename T>
void dispatch(const FftPass& q, const void* in, void* out, const void* tw, hipStream_t s) {
  switch (q.L) {
#define GP_FFT_CASE(N) \
  case N:              \
    launch_len<T, N>(q, in, out, tw, s); \
    return;
    GP_FFT_CASE(8)
    GP_FFT_CASE(16)
    GP_FFT_CASE(32)
    GP_FFT_CASE(64)
    GP_FFT_CASE(128)
    GP_FFT_CASE(256)
    GP_FFT_CASE(512)
    GP_FFT_CASE(1024)
    GP_FFT_CASE(2048)
    GP_FFT_CASE(4096)
    GP_FFT_CASE(8192)
    GP_FFT_CASE(24)
    GP_FFT_CASE(48)
    GP_FFT_CASE(96)
    GP_FFT_CASE(192)
    GP_FFT_CASE(384)
    GP_FFT_CASE(768)
    GP_FFT_CASE(1536)
    GP_FFT_CASE(3072)
    GP_FFT_CASE(6144)
#undef GP_FFT_CASE
    default:
      throw Error{GP_EUNSUPPORTED, "FFT length " + std::to_string(q.L) + " not compiled"};
  }
}

}  // namespace


void fft_pass(int fp64, const FftPass& p, const void* in, void* out, const void* twiddles,
              hipStream_t s) {
  if (p.n_in > p.L || p.n_out > p.L || p.n_in < 0 || p.n_out < 0)
    throw Error{GP_EINVAL, "fft_pass: window longer than the transform"};
  for (int f : {p.in_cp, p.in_ip, p.out_cp, p.out_ip})
    if (f != 1 && f != 2) throw Error{GP_EINVAL, "fft_pass: interleave factor must be 1 or 2"};
  if (fp64)
    dispatch<double>(p, in, out, twiddles, s);
  else
    dispatch<float>(p, in, out, twiddles, s);
}

}  // namespace gp
