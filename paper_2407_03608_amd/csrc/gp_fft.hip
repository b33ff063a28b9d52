// Batched, pruned 1-D FFT passes for gfx950 (Stockham autosort, LDS resident).
//
// Steps 2 and 4 of the matvec (section 4.2) transform every fine grid along
// each axis in turn.  One workgroup transforms B sequences of length L: it
// loads the non-zero input window of each sequence (zero elsewhere) from HBM
// into LDS, runs the radix-8/4/3/2 stages with each thread holding EPT
// elements in registers between LDS exchanges, and writes back only the
// output window that later steps read.  Pruning both windows is what keeps
// the empty border of the oversampled grid (the points fill only a fraction
// 2*Delta-omega of the period) and the discarded high frequencies out of HBM.
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

constexpr int next_radix(int rem, int ept) {
  return (rem % 8 == 0 && ept % 8 == 0)   ? 8
         : (rem % 4 == 0 && ept % 4 == 0) ? 4
         : (rem % 2 == 0 && ept % 2 == 0) ? 2
         : (rem % 3 == 0 && ept % 3 == 0) ? 3
                                          : 0;
}

// One Stockham stage: butterflies j = jt + TPT*u, k = j mod Ls,
// inputs X[j + m L/R], twiddle exp(s 2 pi i k m / (Ls R)), outputs
// Y[(j - k) R + k + q Ls].  tw[i] = exp(-2 pi i i / L).
template <typename T, typename V, int L, int EPT, int R, int Ls>
__device__ __forceinline__ void stage(V* buf, int jt, const V* __restrict__ tw, int s) {
  constexpr int TPT = L / EPT;
  constexpr int NB = EPT / R;
  V v[EPT];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int j = jt + TPT * u;
    const int k = j % Ls;
#pragma unroll
    for (int m = 0; m < R; ++m) v[u * R + m] = buf[j + m * (L / R)];
    if (Ls > 1) {
#pragma unroll
      for (int m = 1; m < R; ++m) {
        V t = tw[k * m * (L / (Ls * R))];
        if (s > 0) t.y = -t.y;
        v[u * R + m] = cmul(v[u * R + m], t);
      }
    }
    Dft<T, V, R>::run(v + u * R, s);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int j = jt + TPT * u;
    const int k = j % Ls;
#pragma unroll
    for (int q = 0; q < R; ++q) buf[(j - k) * R + k + q * Ls] = v[u * R + q];
  }
  __syncthreads();
}

template <typename T, typename V, int L, int EPT, int Ls>
__device__ __forceinline__ void run_stages(V* buf, int jt, const V* __restrict__ tw, int s) {
  if constexpr (Ls < L) {
    constexpr int R = next_radix(L / Ls, EPT);
    static_assert(R > 0, "unsupported FFT length");
    stage<T, V, L, EPT, R, Ls>(buf, jt, tw, s);
    run_stages<T, V, L, EPT, Ls * R>(buf, jt, tw, s);
  }
}

struct KParams {
  int64_t ntrans, inner, in_os, out_os;
  int n_in, in_start, n_out, out_start, sign;
  int64_t L4, tw4_mod;
  int tw4_at_load;
};

template <typename T, int L, int EPT, int B>
__global__ __launch_bounds__(B*(L / EPT)) void fft_pass_kernel(
    const typename V2<T>::type* __restrict__ in, typename V2<T>::type* __restrict__ out,
    const typename V2<T>::type* __restrict__ tw, const typename V2<T>::type* __restrict__ tw4,
    KParams p) {
  using V = typename V2<T>::type;
  constexpr int TPT = L / EPT;
  constexpr int NTHR = B * TPT;
  __shared__ V buf[B * L];
  // Workgroups go to the 8 XCDs round-robin by id.  For strided (column)
  // passes, give each XCD a contiguous range of transforms so neighbouring
  // columns, which share cache lines, run on the same XCD (same L2).
  int64_t bid = blockIdx.x;
  if (p.inner > 1) {
    const int64_t nb = gridDim.x, q = nb / 8, r = nb % 8;
    const int64_t x = bid % 8, slot = bid / 8;
    bid = x < r ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
  }
  const int64_t t0 = bid * B;

  for (int e = threadIdx.x; e < B * L; e += NTHR) {
    int b, pos;
    if (p.inner == 1) {
      b = e / L;
      pos = e % L;
    } else {
      pos = e / B;
      b = e % B;
    }
    const int64_t t = t0 + b;
    V v = V{T(0), T(0)};
    if (t < p.ntrans) {
      int i = pos - p.in_start;
      if (i < 0) i += L;
      if (i < p.n_in) {
        const int64_t o = t / p.inner, c = t - o * p.inner;
        v = in[o * p.in_os + (int64_t)i * p.inner + c];
        if (tw4 != nullptr && p.tw4_at_load) {
          const int64_t row = o % p.tw4_mod;
          V w = tw4[((int64_t)pos * row) % p.L4];
          if (p.sign > 0) w.y = -w.y;
          v = cmul(v, w);
        }
      }
    }
    buf[b * L + pos] = v;
  }
  __syncthreads();

  {
    const int b = threadIdx.x / TPT;
    const int jt = threadIdx.x % TPT;
    run_stages<T, V, L, EPT, 1>(buf + b * L, jt, tw, p.sign);
  }

  for (int e = threadIdx.x; e < B * p.n_out; e += NTHR) {
    int b, i;
    if (p.inner == 1) {
      b = e / p.n_out;
      i = e - b * p.n_out;
    } else {
      i = e / B;
      b = e - i * B;
    }
    const int64_t t = t0 + b;
    if (t >= p.ntrans) continue;
    int pos = p.out_start + i;
    if (pos >= L) pos -= L;
    V v = buf[b * L + pos];
    const int64_t o = t / p.inner, c = t - o * p.inner;
    if (tw4 != nullptr && !p.tw4_at_load) {
      const int64_t row = o % p.tw4_mod;
      V w = tw4[((int64_t)pos * row) % p.L4];
      if (p.sign > 0) w.y = -w.y;
      v = cmul(v, w);
    }
    out[o * p.out_os + (int64_t)i * p.inner + c] = v;
  }
}

constexpr int ept_for(int L) { return (L % 3 == 0) ? 24 : 8; }
constexpr int batch_for(int L, int elem_bytes) {
  int tpt = L / ept_for(L);
  int b = 256 / tpt;
  if (b < 1) b = 1;
  int cap = (64 * 1024) / (L * elem_bytes);
  if (cap < 1) cap = 1;
  return b < cap ? b : cap;
}

template <typename T, int L>
void launch_len(const FftPass& q, const void* in, void* out, const void* tw, hipStream_t s) {
  using V = typename V2<T>::type;
  constexpr int EPT = ept_for(L);
  constexpr int B = batch_for(L, (int)sizeof(V));
  KParams p;
  p.ntrans = q.n_outer * q.inner;
  p.inner = q.inner;
  p.in_os = q.in_os;
  p.out_os = q.out_os;
  p.n_in = q.n_in;
  p.in_start = ((q.in_start % L) + L) % L;
  p.n_out = q.n_out;
  p.out_start = ((q.out_start % L) + L) % L;
  p.sign = q.sign;
  p.L4 = q.L4 > 0 ? q.L4 : 1;
  p.tw4_mod = q.L4 > 0 ? (q.L4 / L) : 1;
  p.tw4_at_load = q.tw4_at_load;
  const int64_t nblk = (p.ntrans + B - 1) / B;
  if (nblk <= 0) return;
  hipLaunchKernelGGL((fft_pass_kernel<T, L, EPT, B>), dim3((unsigned)nblk), dim3(B * (L / EPT)),
                     0, s, static_cast<const V*>(in), static_cast<V*>(out),
                     static_cast<const V*>(tw), static_cast<const V*>(q.tw4), p);
  GP_CHECK_LAUNCH();
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

bool fft_length_supported(int L) {
  switch (L) {
    case 8: case 16: case 32: case 64: case 128: case 256: case 512: case 1024: case 2048:
    case 4096: case 8192: case 24: case 48: case 96: case 192: case 384: case 768: case 1536:
    case 3072: case 6144:
      return true;
    default:
      return false;
  }
}

void fft_pass(int fp64, const FftPass& p, const void* in, void* out, const void* twiddles,
              hipStream_t s) {
  if (p.n_in > p.L || p.n_out > p.L || p.n_in < 0 || p.n_out < 0)
    throw Error{GP_EINVAL, "fft_pass: window longer than the transform"};
  if (fp64)
    dispatch<double>(p, in, out, twiddles, s);
  else
    dispatch<float>(p, in, out, twiddles, s);
}

}  // namespace gp
