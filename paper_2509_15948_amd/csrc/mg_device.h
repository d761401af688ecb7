// Device-side helpers shared by the mixgraph kernels (gfx950, wave64).
//
//  * complex float arithmetic on float2
//  * an LDS-resident, batched, Stockham-autosort complex FFT (radix-8 passes
//    plus one radix-4 or radix-2 pass for the rest of log2 n), data kept in LDS and each
//    butterfly's operands in registers between a read phase and a write phase,
//    so one buffer of n complex values per transform suffices
//  * fixed-order block reductions (no floating-point atomics anywhere, so every
//    result is bitwise reproducible)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MG_TWN 8192          // size of the LDS-FFT twiddle table
#define MG_BLOCK 256         // threads per workgroup for most kernels

__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 c_mulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 c_conj(float2 a) { return make_float2(a.x, -a.y); }

__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_scale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 c_conj(double2 a) { return make_double2(a.x, -a.y); }

// multiply by -i (DIR < 0) or +i (DIR > 0)
template <int DIR, typename V>
__device__ __forceinline__ V c_rot(V a) {
  V r;
  if (DIR < 0) {
    r.x = a.y;
    r.y = -a.x;
  } else {
    r.x = -a.y;
    r.y = a.x;
  }
  return r;
}

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n >> 1); }

// Twiddles of an N-point transform, staged in LDS by the calling kernel, so
// no butterfly reads global memory.  W_N = exp(-2 pi i / N).
//  * float2, N <= 1024: the full table lo[e] = W_N^e, each entry rounded once
//    from FP64 (copied from g[m] = exp(-2 pi i m / MG_TWN));
//  * float2, N > 1024: W_N^e = h (1 + d) with h = hi[e >> 6] = W_N^{64 (e >> 6)}
//    and d = lo[e & 63] = W_N^{e & 63} - 1 taken from gd (also rounded from
//    FP64), whose small magnitude keeps the product within about one rounding;
//  * double2: W_N^e = hi[e >> 6] lo[e & 63] (FP64 rounding is far below the
//    FP32 signals).
template <int N, typename V>
struct TwTab {
  static constexpr bool F32 = sizeof(V) == 8;
  static constexpr bool FULL = F32 && N <= 1024;
  static constexpr bool DELTA = F32 && N > 1024;
  static constexpr int NH = FULL ? 1 : (N >= 64 ? N / 64 : 1);
  static constexpr int NL = FULL ? N : 64;
  V hi[NH];
  V lo[NL];
};

// Fill t from the global tables (gd: W^m - 1, used for float2 with N > 1024);
// the caller synchronises before the first transform.
template <int N, typename V>
__device__ __forceinline__ void tw_fill(TwTab<N, V>& t, const V* __restrict__ g, const V* __restrict__ gd) {
  static_assert(N <= MG_TWN && MG_TWN % N == 0, "N must divide the table size");
  constexpr int S = MG_TWN / N;
  using T = TwTab<N, V>;
  for (int i = threadIdx.x; i < T::NH + T::NL; i += blockDim.x) {
    if (i < T::NH) {
      t.hi[i] = g[(64 * i * S) & (MG_TWN - 1)];
    } else {
      const int j = i - T::NH;
      t.lo[j] = T::DELTA ? gd[(j * S) & (MG_TWN - 1)] : g[(j * S) & (MG_TWN - 1)];
    }
  }
}

// W = exp(DIR * 2 pi i * e / N) for 0 <= e < N.
template <int DIR, int N, typename V>
__device__ __forceinline__ V tw_get(const TwTab<N, V>& t, int e) {
  using T = TwTab<N, V>;
  V w;
  if constexpr (T::FULL) {
    w = t.lo[e];
  } else if constexpr (T::DELTA) {
    const V h = t.hi[e >> 6], d = t.lo[e & 63];
    w.x = h.x + (h.x * d.x - h.y * d.y);
    w.y = h.y + (h.x * d.y + h.y * d.x);
  } else {
    w = c_mul(t.hi[e >> 6], t.lo[e & 63]);
  }
  if (DIR > 0) w.y = -w.y;
  return w;
}

// Stockham passes over B transforms of length N stored at buf[b * BS + i]:
// each butterfly reads its R inputs (stride N/R, contiguous across threads)
// into registers, the block synchronises, then every butterfly applies its
// twiddles, an R-point DFT and writes its R outputs.  Ns is the product of
// the radices of the earlier passes.  When B N / R is not a multiple of NT the
// threads past the last butterfly only take part in the barriers.

// 4-point DFT in place (natural order)
template <int DIR, typename V>
__device__ __forceinline__ void dft4(V& x0, V& x1, V& x2, V& x3) {
  const V t0 = c_add(x0, x2), t1 = c_sub(x0, x2);
  const V t2 = c_add(x1, x3), t3 = c_rot<DIR>(c_sub(x1, x3));
  x0 = c_add(t0, t2);
  x1 = c_add(t1, t3);
  x2 = c_sub(t0, t2);
  x3 = c_sub(t1, t3);
}

// LDS slot of element i of a transform stored with one spare slot after every
// 2^PAD elements (PAD = 0: no padding).  The early Stockham passes write with
// strides of 8 and 64 elements, which would put many lanes of a wave on the
// same LDS banks; the spare slots spread them.
template <int PAD>
__device__ __forceinline__ int lds_ix(int i) {
  return PAD ? i + (i >> PAD) : i;
}
template <int N, int PAD>
constexpr int lds_len() {
  return PAD ? N + (N >> PAD) : N;
}

template <int N, int R, int B, int BS, int NT, int DIR, int PAD, typename V>
__device__ __forceinline__ void fft_pass(V* buf, const TwTab<N, V>& tw, int Ns) {
  constexpr int Q = N / R;
  constexpr int NB = B * Q;
  constexpr int PER = (NB + NT - 1) / NT;
  V v[PER][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int g = tid + q * NT;
    if (NB % NT == 0 || g < NB) {
      const int b = g / Q, j = g % Q;
      const V* base = buf + b * BS;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = base[lds_ix<PAD>(j + r * Q)];
    }
  }
  __syncthreads();
  const int stride = N / (R * Ns);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int g = tid + q * NT;
    if (NB % NT != 0 && g >= NB) continue;
    const int b = g / Q, j = g % Q;
    const int k = j & (Ns - 1);
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[q][r] = c_mul(v[q][r], tw_get<DIR>(tw, r * k * stride));
    }
    V* base = buf + b * BS;
    const int idx = (j - k) * R + k;
    if (R == 2) {
      base[lds_ix<PAD>(idx)] = c_add(v[q][0], v[q][1]);
      base[lds_ix<PAD>(idx + Ns)] = c_sub(v[q][0], v[q][1]);
    } else if (R == 4) {
      dft4<DIR>(v[q][0], v[q][1], v[q][2], v[q][3]);
#pragma unroll
      for (int r = 0; r < 4; ++r) base[lds_ix<PAD>(idx + r * Ns)] = v[q][r];
    } else {  // R == 8: radix-2 step, then two 4-point DFTs (even and odd outputs)
      using S = decltype(v[q][0].x);
      const S h = (S)0.70710678118654752440;
      V a[4], c[4];
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        a[n] = c_add(v[q][n], v[q][n + 4]);
        c[n] = c_sub(v[q][n], v[q][n + 4]);
      }
      // c[n] *= W8^n, W8 = exp(DIR i pi / 4)
      {
        V t = c[1];
        // (1 + DIR i) / sqrt 2 times t
        c[1].x = h * (t.x - (S)DIR * t.y);
        c[1].y = h * (t.y + (S)DIR * t.x);
        c[2] = c_rot<DIR>(c[2]);
        t = c[3];
        // (-1 + DIR i) / sqrt 2 times t
        c[3].x = h * (-t.x - (S)DIR * t.y);
        c[3].y = h * (-t.y + (S)DIR * t.x);
      }
      dft4<DIR>(a[0], a[1], a[2], a[3]);
      dft4<DIR>(c[0], c[1], c[2], c[3]);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        base[lds_ix<PAD>(idx + (2 * r) * Ns)] = a[r];
        base[lds_ix<PAD>(idx + (2 * r + 1) * Ns)] = c[r];
      }
    }
  }
  __syncthreads();
}

// B unnormalised transforms of length N (4 <= N <= MG_TWN), in place in LDS:
// radix-8 passes, then one radix-4 or radix-2 pass for the remaining factor.
// DIR = -1: X[k] = sum x[n] e^{-2 pi i nk/N};  DIR = +1: the inverse sign.
// V is float2 or double2 (with twiddle tables of the same type).  Element i
// of transform b sits at buf[b * BS + lds_ix<PAD>(i)] (BS >= lds_len<N, PAD>).
// The caller must __syncthreads() after filling buf and tw.
template <int N, int B, int BS, int NT, int DIR, int PAD = 0, typename V>
__device__ __forceinline__ void fft_lds(V* buf, const TwTab<N, V>& tw) {
  constexpr int LOG = ilog2c(N);
  static_assert((1 << LOG) == N, "power of two");
  static_assert(B == 1 || BS >= lds_len<N, PAD>(), "transforms overlap");
  int Ns = 1;
#pragma unroll
  for (int p = 0; p < LOG / 3; ++p) {
    fft_pass<N, 8, B, BS, NT, DIR, PAD>(buf, tw, Ns);
    Ns *= 8;
  }
  if (LOG % 3 == 2) fft_pass<N, 4, B, BS, NT, DIR, PAD>(buf, tw, Ns);
  if (LOG % 3 == 1) fft_pass<N, 2, B, BS, NT, DIR, PAD>(buf, tw, Ns);
}

// Fixed-order sum over the workgroup; every thread gets the result.  Each
// wave folds its 64 lanes with an xor butterfly (a + b and b + a agree, so all
// lanes hold the same bits), then every thread adds the NT/64 wave sums in
// wave order.  red must hold NT/64 entries.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int NT, typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  static_assert(NT % 64 == 0, "whole waves");
  constexpr int NW = NT / 64;
  v = wave_sum(v);
  if (NW == 1) return v;
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  T r = red[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) r += red[i];
  __syncthreads();
  return r;
}

__device__ __forceinline__ float sigmoidf_(float x) { return 1.0f / (1.0f + __expf(-x)); }
