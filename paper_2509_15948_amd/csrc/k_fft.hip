// FIR convolution engine: FP32 four-step FFT of length N = N1 * N2 over HBM,
// each sub-transform staged in LDS (mg_device.h), used by every FIR processor
// of the console (Sec. 3.3 equalizer, Sec. 3.4 reverb, Sec. 3.7 multitap
// delay) for the forward convolution and for both backward correlations.
//
// Index map: x[n1 + N1 n2]; spectrum stored as S[k2][k1] = X[k2 + N2 k1].
//   cols  (KA): per column n1, FFT over n2 (length N2), twiddle W_N^{n1 k2},
//               write T[k2][n1]                       (loader functor fills x)
//   rows  (KB): per row pair (k2, N2-k2), FFT over n1 (length N1) -> S rows,
//               spectral product (with the mirrored bins that separate the
//               packed left/right spectra), inverse FFT over k1, twiddle
//               W_N^{-n1 k2}
//   icols (KC): per column n1, inverse FFT over k2, scale 1/N (store functor
//               consumes x: dry/wet output, input gradient or FIR gradient)
// Stereo signals are packed as l + i r; the FIRs as h_l + i h_r.  With N at
// least L plus the FIR's extent, circular convolution equals the linear one.
#include <cstring>
#include <vector>

#include "mg_device.h"
#include "mg_kernels.h"

namespace mg {

// threads per block: the column kernels hold 64-72 KB of LDS (two blocks per
// CU) and need few registers, so 1024 threads give 32 waves per CU (512
// threads, 16 waves, measured 4 % slower per step; 4096-element tiles, 64-byte
// row segments, slower still); row kernels use 512 threads from N1 = 1024 up
// (fewer rows of butterflies below), except the backward rows, which batch
// four transforms and take 1024 from N1 = 2048 (rowb_nt).  A pair of
// 3072-point rows is six 1024-point transforms, 768 radix-8 butterflies per
// pass: 768 threads take one each (512 left half the lanes idle in every
// second round) and, at 57 KB of LDS, two blocks still fit a CU (24 waves;
// the large console's step 49.2 -> 48.5 ms)
// Threads of a column workgroup: 512 for 1024-point columns (two butterflies
// per thread and pass; 45.05 -> 44.51 ms per step on the 3 x 2^20-point
// engine), 1024 for shorter ones (the 2^19-point engine's 256-point columns
// were 0.5 % slower at 512).  Two workgroups per CU (their LDS tiles fit
// twice), so the registers are held to 128 and 64.
template <int N2>
constexpr int col_nt() { return N2 >= 1024 ? 512 : 1024; }
template <int N2>
constexpr int col_min_waves() { return 2 * col_nt<N2>() / 256; }
// elements per thread whose loads are in flight together in the column
// passes (data, then twiddles): within 64 registers the short columns, whose
// transforms hold more registers, take smaller batches
template <int N2>
constexpr int col_batch() { return N2 >= 512 ? 8 : 4; }
template <int N2>
constexpr int col_tw_batch() { return N2 >= 512 ? 4 : 2; }
template <int N1>
constexpr int row_nt() { return N1 == 3072 ? 768 : (N1 >= 4096 ? 1024 : (N1 >= 1024 ? 512 : 256)); }
// the backward rows batch four transforms: 1024 threads from 2048 points
template <int N1>
constexpr int rowb_nt() { return N1 >= 2048 ? 1024 : row_nt<N1>(); }
// 2048-point backward rows: two 1024-thread workgroups per CU (70 KB of LDS
// each), registers held to 64; longer rows hold one workgroup per CU
template <int N1>
constexpr int rows_bwd_min_waves() { return N1 == 2048 ? 8 : 4; }

// Row transforms up to 2048 points and column transforms up to 256 keep one
// spare LDS slot per 16 points: the first two radix-8 passes then put at most
// two lanes on a bank where they put eight to sixteen (1.9 % faster per step
// at 2^19 points).  The longer transforms of a 2^22-point engine stay
// unpadded: there the larger blocks left less LDS to the other stream's
// kernels and the step measured 4 % slower.  The equalizer windows stay
// unpadded too (register spills: slower); the FP64 loss frames, with 16-byte
// points, keep one spare slot per 8 points instead.
template <int N, bool ROW>
constexpr int eng_pad() { return (ROW ? N <= 2048 : N <= 256) ? 4 : 0; }
template <int N, bool ROW>
constexpr int pad_len() { return lds_len<N, eng_pad<N, ROW>()>(); }
template <int N, bool ROW>
__device__ __forceinline__ int px(int i) { return lds_ix<eng_pad<N, ROW>()>(i); }

// Rows of 3072 points (3 x 1024) let the engine take N = 3 * 2^k where the
// next power of two would hold a third more points.  Such a row is
// transformed as three interleaved 1024-point transforms plus one radix-3
// pass: element i of the time-domain row sits at LDS slot (i % 3) 1024 + i / 3,
// frequency bin k at slot k.  Other rows are powers of two, in natural order
// (with the spare slots of eng_pad) on both sides.
template <int N1>
constexpr bool row3() { return N1 == 3072; }
template <int N1>
constexpr int row_tw() { return row3<N1>() ? 1024 : N1; }
// the three 1024-point transforms of a 3072-point row keep one spare slot
// per 16 points, as the power-of-two rows up to 2048 do (bit-identical
// results; the large console's step 48.4 -> 48.2 ms)
constexpr int R3_PAD = 4;
constexpr int R3_SB = lds_len<1024, R3_PAD>();
template <int N1>
constexpr int row_len() { return row3<N1>() ? 3 * R3_SB : pad_len<N1, true>(); }
template <int N1>
using RowTw = TwTab<row_tw<N1>(), float2>;
template <int N1>
__device__ __forceinline__ int tslot(int i) {
  if constexpr (row3<N1>()) return (i % 3) * R3_SB + lds_ix<R3_PAD>(i / 3);
  else return px<N1, true>(i);
}
template <int N1>
__device__ __forceinline__ int fslot(int k) {
  if constexpr (row3<N1>()) return (k >> 10) * R3_SB + lds_ix<R3_PAD>(k & 1023);
  else return px<N1, true>(k);
}

// W_N^e for e in [0, N) as h (1 + d), from two FP32 tables rounded from FP64
// on the host: twhi[j] = W_N^{1024 j} and twlo[j] = W_N^j - 1 (small, so the
// product adds little to the rounding of h).
constexpr int cmin(int a, int b) { return a < b ? a : b; }

// big_tw in two halves, the table loads and the product, so that a loop can
// issue the loads of all its twiddles before it uses the first one
struct TwRaw {
  float2 h, d;
};
__device__ __forceinline__ TwRaw big_tw_fetch(const float2* __restrict__ twhi, const float2* __restrict__ twlo,
                                              int64_t e) {
  return TwRaw{twhi[e >> 10], twlo[e & 1023]};
}
__device__ __forceinline__ float2 big_tw_make(const TwRaw& t) {
  const float2 h = t.h, d = t.d;
  return make_float2(h.x + (h.x * d.x - h.y * d.y), h.y + (h.x * d.y + h.y * d.x));
}
__device__ __forceinline__ float2 big_tw(const float2* __restrict__ twhi, const float2* __restrict__ twlo, int64_t e) {
  return big_tw_make(big_tw_fetch(twhi, twlo, e));
}

__device__ __forceinline__ int64_t signed_lag(int64_t n, int64_t N) { return n < N / 2 ? n : n - N; }

struct EngineArgs {
  int N, N1, N2;
  const float2* tw;
  const float2* twdl;
  const float2* twhi;
  const float2* twlo;
};

// Radix-3 pass of B 3072-point rows (row b at buf + 3072 b).  Forward (DIR =
// -1): slots r 1024 + k hold the 1024-point transforms F_r[k] of the
// elements 3m + r; X[k + 1024 s] = sum_r W_3072^{rk} W_3^{rs} F_r[k] goes to
// slot k + 1024 s.  Inverse (DIR = +1), the transpose: from the bins in
// natural order, slot r 1024 + k receives W_3072^{-rk} sum_s X[k + 1024 s]
// W_3^{-rs}, whose 1024-point inverse transforms give the elements 3m + r.
// W_3072^e = W_N^{e N2} comes from the engine's table of W_N.
// one bin of the radix-3 pass (slots kk, kk + R3_SB, kk + 2 R3_SB of row r)
template <int DIR>
__device__ __forceinline__ void radix3_bin(float2* r, int kk, float2 w1, float2 w2) {
  const float c3 = -0.5f, s3 = 0.866025403784438647f;
  float2 a0 = r[kk], a1 = r[R3_SB + kk], a2 = r[2 * R3_SB + kk];
  if (DIR < 0) {
    a1 = c_mul(a1, w1);
    a2 = c_mul(a2, w2);
  }
  // 3-point DFT with the sign of DIR
  const float2 sm = c_add(a1, a2), df = c_sub(a1, a2);
  const float2 m = make_float2(a0.x + c3 * sm.x, a0.y + c3 * sm.y);
  const float2 t = DIR < 0 ? make_float2(s3 * df.y, -s3 * df.x) : make_float2(-s3 * df.y, s3 * df.x);
  float2 y1 = c_add(m, t), y2 = c_sub(m, t);
  if (DIR > 0) {
    y1 = c_mul(y1, c_conj(w1));
    y2 = c_mul(y2, c_conj(w2));
  }
  r[kk] = c_add(a0, sm);
  r[R3_SB + kk] = y1;
  r[2 * R3_SB + kk] = y2;
}

// LEAN: one bin's twiddle loads in flight at a time (kernels held to few
// registers); otherwise every bin's twiddles are fetched first.
template <int B, int NT, int DIR, bool LEAN>
__device__ __forceinline__ void radix3_pass(float2* buf, const EngineArgs& ea) {
  if constexpr (LEAN) {
    for (int idx = threadIdx.x; idx < B * 1024; idx += NT) {
      const int k = idx & 1023;
      radix3_bin<DIR>(buf + (idx >> 10) * (3 * R3_SB), lds_ix<R3_PAD>(k),
                      big_tw(ea.twhi, ea.twlo, (int64_t)k * ea.N2), big_tw(ea.twhi, ea.twlo, (int64_t)(2 * k) * ea.N2));
    }
  } else {
    constexpr int PER = (B * 1024 + NT - 1) / NT;
    TwRaw t1[PER], t2[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int k = (threadIdx.x + i * NT) & 1023;  // past the end: in-bounds table entries, unused
      t1[i] = big_tw_fetch(ea.twhi, ea.twlo, (int64_t)k * ea.N2);
      t2[i] = big_tw_fetch(ea.twhi, ea.twlo, (int64_t)(2 * k) * ea.N2);
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int idx = threadIdx.x + i * NT;
      if (idx >= B * 1024) break;
      const int k = idx & 1023;
      radix3_bin<DIR>(buf + (idx >> 10) * (3 * R3_SB), lds_ix<R3_PAD>(k), big_tw_make(t1[i]), big_tw_make(t2[i]));
    }
  }
}

// B row transforms in LDS (rows at stride row_len<N1>), unnormalised; ends
// with a barrier like fft_lds.
template <int N1, int B, int NT, int DIR, bool LEAN = false>
__device__ __forceinline__ void row_fft(float2* buf, const RowTw<N1>& tt, const EngineArgs& ea) {
  if constexpr (row3<N1>()) {
    if (DIR > 0) {
      radix3_pass<B, NT, DIR, LEAN>(buf, ea);
      __syncthreads();
    }
    fft_lds<1024, 3 * B, R3_SB, NT, DIR, R3_PAD>(buf, tt);
    if (DIR < 0) {
      radix3_pass<B, NT, DIR, LEAN>(buf, ea);
      __syncthreads();
    }
  } else {
    fft_lds<N1, B, pad_len<N1, true>(), NT, DIR, eng_pad<N1, true>()>(buf, tt);
  }
}

// ---------------------------------------------------------------- loaders
struct NodeView {
  const NodeDesc* desc;
  const float* dry;
  const float* U;
  const float* G;
  int64_t L;
  int C;
};

__device__ __forceinline__ const float* node_input(const NodeView& v, const NodeDesc& d, int64_t& cs) {
  if (d.in_kind == 0) {
    cs = (v.C == 1) ? 0 : v.L;
    return v.dry + (int64_t)d.in_slot * v.C * v.L;
  }
  cs = v.L;
  return v.U + (int64_t)d.in_slot * 2 * v.L;
}

// Loaders of the column pass: fetch(n) issues the global loads of element n,
// finish(n, raw) turns them into the packed value (and does any per-element
// arithmetic, in the order of the calls); BATCH elements are fetched before
// the first is finished.  Stores of the inverse column pass work the same
// way: fetch(n) loads what store(n, value, raw) needs.

// forward input u packed l + i r
struct LdSignal {
  NodeView v;
  const float* u;
  int64_t cs;
  using Raw = float2;
  static constexpr int BATCH = 8;
  __device__ void begin(int j) {
    const NodeDesc d = v.desc[j];
    u = node_input(v, d, cs);
  }
  __device__ Raw fetch(int64_t n) const { return n < v.L ? make_float2(u[n], u[cs + n]) : make_float2(0.f, 0.f); }
  __device__ float2 finish(int64_t, const Raw& r) { return r; }
  template <int NT>
  __device__ void end(int, int) {}
};

// compact FIR [2][Nh] (or [Nh] shared) whose first tap sits at lag lag0
struct LdFir {
  const NodeDesc* desc;
  const float* h;      // base of the compact FIRs of this type
  int64_t Nh, lag0, N, stride;
  int shared;          // 1: one FIR for both channels
  const float* hl;
  const float* hr;
  __device__ void begin(int j) {
    const NodeDesc d = desc[j];
    hl = h + (int64_t)d.aux * stride;
    hr = shared ? hl : hl + Nh;
  }
  using Raw = float2;
  static constexpr int BATCH = 8;
  __device__ Raw fetch(int64_t n) const {
    const int64_t i = signed_lag(n, N) - lag0;
    return (i >= 0 && i < Nh) ? make_float2(hl[i], hr[i]) : make_float2(0.f, 0.f);
  }
  __device__ float2 finish(int64_t, const Raw& r) { return r; }
  __device__ float2 load(int64_t n) const { return fetch(n); }
  template <int NT>
  __device__ void end(int, int) {}
};

// backward: dL/dybar = w dL/dy + alpha_g s ybar_m / E_ybar, and the dry/wet
// partial sum of dL/dy * (ybar - u)
struct LdGrad {
  NodeView v;
  const float* ybar_base;
  const double* lg;
  const float* wet;
  const float* mask;
  float alpha_g;
  int yb0;             // ybar slot of type row 0
  float* part;
  int PB;
  const float* dy;
  const float* yb;
  const float* u;
  int64_t cs;
  float w, kreg;
  float acc;
  __device__ void begin(int j) {
    const NodeDesc d = v.desc[j];
    u = node_input(v, d, cs);
    dy = v.G + (int64_t)d.gout * 2 * v.L;
    yb = ybar_base + (int64_t)(yb0 + d.aux) * 2 * v.L;
    w = node_w(wet, mask, d);
    const double Ey = lg[2 * j] + 1e-12, Eu = lg[2 * j + 1] + 1e-12;
    const double diff = 0.5 * log(Ey) - 0.5 * log(Eu);
    const double s = diff > 0 ? 1.0 : (diff < 0 ? -1.0 : 0.0);
    kreg = (float)((double)alpha_g * s / Ey);
    acc = 0.f;
  }
  struct Raw {
    float gl, gr, bl, br, ul, ur;
  };
  static constexpr int BATCH = 4;
  __device__ Raw fetch(int64_t n) const {
    if (n >= v.L) return Raw{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    return Raw{dy[n], dy[v.L + n], yb[n], yb[v.L + n], u[n], u[cs + n]};
  }
  __device__ float2 finish(int64_t n, const Raw& r) {
    if (n >= v.L) return make_float2(0.f, 0.f);
    acc += r.gl * (r.bl - r.ul) + r.gr * (r.br - r.ur);
    const float rm = kreg * (r.bl + r.br);
    return make_float2(w * r.gl + rm, w * r.gr + rm);
  }
  template <int NT>
  __device__ void end(int j, int blk) {
    __shared__ float red[NT];
    const float s = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) part[((int64_t)j * PB + blk) * PK + 2] = s;
  }
};

// ---------------------------------------------------------------- stores
// forward: ybar from the engine; y = w ybar + (1 - w) u; L_g energies
struct StFwd {
  NodeView v;
  float* ybar_base;
  const float* wet;
  const float* mask;
  int yb0;
  float* part;
  int PB;
  float* y;
  float* yb;
  const float* u;
  int64_t cs;
  float w, ey, eu;
  __device__ void begin(int j) {
    const NodeDesc d = v.desc[j];
    u = node_input(v, d, cs);
    y = const_cast<float*>(v.U) + (int64_t)d.out_slot * 2 * v.L;
    yb = ybar_base ? ybar_base + (int64_t)(yb0 + d.aux) * 2 * v.L : nullptr;
    w = node_w(wet, mask, d);
    ey = eu = 0.f;
  }
  using Raw = float2;
  static constexpr int BATCH = 8;
  __device__ Raw fetch(int64_t n) const { return n < v.L ? make_float2(u[n], u[cs + n]) : make_float2(0.f, 0.f); }
  __device__ void store(int64_t n, float2 val, const Raw& ur) {
    if (n >= v.L) return;
    const float l = ur.x, r = ur.y;
    if (yb) {
      yb[n] = val.x;
      yb[v.L + n] = val.y;
    }
    y[n] = w * val.x + (1.0f - w) * l;
    y[v.L + n] = w * val.y + (1.0f - w) * r;
    const float m = val.x + val.y, um = l + r;
    ey += m * m;
    eu += um * um;
  }
  template <int NT>
  __device__ void end(int j, int blk) {
    __shared__ float red[NT];
    const float a = block_sum<NT>(ey, red);
    const float b = block_sum<NT>(eu, red);
    if (threadIdx.x == 0) {
      part[((int64_t)j * PB + blk) * PK + 0] = a;
      part[((int64_t)j * PB + blk) * PK + 1] = b;
    }
  }
};

// backward dL/du = (1 - w) dL/dy + corr(dL/dybar, h) - alpha_g s u_m / E_u
struct StGradU {
  NodeView v;
  const double* lg;
  const float* wet;
  const float* mask;
  float alpha_g;
  float* gin;
  const float* dy;
  const float* u;
  int64_t cs;
  float w, kreg;
  bool active;
  __device__ void begin(int j) {
    const NodeDesc d = v.desc[j];
    active = d.gin >= 0;
    gin = active ? const_cast<float*>(v.G) + (int64_t)d.gin * 2 * v.L : nullptr;
    dy = v.G + (int64_t)d.gout * 2 * v.L;
    u = node_input(v, d, cs);
    w = node_w(wet, mask, d);
    const double Ey = lg[2 * j] + 1e-12, Eu = lg[2 * j + 1] + 1e-12;
    const double diff = 0.5 * log(Ey) - 0.5 * log(Eu);
    const double s = diff > 0 ? 1.0 : (diff < 0 ? -1.0 : 0.0);
    kreg = (float)((double)alpha_g * s / Eu);
  }
  using Raw = float4;  // dL/dy (l, r), u (l, r)
  static constexpr int BATCH = 4;
  __device__ Raw fetch(int64_t n) const {
    if (!active || n >= v.L) return make_float4(0.f, 0.f, 0.f, 0.f);
    return make_float4(dy[n], dy[v.L + n], u[n], u[cs + n]);
  }
  __device__ void store(int64_t n, float2 val, const Raw& r) {
    if (!active || n >= v.L) return;
    const float um = r.z + r.w;
    gin[n] = (1.0f - w) * r.x + val.x - kreg * um;
    gin[v.L + n] = (1.0f - w) * r.y + val.y - kreg * um;
  }
  template <int NT>
  __device__ void end(int, int) {}
};

// backward dL/dh at the FIR's lags: compact [2][Nh] (shared: [Nh], channels summed)
struct StGradH {
  const NodeDesc* desc;
  float* dh;
  int64_t Nh, lag0, N, stride;
  int shared;
  float* o;
  __device__ void begin(int j) { o = dh + (int64_t)desc[j].aux * stride; }
  struct Raw {};
  static constexpr int BATCH = 8;
  __device__ Raw fetch(int64_t) const { return Raw{}; }
  __device__ void store(int64_t n, float2 val, const Raw&) {
    const int64_t i = signed_lag(n, N) - lag0;
    if (i < 0 || i >= Nh) return;
    if (shared) o[i] = val.x + val.y;
    else {
      o[i] = val.x;
      o[Nh + i] = val.y;
    }
  }
  template <int NT>
  __device__ void end(int, int) {}
};

// Column tile of workgroup b of n.  Tiles narrower than a 128-byte line
// (TC < 16 columns) are ordered for the XCDs: workgroups are dealt to the
// eight XCDs in turn and each XCD has its own L2, so workgroup b takes tile
// (b % 8) (n / 8) + b / 8; neighbouring tiles, whose row segments share L2
// lines, then run on one XCD at about the same time.  Partial sums stay
// indexed by tile.
template <int TC>
__device__ __forceinline__ int col_tile(int b, int n) {
  if (TC >= 16 || n % 8) return b;
  return (b % 8) * (n / 8) + b / 8;
}

// ---------------------------------------------------------------- KA: columns forward
template <int N2, int TC, typename LD>
__global__ __launch_bounds__(col_nt<N2>(), col_min_waves<N2>()) void k_cols(LD ld, float2* __restrict__ T, EngineArgs ea) {
  constexpr int BS = pad_len<N2, false>() + 1;
  constexpr int NT = col_nt<N2>();
  __shared__ float2 buf[TC * BS];
  __shared__ TwTab<N2, float2> tt;
  tw_fill<N2>(tt, ea.tw, ea.twdl);
  const int j = blockIdx.y;
  const int tile = col_tile<TC>(blockIdx.x, gridDim.x);
  const int c0 = tile * TC;
  const int N1 = ea.N1;
  ld.begin(j);
  constexpr int PER = TC * N2 / NT;
  static_assert(TC * N2 % NT == 0, "a column tile is a whole number of passes");
  constexpr int BATCH = cmin(cmin(LD::BATCH, col_batch<N2>()), PER);
  static_assert(PER % BATCH == 0, "whole batches");
#pragma unroll 1  // one batch of loads in flight at a time
  for (int k0 = 0; k0 < PER; k0 += BATCH) {
    typename LD::Raw raw[BATCH];
#pragma unroll
    for (int k = 0; k < BATCH; ++k) {
      const int idx = threadIdx.x + (k0 + k) * NT;
      raw[k] = ld.fetch((int64_t)(c0 + idx % TC) + (int64_t)N1 * (idx / TC));
    }
#pragma unroll
    for (int k = 0; k < BATCH; ++k) {
      const int idx = threadIdx.x + (k0 + k) * NT;
      const int n2 = idx / TC, cc = idx % TC;
      buf[cc * BS + px<N2, false>(n2)] = ld.finish((int64_t)(c0 + cc) + (int64_t)N1 * n2, raw[k]);
    }
  }
  ld.template end<NT>(j, tile);
  __syncthreads();
  fft_lds<N2, TC, BS, NT, -1, eng_pad<N2, false>()>(buf, tt);
  float2* Tn = T + (int64_t)j * ea.N;
  constexpr int TB = col_tw_batch<N2>();  // twiddles fetched per batch
  static_assert(PER % TB == 0, "whole batches");
#pragma unroll 1  // one batch of loads in flight at a time
  for (int k0 = 0; k0 < PER; k0 += TB) {
    TwRaw tw[TB];
#pragma unroll
    for (int k = 0; k < TB; ++k) {
      const int idx = threadIdx.x + (k0 + k) * NT;
      tw[k] = big_tw_fetch(ea.twhi, ea.twlo, (int64_t)(c0 + idx % TC) * (idx / TC));  // n1 k2 < N
    }
#pragma unroll
    for (int k = 0; k < TB; ++k) {
      const int idx = threadIdx.x + (k0 + k) * NT;
      const int k2 = idx / TC, cc = idx % TC;
      const int n1 = c0 + cc;
      Tn[(int64_t)k2 * N1 + n1] = c_mul(buf[cc * BS + px<N2, false>(k2)], big_tw_make(tw[k]));
    }
  }
}

// ---------------------------------------------------------------- KC: columns inverse
template <int N2, int TC, typename ST>
__global__ __launch_bounds__(col_nt<N2>(), col_min_waves<N2>()) void k_icols(ST st, const float2* __restrict__ T, EngineArgs ea) {
  constexpr int BS = pad_len<N2, false>() + 1;
  constexpr int NT = col_nt<N2>();
  __shared__ float2 buf[TC * BS];
  __shared__ TwTab<N2, float2> tt;
  tw_fill<N2>(tt, ea.tw, ea.twdl);
  const int j = blockIdx.y;
  const int tile = col_tile<TC>(blockIdx.x, gridDim.x);
  const int c0 = tile * TC;
  const int N1 = ea.N1;
  const float2* Tn = T + (int64_t)j * ea.N;
  constexpr int PER = TC * N2 / NT;
  static_assert(TC * N2 % NT == 0, "a column tile is a whole number of passes");
  constexpr int XB = col_batch<N2>();
  static_assert(PER % XB == 0, "whole batches");
#pragma unroll 1  // one batch of loads in flight at a time
  for (int k0 = 0; k0 < PER; k0 += XB) {
    float2 x[XB];
#pragma unroll
    for (int k = 0; k < XB; ++k) {
      const int idx = threadIdx.x + (k0 + k) * NT;
      x[k] = Tn[(int64_t)(idx / TC) * N1 + c0 + idx % TC];
    }
#pragma unroll
    for (int k = 0; k < XB; ++k) {
      const int idx = threadIdx.x + (k0 + k) * NT;
      buf[(idx % TC) * BS + px<N2, false>(idx / TC)] = x[k];
    }
  }
  __syncthreads();
  fft_lds<N2, TC, BS, NT, +1, eng_pad<N2, false>()>(buf, tt);
  const float sc = 1.0f / (float)ea.N;
  st.begin(j);
  constexpr int BATCH = cmin(cmin(ST::BATCH, col_batch<N2>()), PER);
  static_assert(PER % BATCH == 0, "whole batches");
#pragma unroll 1  // one batch of loads in flight at a time
  for (int k0 = 0; k0 < PER; k0 += BATCH) {
    typename ST::Raw raw[BATCH];
#pragma unroll
    for (int k = 0; k < BATCH; ++k) {
      const int idx = threadIdx.x + (k0 + k) * NT;
      raw[k] = st.fetch((int64_t)(c0 + idx % TC) + (int64_t)N1 * (idx / TC));
    }
#pragma unroll
    for (int k = 0; k < BATCH; ++k) {
      const int idx = threadIdx.x + (k0 + k) * NT;
      const int n2 = idx / TC, cc = idx % TC;
      st.store((int64_t)(c0 + cc) + (int64_t)N1 * n2, c_scale(buf[cc * BS + px<N2, false>(n2)], sc), raw[k]);
    }
  }
  st.template end<NT>(j, tile);
}

// ---------------------------------------------------------------- KB: rows
// the two rows of workgroup p: (0, N2/2) for p = 0, else (p, N2 - p)
__device__ __forceinline__ void row_pair(int p, int N2, int& ra, int& rb) {
  ra = p;
  rb = (p == 0) ? N2 / 2 : N2 - p;
}

// pair q of workgroup p -> LDS indices (ia, ib) of bin k and bin -k.
// returns false when q is past the end.
template <int N1>
__device__ __forceinline__ bool mirror_pair(int p, int q, int& ia, int& ib) {
  if (p != 0) {
    if (q >= N1) return false;
    ia = q;
    ib = N1 + (N1 - 1 - q);
    return true;
  }
  if (q <= N1 / 2) {  // row 0: k1 <-> (N1 - k1) mod N1
    ia = q;
    ib = q == 0 ? 0 : N1 - q;
    return true;
  }
  q -= N1 / 2 + 1;   // row N2/2: k1 <-> N1 - 1 - k1
  if (q >= N1 / 2) return false;
  ia = N1 + q;
  ib = N1 + (N1 - 1 - q);
  return true;
}

__device__ __forceinline__ void split_lr(float2 z, float2 zm, float2& l, float2& r) {
  // l = (z + conj(zm)) / 2, r = -i (z - conj(zm)) / 2
  l = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
  const float2 d = make_float2(0.5f * (z.x - zm.x), 0.5f * (z.y + zm.y));
  r = make_float2(d.y, -d.x);
}

__device__ __forceinline__ float2 pack_lr(float2 l, float2 r) {  // l + i r
  return make_float2(l.x - r.y, l.y + r.x);
}

// LDS slot of element i in [0, 2 N1) of a row pair (row a, then row b)
template <int N1>
__device__ __forceinline__ int rslot(int i) {
  return i < N1 ? fslot<N1>(i) : row_len<N1>() + fslot<N1>(i - N1);
}

// Row loads and stores with NT threads: every thread issues the global loads
// of its row elements (all of them) or of their twiddles (two elements at a
// time) before it uses the first.  LEAN: one element's loads in flight, for
// kernels held to few registers.
template <int N1, int NT, bool LEAN = false>
__device__ __forceinline__ void load_rows(float2* buf, const float2* __restrict__ Tn, int ra, int rb) {
  static_assert(N1 % NT == 0, "whole passes");
  constexpr int PER = N1 / NT;
  if constexpr (LEAN) {
    for (int i = threadIdx.x; i < N1; i += NT) {
      buf[tslot<N1>(i)] = Tn[(int64_t)ra * N1 + i];
      buf[row_len<N1>() + tslot<N1>(i)] = Tn[(int64_t)rb * N1 + i];
    }
    return;
  }
  constexpr int LB = PER;
#pragma unroll
  for (int k0 = 0; k0 < PER; k0 += LB) {
    float2 a[LB], b[LB];
#pragma unroll
    for (int k = 0; k < LB; ++k) {
      const int i = threadIdx.x + (k0 + k) * NT;
      a[k] = Tn[(int64_t)ra * N1 + i];
      b[k] = Tn[(int64_t)rb * N1 + i];
    }
#pragma unroll
    for (int k = 0; k < LB; ++k) {
      const int i = threadIdx.x + (k0 + k) * NT;
      buf[tslot<N1>(i)] = a[k];
      buf[row_len<N1>() + tslot<N1>(i)] = b[k];
    }
  }
}

template <int N1, int NT, bool LEAN = false>
__device__ __forceinline__ void store_rows(const float2* buf, float2* __restrict__ To, int ra, int rb,
                                           const EngineArgs& ea) {
  static_assert(N1 % NT == 0, "whole passes");
  constexpr int PER = N1 / NT;
  if constexpr (LEAN) {
    for (int i = threadIdx.x; i < N1; i += NT) {
      const float2 wa = big_tw(ea.twhi, ea.twlo, (int64_t)i * ra);  // i ra < N
      const float2 wb = big_tw(ea.twhi, ea.twlo, (int64_t)i * rb);
      To[(int64_t)ra * N1 + i] = c_mul(buf[tslot<N1>(i)], c_conj(wa));
      To[(int64_t)rb * N1 + i] = c_mul(buf[row_len<N1>() + tslot<N1>(i)], c_conj(wb));
    }
    return;
  }
  constexpr int SB = PER < 2 ? 1 : 2;  // elements whose twiddle loads are in flight together
#pragma unroll
  for (int k0 = 0; k0 < PER; k0 += SB) {
    TwRaw ta[SB], tb[SB];
#pragma unroll
    for (int k = 0; k < SB && k0 + k < PER; ++k) {
      const int i = threadIdx.x + (k0 + k) * NT;
      ta[k] = big_tw_fetch(ea.twhi, ea.twlo, (int64_t)i * ra);  // i ra < N
      tb[k] = big_tw_fetch(ea.twhi, ea.twlo, (int64_t)i * rb);
    }
#pragma unroll
    for (int k = 0; k < SB && k0 + k < PER; ++k) {
      const int i = threadIdx.x + (k0 + k) * NT;
      To[(int64_t)ra * N1 + i] = c_mul(buf[tslot<N1>(i)], c_conj(big_tw_make(ta[k])));
      To[(int64_t)rb * N1 + i] = c_mul(buf[row_len<N1>() + tslot<N1>(i)], c_conj(big_tw_make(tb[k])));
    }
  }
}

// store_rows of two row pairs that share their twiddles (x -> To, z -> Tz)
template <int N1, int NT>
__device__ __forceinline__ void store_rows2(const float2* x, const float2* z, float2* __restrict__ To,
                                            float2* __restrict__ Tz, int ra, int rb, const EngineArgs& ea) {
  static_assert(N1 % NT == 0, "whole passes");
  constexpr int PER = N1 / NT;
  constexpr int SB = PER < 2 ? PER : 2;
#pragma unroll
  for (int k0 = 0; k0 < PER; k0 += SB) {
    TwRaw ta[SB], tb[SB];
#pragma unroll
    for (int k = 0; k < SB && k0 + k < PER; ++k) {
      const int i = threadIdx.x + (k0 + k) * NT;
      ta[k] = big_tw_fetch(ea.twhi, ea.twlo, (int64_t)i * ra);  // i ra < N
      tb[k] = big_tw_fetch(ea.twhi, ea.twlo, (int64_t)i * rb);
    }
#pragma unroll
    for (int k = 0; k < SB && k0 + k < PER; ++k) {
      const int i = threadIdx.x + (k0 + k) * NT;
      const float2 wa = c_conj(big_tw_make(ta[k]));
      const float2 wb = c_conj(big_tw_make(tb[k]));
      const int ia = tslot<N1>(i), ib = row_len<N1>() + tslot<N1>(i);
      To[(int64_t)ra * N1 + i] = c_mul(x[ia], wa);
      To[(int64_t)rb * N1 + i] = c_mul(x[ib], wb);
      Tz[(int64_t)ra * N1 + i] = c_mul(z[ia], wa);
      Tz[(int64_t)rb * N1 + i] = c_mul(z[ib], wb);
    }
  }
}

// spectrum only: S rows of the FIR -> ZH
template <int N1>
__global__ __launch_bounds__(row_nt<N1>()) void k_rows_spec(const float2* __restrict__ T, float2* __restrict__ Z,
                                                         int z0, const NodeDesc* __restrict__ desc, EngineArgs ea) {
  __shared__ float2 buf[2 * row_len<N1>()];
  __shared__ RowTw<N1> tt;
  tw_fill<row_tw<N1>()>(tt, ea.tw, ea.twdl);
  const int j = blockIdx.y;
  int ra, rb;
  row_pair(blockIdx.x, ea.N2, ra, rb);
  load_rows<N1, row_nt<N1>()>(buf, T + (int64_t)j * ea.N, ra, rb);
  __syncthreads();
  row_fft<N1, 2, row_nt<N1>(), -1>(buf, tt, ea);
  float2* Zn = Z + (int64_t)(z0 + desc[j].aux) * ea.N;
  for (int i = threadIdx.x; i < N1; i += row_nt<N1>()) {
    Zn[(int64_t)ra * N1 + i] = buf[fslot<N1>(i)];
    Zn[(int64_t)rb * N1 + i] = buf[row_len<N1>() + fslot<N1>(i)];
  }
}

// FIR spectrum rows straight from the compact FIR.  The FIR's taps occupy
// few of the N2 rows of the index map n = n1 + N1 n2 (lags [lag0, lag0 + Nh)
// are short next to N), so the column transform is a direct sum over those
// rows: for the row pair (ra, rb) and every n1,
//   t[k2][n1] = W_N^{n1 k2} sum_{n2 in S} h[n1 + N1 n2] W_N2^{n2 k2},
// with S the rows 0 .. khi-1 (lags from 0 up) and the last klo rows (the
// negative lags, circularly at the end); then the row FFT of k_rows_spec.
// This replaces the column pass over all N2 rows, most of them zero, and the
// HBM round trip of its N-point intermediate, but every row-pair workgroup
// reads all the FIR's rows again: on the 3 x 2^20-point engine with 64 nodes
// a stage took 2.2 ms at 9 rows against 3.1 ms for the column path, and
// 5.5 ms at 32 rows.  So only FIRs within FIRSPEC_MAXK rows take it.
constexpr int FIRSPEC_MAXK = 16;
template <int N1>
__global__ __launch_bounds__(row_nt<N1>()) void k_rows_firspec(LdFir ld, float2* __restrict__ Z, int z0, int khi,
                                                             int klo, const NodeDesc* __restrict__ desc,
                                                             EngineArgs ea) {
  __shared__ float2 buf[2 * row_len<N1>()];
  __shared__ RowTw<N1> tt;
  __shared__ float2 twa[FIRSPEC_MAXK], twb[FIRSPEC_MAXK];
  tw_fill<row_tw<N1>()>(tt, ea.tw, ea.twdl);
  const int j = blockIdx.y;
  int ra, rb;
  row_pair(blockIdx.x, ea.N2, ra, rb);
  const int nS = khi + klo;
  for (int q = threadIdx.x; q < nS; q += row_nt<N1>()) {
    const int64_t n2 = q < khi ? q : ea.N2 - klo + (q - khi);
    // W_N2^{n2 r} = W_N^{N1 ((n2 r) mod N2)}
    twa[q] = big_tw(ea.twhi, ea.twlo, (int64_t)N1 * ((n2 * ra) % ea.N2));
    twb[q] = big_tw(ea.twhi, ea.twlo, (int64_t)N1 * ((n2 * rb) % ea.N2));
  }
  ld.begin(j);
  __syncthreads();
  for (int n1 = threadIdx.x; n1 < N1; n1 += row_nt<N1>()) {
    // FP64 accumulation: a direct FP32 sum over up to 64 rows rounds about
    // twice as much as the column FFT it replaces; in FP64 it rounds less
    double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0;
    for (int q = 0; q < nS; ++q) {
      const int64_t n2 = q < khi ? q : ea.N2 - klo + (q - khi);
      const float2 x = ld.load((int64_t)n1 + (int64_t)N1 * n2);
      const float2 ta = twa[q], tb = twb[q];
      ax += (double)x.x * ta.x - (double)x.y * ta.y;
      ay += (double)x.x * ta.y + (double)x.y * ta.x;
      bx += (double)x.x * tb.x - (double)x.y * tb.y;
      by += (double)x.x * tb.y + (double)x.y * tb.x;
    }
    const float2 wa = big_tw(ea.twhi, ea.twlo, (int64_t)n1 * ra);  // n1 ra < N
    const float2 wb = big_tw(ea.twhi, ea.twlo, (int64_t)n1 * rb);
    buf[tslot<N1>(n1)] = make_float2((float)(ax * wa.x - ay * wa.y), (float)(ax * wa.y + ay * wa.x));
    buf[row_len<N1>() + tslot<N1>(n1)] = make_float2((float)(bx * wb.x - by * wb.y), (float)(bx * wb.y + by * wb.x));
  }
  __syncthreads();
  row_fft<N1, 2, row_nt<N1>(), -1>(buf, tt, ea);
  float2* Zn = Z + (int64_t)(z0 + desc[j].aux) * ea.N;
  for (int i = threadIdx.x; i < N1; i += row_nt<N1>()) {
    Zn[(int64_t)ra * N1 + i] = buf[fslot<N1>(i)];
    Zn[(int64_t)rb * N1 + i] = buf[row_len<N1>() + fslot<N1>(i)];
  }
}

// 3072-point rows: registers held to 80 (6 waves per SIMD), so that two
// 768-thread workgroups share a CU; the padded index arithmetic took 81
template <int N1>
constexpr int rows_conv_min_waves() { return N1 == 3072 ? 6 : 1; }
// under that cap the kernel keeps one element's loads in flight at a time:
// batched loads would spill
template <int N1>
constexpr bool rows_conv_lean() { return rows_conv_min_waves<N1>() > 1; }

// the product of one mirrored bin pair (LDS slots sa, sb; FIR bins ha, hb)
__device__ __forceinline__ void conv_pair(float2* buf, int sa, int sb, float2 ha, float2 hb) {
  const float2 za = buf[sa], zb = buf[sb];
  float2 xl, xr, hl, hr;
  split_lr(za, zb, xl, xr);
  split_lr(ha, hb, hl, hr);
  const float2 ya = pack_lr(c_mul(xl, hl), c_mul(xr, hr));
  split_lr(zb, za, xl, xr);
  split_lr(hb, ha, hl, hr);
  const float2 yb = pack_lr(c_mul(xl, hl), c_mul(xr, hr));
  buf[sa] = ya;
  buf[sb] = yb;
}

// forward convolution: Y = Xl Hl + i Xr Hr
template <int N1>
__global__ __launch_bounds__(row_nt<N1>(), rows_conv_min_waves<N1>()) void k_rows_conv(const float2* __restrict__ Tin, float2* __restrict__ Tout,
                                                         const float2* __restrict__ ZH, float2* __restrict__ ZU,
                                                         int z0, const NodeDesc* __restrict__ desc, EngineArgs ea) {
  __shared__ float2 buf[2 * row_len<N1>()];
  __shared__ RowTw<N1> tt;
  tw_fill<row_tw<N1>()>(tt, ea.tw, ea.twdl);
  const int j = blockIdx.y;
  const int p = blockIdx.x;
  int ra, rb;
  row_pair(p, ea.N2, ra, rb);
  constexpr bool LEAN = rows_conv_lean<N1>();
  load_rows<N1, row_nt<N1>(), LEAN>(buf, Tin + (int64_t)j * ea.N, ra, rb);
  __syncthreads();
  row_fft<N1, 2, row_nt<N1>(), -1, LEAN>(buf, tt, ea);
  const int64_t zr = (int64_t)(z0 + desc[j].aux) * ea.N;
  const float2* H = ZH + zr;
  if (ZU) {  // keep the input spectrum for the backward
    float2* Zs = ZU + zr;
    for (int i = threadIdx.x; i < N1; i += row_nt<N1>()) {
      Zs[(int64_t)ra * N1 + i] = buf[fslot<N1>(i)];
      Zs[(int64_t)rb * N1 + i] = buf[row_len<N1>() + fslot<N1>(i)];
    }
    __syncthreads();  // every bin stored before the product below overwrites it
  }
  if constexpr (LEAN) {
    for (int q = threadIdx.x; q < N1 + 1; q += row_nt<N1>()) {
      int ia, ib;
      if (!mirror_pair<N1>(p, q, ia, ib)) continue;
      const int64_t ga = (ia < N1) ? (int64_t)ra * N1 + ia : (int64_t)rb * N1 + (ia - N1);
      const int64_t gb = (ib < N1) ? (int64_t)ra * N1 + ib : (int64_t)rb * N1 + (ib - N1);
      conv_pair(buf, rslot<N1>(ia), rslot<N1>(ib), H[ga], H[gb]);
    }
  } else {
    constexpr int NQ = (N1 + 1 + row_nt<N1>() - 1) / row_nt<N1>();
    constexpr int QB = 3;  // pairs whose spectrum loads are in flight together
#pragma unroll
    for (int k0 = 0; k0 < NQ; k0 += QB) {
      float2 hA[QB], hB[QB];
#pragma unroll
      for (int k = k0; k < k0 + QB && k < NQ; ++k) {
        int ia, ib;
        if (!mirror_pair<N1>(p, threadIdx.x + k * row_nt<N1>(), ia, ib)) continue;
        hA[k - k0] = H[(ia < N1) ? (int64_t)ra * N1 + ia : (int64_t)rb * N1 + (ia - N1)];
        hB[k - k0] = H[(ib < N1) ? (int64_t)ra * N1 + ib : (int64_t)rb * N1 + (ib - N1)];
      }
#pragma unroll
      for (int k = k0; k < k0 + QB && k < NQ; ++k) {
        int ia, ib;
        if (!mirror_pair<N1>(p, threadIdx.x + k * row_nt<N1>(), ia, ib)) continue;
        conv_pair(buf, rslot<N1>(ia), rslot<N1>(ib), hA[k - k0], hB[k - k0]);
      }
    }
  }
  __syncthreads();
  row_fft<N1, 2, row_nt<N1>(), +1, LEAN>(buf, tt, ea);
  store_rows<N1, row_nt<N1>(), LEAN>(buf, Tout + (int64_t)j * ea.N, ra, rb, ea);
}

// backward: P1 = Gl conj(Hl) + i Gr conj(Hr)   (input gradient)
//           P2 = Gl conj(Xl) + i Gr conj(Xr)   (FIR gradient)
template <int N1>
__global__ __launch_bounds__(rowb_nt<N1>(), rows_bwd_min_waves<N1>()) void k_rows_bwd(const float2* __restrict__ Tin, float2* __restrict__ Tu,
                                                        float2* __restrict__ Th, const float2* __restrict__ ZH,
                                                        const float2* __restrict__ ZU, int z0,
                                                        const NodeDesc* __restrict__ desc, int want_u,
                                                        EngineArgs ea) {
  __shared__ float2 buf[4 * row_len<N1>()];
  __shared__ RowTw<N1> tt;
  tw_fill<row_tw<N1>()>(tt, ea.tw, ea.twdl);
  float2* b1 = buf;
  float2* b2 = buf + 2 * row_len<N1>();
  const int j = blockIdx.y;
  const int p = blockIdx.x;
  int ra, rb;
  row_pair(p, ea.N2, ra, rb);
  load_rows<N1, rowb_nt<N1>()>(b1, Tin + (int64_t)j * ea.N, ra, rb);
  __syncthreads();
  row_fft<N1, 2, rowb_nt<N1>(), -1>(b1, tt, ea);
  const int64_t zr = (int64_t)(z0 + desc[j].aux) * ea.N;
  const float2* H = ZH + zr;
  const float2* X = ZU + zr;
  constexpr int NQ = (N1 + 1 + rowb_nt<N1>() - 1) / rowb_nt<N1>();
  // pairs whose spectrum loads are in flight together (one within the
  // 64-register budget of the 2048-point rows)
  constexpr int QB = rows_bwd_min_waves<N1>() > 4 ? 1 : NQ;
#pragma unroll
  for (int k0 = 0; k0 < NQ; k0 += QB) {
  float2 hA[QB], hB[QB], xA[QB], xB[QB];
#pragma unroll
  for (int kq = 0; kq < QB; ++kq) {
    const int k = k0 + kq;
    int ia, ib;
    if (k >= NQ || !mirror_pair<N1>(p, threadIdx.x + k * rowb_nt<N1>(), ia, ib)) continue;
    const int64_t ga = (ia < N1) ? (int64_t)ra * N1 + ia : (int64_t)rb * N1 + (ia - N1);
    const int64_t gb = (ib < N1) ? (int64_t)ra * N1 + ib : (int64_t)rb * N1 + (ib - N1);
    hA[kq] = H[ga];
    hB[kq] = H[gb];
    xA[kq] = X[ga];
    xB[kq] = X[gb];
  }
#pragma unroll
  for (int kq = 0; kq < QB; ++kq) {
    const int k = k0 + kq;
    int ia, ib;
    if (k >= NQ || !mirror_pair<N1>(p, threadIdx.x + k * rowb_nt<N1>(), ia, ib)) continue;
    const int sa = rslot<N1>(ia), sb = rslot<N1>(ib);
    const float2 za = b1[sa], zb = b1[sb];
    const float2 ha = hA[kq], hb = hB[kq];
    const float2 xa = xA[kq], xb = xB[kq];
    float2 gl, gr, hl, hr, xl, xr;
    // bin k
    split_lr(za, zb, gl, gr);
    split_lr(ha, hb, hl, hr);
    split_lr(xa, xb, xl, xr);
    const float2 u_a = pack_lr(c_mulc(gl, hl), c_mulc(gr, hr));
    const float2 h_a = pack_lr(c_mulc(gl, xl), c_mulc(gr, xr));
    // bin -k
    split_lr(zb, za, gl, gr);
    split_lr(hb, ha, hl, hr);
    split_lr(xb, xa, xl, xr);
    const float2 u_b = pack_lr(c_mulc(gl, hl), c_mulc(gr, hr));
    const float2 h_b = pack_lr(c_mulc(gl, xl), c_mulc(gr, xr));
    b1[sa] = u_a;
    b1[sb] = u_b;
    b2[sa] = h_a;
    b2[sb] = h_b;
  }
  }
  __syncthreads();
  if (want_u) {
    // both products (b1, b2: four consecutive rows) in one batch of
    // transforms: half the barriers, twice the butterflies between them
    row_fft<N1, 4, rowb_nt<N1>(), +1>(buf, tt, ea);
    store_rows2<N1, rowb_nt<N1>()>(b1, b2, Tu + (int64_t)j * ea.N, Th + (int64_t)j * ea.N, ra, rb, ea);
  } else {
    row_fft<N1, 2, rowb_nt<N1>(), +1>(b2, tt, ea);
    store_rows<N1, rowb_nt<N1>()>(b2, Th + (int64_t)j * ea.N, ra, rb, ea);
  }
}

// ---------------------------------------------------------------- dispatch
template <typename LD>
void run_cols(const Ctx& c, const LD& ld, float2* T, int n, const EngineArgs& ea, double in_bytes) {
  const int N2 = ea.N2;
  const int TC = COL_TILE / N2;
  dim3 grid(ea.N1 / TC, n);
  ProfScope ps(c, "conv_cols", (double)n * (in_bytes + 8.0 * ea.N));
  switch (N2) {
#define MG_CASE(NN)                                                                                      \
  case NN:                                                                                               \
    MG_LAUNCH(c, (k_cols<NN, COL_TILE / NN, LD>), grid, dim3(col_nt<NN>()), 0, c.st, ld, T, ea); \
    break;
    MG_CASE(16) MG_CASE(32) MG_CASE(64) MG_CASE(128) MG_CASE(256) MG_CASE(512) MG_CASE(1024)
#undef MG_CASE
  }
}

template <typename ST>
void run_icols(const Ctx& c, const ST& st, const float2* T, int n, const EngineArgs& ea, double out_bytes) {
  const int N2 = ea.N2;
  const int TC = COL_TILE / N2;
  dim3 grid(ea.N1 / TC, n);
  ProfScope ps(c, "conv_icols", (double)n * (out_bytes + 8.0 * ea.N));
  switch (N2) {
#define MG_CASE(NN)                                                                                       \
  case NN:                                                                                                \
    MG_LAUNCH(c, (k_icols<NN, COL_TILE / NN, ST>), grid, dim3(col_nt<NN>()), 0, c.st, st, T, ea); \
    break;
    MG_CASE(16) MG_CASE(32) MG_CASE(64) MG_CASE(128) MG_CASE(256) MG_CASE(512) MG_CASE(1024)
#undef MG_CASE
  }
}

static EngineArgs engine_args(const Ctx& c) {
  const mg_graph* g = c.g;
  EngineArgs ea;
  ea.N = g->fft.N;
  ea.N1 = g->fft.N1;
  ea.N2 = g->fft.N2;
  ea.tw = wsp<float2>(c, g->ws.tw);
  ea.twdl = wsp<float2>(c, g->ws.twdl);
  ea.twhi = wsp<float2>(c, g->ws.twhi);
  ea.twlo = wsp<float2>(c, g->ws.twlo);
  return ea;
}

// row 0 of each long-FIR type in the spectrum arrays (delay, then reverb)
static int conv_base(const mg_graph* g, int type) {
  return type == MG_DELAY ? 0 : g->type_count[MG_DELAY];
}

// row 0 of each FIR type in the stored wet outputs (EQ, delay, reverb)
static int ybar_base(const mg_graph* g, int type) {
  if (type == MG_EQ) return 0;
  if (type == MG_DELAY) return g->type_count[MG_EQ];
  return g->type_count[MG_EQ] + g->type_count[MG_DELAY];
}

static NodeView node_view(const Ctx& c, int desc_off) {
  NodeView v;
  v.desc = c.desc + desc_off;
  v.dry = c.dry;
  v.U = c.U;
  v.G = c.G;
  v.L = c.L;
  v.C = c.C;
  return v;
}

template <int N1>
static void rows_spec_n(const Ctx& c, const float2* T, float2* Z, int z0, int desc_off, int n, const EngineArgs& ea) {
  ProfScope ps(c, "conv_rows", (double)n * 16.0 * ea.N);
  MG_LAUNCH(c, k_rows_spec<N1>, dim3(ea.N2 / 2, n), dim3(row_nt<N1>()), 0, c.st, T, Z, z0, c.desc + desc_off, ea);
}
template <int N1>
static void rows_conv_n(const Ctx& c, const float2* Tin, float2* Tout, const float2* ZH, float2* ZU, int z0,
                        int desc_off, int n, const EngineArgs& ea) {
  ProfScope ps(c, "conv_rows", (double)n * (ZU ? 32.0 : 24.0) * ea.N);
  MG_LAUNCH(c, k_rows_conv<N1>, dim3(ea.N2 / 2, n), dim3(row_nt<N1>()), 0, c.st, Tin, Tout, ZH, ZU, z0,
                     c.desc + desc_off, ea);
}
template <int N1>
static void rows_bwd_n(const Ctx& c, const float2* Tin, float2* Tu, float2* Th, const float2* ZH, const float2* ZU,
                       int z0, int desc_off, int n, int want_u, const EngineArgs& ea) {
  ProfScope ps(c, "conv_rows", (double)n * (want_u ? 40.0 : 32.0) * ea.N);
  MG_LAUNCH(c, k_rows_bwd<N1>, dim3(ea.N2 / 2, n), dim3(rowb_nt<N1>()), 0, c.st, Tin, Tu, Th, ZH, ZU, z0,
                     c.desc + desc_off, want_u, ea);
}

template <int N1>
static void rows_firspec_n(const Ctx& c, const LdFir& ld, float2* Z, int z0, int khi, int klo, int desc_off, int n,
                           const EngineArgs& ea) {
  ProfScope ps(c, "conv_rows", (double)n * 8.0 * ea.N);
  MG_LAUNCH(c, k_rows_firspec<N1>, dim3(ea.N2 / 2, n), dim3(row_nt<N1>()), 0, c.st, ld, Z, z0, khi, klo,
            c.desc + desc_off, ea);
}

#define MG_N1_SWITCH(FN, ...)                   \
  switch (ea.N1) {                              \
    case 512: FN<512>(__VA_ARGS__); break;      \
    case 1024: FN<1024>(__VA_ARGS__); break;    \
    case 2048: FN<2048>(__VA_ARGS__); break;    \
    case 3072: FN<3072>(__VA_ARGS__); break;    \
    case 4096: FN<4096>(__VA_ARGS__); break;    \
  }

// FIR spectra of the stage's nodes -> ZH (from the compact FIRs)
void conv_fir_spectrum(const Ctx& c, int type, int desc_off, int n, float2* T1) {
  const mg_graph* g = c.g;
  const mg_config& cf = g->cfg;
  EngineArgs ea = engine_args(c);
  float2* ZH = wsp<float2>(c, g->ws.ZH);
  const int z0 = conv_base(g, type);
  LdFir ld;
  ld.desc = c.desc + desc_off;
  ld.N = ea.N;
  double bytes;
  if (type == MG_EQ) {
    ld.h = wsp<float>(c, g->ws.eq_h);
    ld.Nh = cf.eq_taps;
    ld.lag0 = -(cf.eq_taps - 1) / 2;
    ld.stride = cf.eq_taps;
    ld.shared = 1;
    bytes = 4.0 * cf.eq_taps;
  } else if (type == MG_REVERB) {
    ld.h = wsp<float>(c, g->ws.rv_h);
    ld.Nh = cf.reverb_length;
    ld.lag0 = 0;
    ld.stride = 2 * (int64_t)cf.reverb_length;
    ld.shared = 0;
    bytes = 8.0 * cf.reverb_length;
  } else {
    // the compact delay FIR [2][dl_len] written by the synthesis
    ld.h = wsp<float>(c, g->ws.dl_h);
    ld.Nh = g->dl_len;
    ld.lag0 = -(cf.delay_fir_taps - 1) / 2;
    ld.stride = 2 * g->dl_len;
    ld.shared = 0;
    bytes = 8.0 * g->dl_len;
  }
  // rows of the index map that hold taps: lags from 0 up fill the first khi
  // rows, negative lags the last klo
  const int64_t hi = ld.lag0 + ld.Nh;  // one past the last lag
  const int khi = hi > 0 ? (int)((hi + ea.N1 - 1) / ea.N1) : 0;
  const int klo = ld.lag0 < 0 ? (int)((-ld.lag0 + ea.N1 - 1) / ea.N1) : 0;
  if (khi + klo <= FIRSPEC_MAXK && khi + klo <= ea.N2 / 2) {
    MG_N1_SWITCH(rows_firspec_n, c, ld, ZH, z0, khi, klo, desc_off, n, ea);
    return;
  }
  run_cols(c, ld, T1, n, ea, bytes);
  MG_N1_SWITCH(rows_spec_n, c, T1, ZH, z0, desc_off, n, ea);
}

void conv_forward(const Ctx& c, int type, int desc_off, int n, bool keep_input_spectrum) {
  const mg_graph* g = c.g;
  EngineArgs ea = engine_args(c);
  float2* T1 = wsp<float2>(c, g->ws.T1);
  float2* T2 = wsp<float2>(c, g->ws.T2);
  float2* ZH = wsp<float2>(c, g->ws.ZH);
  float2* ZU = keep_input_spectrum ? wsp<float2>(c, g->ws.ZU) : nullptr;
  const int z0 = conv_base(g, type);
  LdSignal ld;
  ld.v = node_view(c, desc_off);
  run_cols(c, ld, T1, n, ea, 8.0 * c.L);
  MG_N1_SWITCH(rows_conv_n, c, T1, T2, ZH, ZU, z0, desc_off, n, ea);
  StFwd st;
  st.v = node_view(c, desc_off);
  st.ybar_base = keep_input_spectrum ? wsp<float>(c, g->ws.YB) : nullptr;
  st.wet = c.wet;
  st.mask = c.mask;
  st.yb0 = ybar_base(g, type);
  st.part = c.part + (int64_t)desc_off * c.PB * PK;
  st.PB = c.PB;
  if (!keep_input_spectrum) {
    // forward-only: no ybar buffer; StFwd skips the ybar store
    st.ybar_base = nullptr;
  }
  run_icols(c, st, T2, n, ea, (keep_input_spectrum ? 24.0 : 16.0) * c.L);
  launch_reduce_lg(c, desc_off, n, ea.N1 / (COL_TILE / ea.N2));
}

// Backward of one stage, input-gradient part: column FFTs of dL/dybar, the
// row pass (both products), inverse columns of the input gradient.  The FIR
// gradient spectrum is left in T3 for conv_backward_fir.
void conv_backward(const Ctx& c, int type, int desc_off, int n, float2* T3) {
  const mg_graph* g = c.g;
  EngineArgs ea = engine_args(c);
  float2* T1 = wsp<float2>(c, g->ws.T1);
  float2* T2 = wsp<float2>(c, g->ws.T2);
  const float2* ZH = wsp<float2>(c, g->ws.ZH);
  const float2* ZU = wsp<float2>(c, g->ws.ZU);
  const int z0 = conv_base(g, type);
  LdGrad ld;
  ld.v = node_view(c, desc_off);
  ld.ybar_base = wsp<float>(c, g->ws.YB);
  ld.lg = c.lg + 2 * desc_off;
  ld.wet = c.wet;
  ld.mask = c.mask;
  ld.alpha_g = c.alpha_g;
  ld.yb0 = ybar_base(g, type);
  ld.part = c.part + (int64_t)desc_off * c.PB * PK;
  ld.PB = c.PB;
  run_cols(c, ld, T1, n, ea, 24.0 * c.L);
  int want_u = 0;
  for (int j = 0; j < n; ++j)
    if (g->desc[desc_off + j].gin >= 0) want_u = 1;
  MG_N1_SWITCH(rows_bwd_n, c, T1, T2, T3, ZH, ZU, z0, desc_off, n, want_u, ea);
  if (want_u) {
    StGradU su;
    su.v = node_view(c, desc_off);
    su.lg = c.lg + 2 * desc_off;
    su.wet = c.wet;
    su.mask = c.mask;
    su.alpha_g = c.alpha_g;
    run_icols(c, su, T2, n, ea, 24.0 * c.L);
  }
}

// Backward of one stage, FIR-gradient part: inverse columns of T3 at the
// FIR's lags only.
void conv_backward_fir(const Ctx& c, int type, int desc_off, int n, const float2* T3) {
  const mg_graph* g = c.g;
  const mg_config& cf = g->cfg;
  EngineArgs ea = engine_args(c);
  StGradH sh;
  sh.desc = c.desc + desc_off;
  sh.N = ea.N;
  if (type == MG_REVERB) {
    sh.dh = wsp<float>(c, g->ws.rv_dh);
    sh.Nh = cf.reverb_length;
    sh.lag0 = 0;
    sh.stride = 2 * (int64_t)cf.reverb_length;
    sh.shared = 0;
  } else {
    sh.dh = wsp<float>(c, g->ws.dl_dh);
    sh.Nh = g->dl_len;
    sh.lag0 = -(cf.delay_fir_taps - 1) / 2;
    sh.stride = 2 * g->dl_len;
    sh.shared = 0;
  }
  run_icols(c, sh, T3, n, ea, 8.0 * sh.Nh);
}

// tables for the LDS FFT (size MG_TWN) and for the big twiddles of N
void fft_init_tables(const Ctx& c, float2* tw, float2* twhi, float2* twlo, int N, hipStream_t st) {
  std::vector<float2> a(MG_TWN);
  const double pi = 3.14159265358979323846;
  for (int m = 0; m < MG_TWN; ++m) {
    double ang = -2.0 * pi * (double)m / MG_TWN;
    a[m] = make_float2((float)cos(ang), (float)sin(ang));
  }
  hipMemcpyAsync(tw, a.data(), a.size() * sizeof(float2), hipMemcpyHostToDevice, st);
  // W^m - 1 = (-2 sin^2(pi m / MG_TWN), -sin(2 pi m / MG_TWN)), without cancellation
  std::vector<float2> dl(MG_TWN);
  for (int m = 0; m < MG_TWN; ++m) {
    const double h = pi * (double)m / MG_TWN;
    dl[m] = make_float2((float)(-2.0 * sin(h) * sin(h)), (float)(-sin(2.0 * h)));
  }
  hipMemcpyAsync(wsp<float2>(c, c.g->ws.twdl), dl.data(), dl.size() * sizeof(float2), hipMemcpyHostToDevice, st);
  std::vector<double2> ad(MG_TWN);
  for (int m = 0; m < MG_TWN; ++m) {
    double ang = -2.0 * pi * (double)m / MG_TWN;
    ad[m] = make_double2(cos(ang), sin(ang));
  }
  hipMemcpyAsync(wsp<double2>(c, c.g->ws.twd), ad.data(), ad.size() * sizeof(double2), hipMemcpyHostToDevice, st);
  if (N > 0) {
    std::vector<float2> hi(N / 1024 > 0 ? N / 1024 : 1), lo(1024);
    for (size_t j = 0; j < hi.size(); ++j) {
      double ang = -2.0 * pi * (double)(1024 * (int64_t)j) / N;
      hi[j] = make_float2((float)cos(ang), (float)sin(ang));
    }
    for (int j = 0; j < 1024; ++j) {  // W_N^j - 1 without cancellation
      const double h = pi * (double)j / N;
      lo[j] = make_float2((float)(-2.0 * sin(h) * sin(h)), (float)(-sin(2.0 * h)));
    }
    hipMemcpyAsync(twhi, hi.data(), hi.size() * sizeof(float2), hipMemcpyHostToDevice, st);
    hipMemcpyAsync(twlo, lo.data(), lo.size() * sizeof(float2), hipMemcpyHostToDevice, st);
    hipStreamSynchronize(st);  // host vectors go out of scope
  } else {
    hipStreamSynchronize(st);
  }
}

}  // namespace mg
