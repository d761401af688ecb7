// Equalizer convolution by overlap-save in LDS (Sec. 3.3).
//
// The zero-phase FIR h (N taps, centred) is short next to the signal, so each
// workgroup owns V = P - (N - 1) consecutive output samples and transforms
// one P = 8192-point window of the packed stereo input (l + i r) entirely in
// LDS: HBM traffic is the input window (P / V x 8 bytes per stereo sample)
// plus the outputs.  The filter spectrum H_P = FFT_P(h placed circularly) is
// real (h is real and even) and is built once per node and step.
//   forward : y = IFFT(FFT(x) H_P) on the valid part; dry/wet; L_g energies
//   backward: dL/du = (1 - w) dL/dy + (dL/dybar correlated with h) - L_g term;
//             dL/dh[m] = Re sum_n Zg[n] conj(Zu[n - m]) per block (valid n
//             only), reduced over blocks in a fixed order; dry/wet partials.
#include "mg_device.h"
#include "mg_kernels.h"

namespace mg {

constexpr int EQ_P = 8192;
// 8 waves per block, two blocks per CU (one 66 KB window each), registers
// held to 128: the forward takes 106, the backward 128 with a 20-byte spill.
// With 1024 threads two blocks per CU left 64 registers and both kernels
// spilled; one 1024-thread block per CU took twice as long per step.
constexpr int EQ_NT = 512;   // forward and spectrum
constexpr int EQ_BNT = 512;  // backward: one window in LDS
// two windows per CU: waves per SIMD the register budget is sized for
constexpr int EQ_MIN_WAVES = 2 * EQ_NT / 256;
static_assert(EQ_NT == EQ_BNT, "one budget for both");
// window elements per thread whose global loads are issued together before
// any is used (a rolled loop over batches bounds the registers they hold)
constexpr int EQ_LB = 4;
static_assert(EQ_P % (EQ_NT * EQ_LB) == 0 && EQ_P % (EQ_BNT * EQ_LB) == 0, "whole batches");

struct EqArgs {
  const NodeDesc* desc;
  const float* dry;
  const float* U;
  float* G;
  float* Uo;            // node outputs (written)
  float* ybar;          // YB rows of EQ nodes (row = aux), or null
  const float* h;       // compact FIRs [row][N]
  float* HP;            // [row][P] real spectra
  float* dhp;           // [row][nblk][N] per-block FIR gradients
  float2* XU;           // [row][nblk][P] input-window spectra kept by the forward (or null)
  float* dh;            // [row][N]
  const float* wet;
  const float* mask;
  const double* lg;     // per stage node: E_ybar, E_u
  float* part;          // per stage node partial rows
  int PB;
  int64_t L;
  int C, N, V, nblk;
  float alpha_g;
  const float2* tw;
  const float2* twdl;
};

__device__ __forceinline__ const float* eq_input(const EqArgs& a, const NodeDesc& d, int64_t& cs) {
  if (d.in_kind == 0) {
    cs = (a.C == 1) ? 0 : a.L;
    return a.dry + (int64_t)d.in_slot * a.C * a.L;
  }
  cs = a.L;
  return a.U + (int64_t)d.in_slot * 2 * a.L;
}

// H_P of every node of the stage: grid (nodes)
__global__ __launch_bounds__(EQ_NT) void k_eq_spec(EqArgs a) {
  __shared__ float2 buf[EQ_P];
  __shared__ TwTab<EQ_P, float2> tt;
  tw_fill<EQ_P>(tt, a.tw, a.twdl);
  const NodeDesc d = a.desc[blockIdx.x];
  const float* h = a.h + (int64_t)d.aux * a.N;
  const int half = (a.N - 1) / 2;
  for (int i = threadIdx.x; i < EQ_P; i += EQ_NT) {
    // circular position i holds tap m = i (i <= half) or m = i - P (i >= P - half)
    float v = 0.f;
    if (i <= half) v = h[half + i];
    else if (i >= EQ_P - half) v = h[half + i - EQ_P];
    buf[i] = make_float2(v, 0.f);
  }
  __syncthreads();
  fft_lds<EQ_P, 1, EQ_P, EQ_NT, -1>(buf, tt);
  float* o = a.HP + (int64_t)d.aux * EQ_P;
  for (int i = threadIdx.x; i < EQ_P; i += EQ_NT) o[i] = buf[i].x;
}

// forward: grid (nblk, nodes)
__global__ __launch_bounds__(EQ_NT, EQ_MIN_WAVES) void k_eq_fwd(EqArgs a) {
  __shared__ float2 buf[EQ_P];
  __shared__ float red[EQ_NT / 64];
  __shared__ TwTab<EQ_P, float2> tt;
  tw_fill<EQ_P>(tt, a.tw, a.twdl);
  const int j = blockIdx.y, blk = blockIdx.x;
  const NodeDesc d = a.desc[j];
  int64_t cs;
  const float* u = eq_input(a, d, cs);
  const int half = (a.N - 1) / 2;
  const int64_t s0 = (int64_t)blk * a.V - half;   // window start
#pragma unroll 1
  for (int i0 = threadIdx.x; i0 < EQ_P; i0 += EQ_NT * EQ_LB) {
    float2 v[EQ_LB];
#pragma unroll
    for (int k = 0; k < EQ_LB; ++k) {
      const int64_t n = s0 + i0 + k * EQ_NT;
      v[k] = (n >= 0 && n < a.L) ? make_float2(u[n], u[cs + n]) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < EQ_LB; ++k) buf[i0 + k * EQ_NT] = v[k];
  }
  __syncthreads();
  fft_lds<EQ_P, 1, EQ_P, EQ_NT, -1>(buf, tt);
  const float* H = a.HP + (int64_t)d.aux * EQ_P;
  float2* xu = a.XU ? a.XU + ((int64_t)d.aux * a.nblk + blk) * EQ_P : nullptr;
#pragma unroll 1
  for (int i0 = threadIdx.x; i0 < EQ_P; i0 += EQ_NT * EQ_LB) {
    float hv[EQ_LB];
#pragma unroll
    for (int k = 0; k < EQ_LB; ++k) hv[k] = H[i0 + k * EQ_NT];
#pragma unroll
    for (int k = 0; k < EQ_LB; ++k) {
      const int i = i0 + k * EQ_NT;
      const float2 x = buf[i];
      if (xu) xu[i] = x;   // kept for the FIR gradient of the backward
      buf[i] = c_scale(x, hv[k] * (1.0f / EQ_P));
    }
  }
  __syncthreads();
  fft_lds<EQ_P, 1, EQ_P, EQ_NT, +1>(buf, tt);
  float w = node_w(a.wet, a.mask, d);
  float* y = a.Uo + (int64_t)d.out_slot * 2 * a.L;
  float* yb = a.ybar ? a.ybar + (int64_t)d.aux * 2 * a.L : nullptr;
  float ey = 0.f, eu = 0.f;
  for (int i = half + threadIdx.x; i < half + a.V; i += EQ_NT) {
    const int64_t n = s0 + i;
    if (n >= a.L) break;
    const float2 v = buf[i];
    const float l = u[n], r = u[cs + n];
    if (yb) {
      yb[n] = v.x;
      yb[a.L + n] = v.y;
    }
    y[n] = w * v.x + (1.0f - w) * l;
    y[a.L + n] = w * v.y + (1.0f - w) * r;
    const float m = v.x + v.y, um = l + r;
    ey += m * m;
    eu += um * um;
  }
  const float sa = block_sum<EQ_NT>(ey, red);
  const float sb = block_sum<EQ_NT>(eu, red);
  if (threadIdx.x == 0) {
    float* pr = a.part + ((int64_t)j * a.PB + blk) * PK;
    pr[0] = sa;
    pr[1] = sb;
  }
}

// backward: grid (nblk, nodes, 2); one P-point window in LDS.
//   input gradient: gbar over the whole window (packed l + i r) times H_P;
//   FIR gradient: gbar over the valid part only, times the conjugate of the
//   input-window spectrum the forward kept, inverse -> lags -half..half.
__global__ __launch_bounds__(EQ_BNT, EQ_MIN_WAVES) void k_eq_bwd(EqArgs a) {
  __shared__ float2 A[EQ_P];
  __shared__ float red[EQ_BNT / 64];
  __shared__ TwTab<EQ_P, float2> tt;
  tw_fill<EQ_P>(tt, a.tw, a.twdl);
  const int j = blockIdx.y, blk = blockIdx.x;
  const NodeDesc d = a.desc[j];
  int64_t cs;
  const float* u = eq_input(a, d, cs);
  const int half = (a.N - 1) / 2;
  const int64_t s0 = (int64_t)blk * a.V - half;
  const float* dy = a.G + (int64_t)d.gout * 2 * a.L;
  const float* yb = a.ybar + (int64_t)d.aux * 2 * a.L;
  float w = node_w(a.wet, a.mask, d);
  const double Ey = a.lg[2 * j] + 1e-12, Eu = a.lg[2 * j + 1] + 1e-12;
  const double diff = 0.5 * log(Ey) - 0.5 * log(Eu);
  const double sgn = diff > 0 ? 1.0 : (diff < 0 ? -1.0 : 0.0);
  const float ky = (float)((double)a.alpha_g * sgn / Ey), ku = (float)((double)a.alpha_g * sgn / Eu);
  // grid.z = 2 gives the two halves to separate workgroups (z = 0: dL/du;
  // z = 1: FIR gradient and dry/wet partial), each with the arithmetic it has
  // in one workgroup: twice the workgroups, half the transforms in a row
  const bool do_gin = gridDim.z == 1 || blockIdx.z == 0;
  const bool do_dh = gridDim.z == 1 || blockIdx.z == 1;
  float* gin = (do_gin && d.gin >= 0) ? a.G + (int64_t)d.gin * 2 * a.L : nullptr;
  if (gin) {
#pragma unroll 1
    for (int i0 = threadIdx.x; i0 < EQ_P; i0 += EQ_BNT * EQ_LB) {
      float4 r[EQ_LB];  // ybar (l, r), dL/dy (l, r)
#pragma unroll
      for (int k = 0; k < EQ_LB; ++k) {
        const int64_t n = s0 + i0 + k * EQ_BNT;
        r[k] = (n >= 0 && n < a.L) ? make_float4(yb[n], yb[a.L + n], dy[n], dy[a.L + n])
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int k = 0; k < EQ_LB; ++k) {
        const int64_t n = s0 + i0 + k * EQ_BNT;
        float2 g = make_float2(0.f, 0.f);
        if (n >= 0 && n < a.L) {
          const float rm = ky * (r[k].x + r[k].y);
          g = make_float2(w * r[k].z + rm, w * r[k].w + rm);
        }
        A[i0 + k * EQ_BNT] = g;
      }
    }
    __syncthreads();
    fft_lds<EQ_P, 1, EQ_P, EQ_BNT, -1>(A, tt);
    const float* H = a.HP + (int64_t)d.aux * EQ_P;
#pragma unroll 1
    for (int i0 = threadIdx.x; i0 < EQ_P; i0 += EQ_BNT * EQ_LB) {
      float hv[EQ_LB];
#pragma unroll
      for (int k = 0; k < EQ_LB; ++k) hv[k] = H[i0 + k * EQ_BNT];
#pragma unroll
      for (int k = 0; k < EQ_LB; ++k) A[i0 + k * EQ_BNT] = c_scale(A[i0 + k * EQ_BNT], hv[k] * (1.0f / EQ_P));
    }
    __syncthreads();
    fft_lds<EQ_P, 1, EQ_P, EQ_BNT, +1>(A, tt);
    for (int i = half + threadIdx.x; i < half + a.V; i += EQ_BNT) {
      const int64_t n = s0 + i;
      if (n >= a.L) break;
      const float um = u[n] + u[cs + n];
      gin[n] = (1.0f - w) * dy[n] + A[i].x - ku * um;
      gin[a.L + n] = (1.0f - w) * dy[a.L + n] + A[i].y - ku * um;
    }
    __syncthreads();
  }
  if (!do_dh) return;
  // FIR gradient: the valid-part gradient correlated with the input window
  float dw = 0.f;
#pragma unroll 1
  for (int i0 = threadIdx.x; i0 < EQ_P; i0 += EQ_BNT * EQ_LB) {
    float4 r[EQ_LB];   // ybar (l, r), dL/dy (l, r)
    float2 uv[EQ_LB];  // u (l, r)
#pragma unroll
    for (int k = 0; k < EQ_LB; ++k) {
      const int i = i0 + k * EQ_BNT;
      const int64_t n = s0 + i;
      const bool ok = i >= half && i < half + a.V && n < a.L;
      r[k] = ok ? make_float4(yb[n], yb[a.L + n], dy[n], dy[a.L + n]) : make_float4(0.f, 0.f, 0.f, 0.f);
      uv[k] = ok ? make_float2(u[n], u[cs + n]) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < EQ_LB; ++k) {
      const int i = i0 + k * EQ_BNT;
      const int64_t n = s0 + i;
      float2 g = make_float2(0.f, 0.f);
      if (i >= half && i < half + a.V && n < a.L) {
        const float bl = r[k].x, br = r[k].y;
        const float rm = ky * (bl + br);
        const float gl = r[k].z, gr = r[k].w;
        g = make_float2(w * gl + rm, w * gr + rm);
        dw += gl * (bl - uv[k].x) + gr * (br - uv[k].y);
      }
      A[i] = g;
    }
  }
  __syncthreads();
  fft_lds<EQ_P, 1, EQ_P, EQ_BNT, -1>(A, tt);
  const float2* xu = a.XU + ((int64_t)d.aux * a.nblk + blk) * EQ_P;
#pragma unroll 1
  for (int i0 = threadIdx.x; i0 < EQ_P; i0 += EQ_BNT * EQ_LB) {
    float2 xv[EQ_LB];
#pragma unroll
    for (int k = 0; k < EQ_LB; ++k) xv[k] = xu[i0 + k * EQ_BNT];
#pragma unroll
    for (int k = 0; k < EQ_LB; ++k) A[i0 + k * EQ_BNT] = c_scale(c_mulc(A[i0 + k * EQ_BNT], xv[k]), 1.0f / EQ_P);
  }
  __syncthreads();
  fft_lds<EQ_P, 1, EQ_P, EQ_BNT, +1>(A, tt);
  // lag m sits at circular index m mod P; dh index = m + half
  float* o = a.dhp + ((int64_t)d.aux * a.nblk + blk) * a.N;
  for (int t = threadIdx.x; t < a.N; t += EQ_BNT) {
    const int m = t - half;
    o[t] = A[m >= 0 ? m : m + EQ_P].x;
  }
  const float s = block_sum<EQ_BNT>(dw, red);
  if (threadIdx.x == 0) a.part[((int64_t)j * a.PB + blk) * PK + 2] = s;
}

// dh[row][t] = sum over blocks (fixed order, FP64): each tap's blocks are
// split into DH_SPLIT runs added by separate lanes, then the runs in order.
// grid (ceil(N / DH_TAPS), nodes), DH_TAPS x DH_SPLIT threads
constexpr int DH_SPLIT = 8;
constexpr int DH_TAPS = MG_BLOCK / DH_SPLIT;

__global__ __launch_bounds__(MG_BLOCK) void k_eq_dh_reduce(EqArgs a) {
  __shared__ double part[DH_SPLIT][DH_TAPS];
  const NodeDesc d = a.desc[blockIdx.y];
  const int lane = threadIdx.x % DH_TAPS, r = threadIdx.x / DH_TAPS;
  const int t = blockIdx.x * DH_TAPS + lane;
  const int Q = (a.nblk + DH_SPLIT - 1) / DH_SPLIT;
  const int b0 = r * Q, b1 = min(a.nblk, b0 + Q);
  double s = 0.0;
  if (t < a.N) {
    const float* src = a.dhp + (int64_t)d.aux * a.nblk * a.N + t;
    for (int b = b0; b < b1; ++b) s += (double)src[(int64_t)b * a.N];
  }
  part[r][lane] = s;
  __syncthreads();
  if (r != 0 || t >= a.N) return;
  double tot = 0.0;
  for (int q = 0; q < DH_SPLIT; ++q) tot += part[q][lane];
  a.dh[(int64_t)d.aux * a.N + t] = (float)tot;
}

static EqArgs eq_args(const Ctx& c, int desc_off, bool keep) {
  const mg_graph* g = c.g;
  EqArgs a;
  a.desc = c.desc + desc_off;
  a.dry = c.dry;
  a.U = c.U;
  a.G = c.G;
  a.Uo = c.U;
  a.ybar = keep ? wsp<float>(c, g->ws.YB) : nullptr;  // EQ rows come first in YB
  a.h = wsp<float>(c, g->ws.eq_h);
  a.HP = wsp<float>(c, g->ws.eq_HP);
  a.dhp = g->mode ? wsp<float>(c, g->ws.eq_dhp) : nullptr;
  a.XU = (g->mode && keep) ? wsp<float2>(c, g->ws.eq_XU) : nullptr;
  a.dh = g->mode ? wsp<float>(c, g->ws.eq_dh) : nullptr;
  a.wet = c.wet;
  a.mask = c.mask;
  a.lg = c.lg + 2 * desc_off;
  a.part = c.part + (int64_t)desc_off * c.PB * PK;
  a.PB = c.PB;
  a.L = c.L;
  a.C = c.C;
  a.N = g->cfg.eq_taps;
  a.V = EQ_P - (a.N - 1);
  a.nblk = (int)((c.L + a.V - 1) / a.V);
  a.alpha_g = c.alpha_g;
  a.tw = wsp<float2>(c, g->ws.tw);
  a.twdl = wsp<float2>(c, g->ws.twdl);
  return a;
}

int eq_blocks(const mg_graph* g) {
  const int V = EQ_P - (g->cfg.eq_taps - 1);
  return (int)((g->cfg.length + V - 1) / V);
}

void eq_spectrum(const Ctx& c, int desc_off, int n) {
  EqArgs a = eq_args(c, desc_off, false);
  ProfScope ps(c, "eq_spec", (double)n * (4.0 * a.N + 4.0 * EQ_P));
  MG_LAUNCH(c, k_eq_spec, dim3(n), dim3(EQ_NT), 0, c.st, a);
}

void eq_forward(const Ctx& c, int desc_off, int n, bool keep) {
  EqArgs a = eq_args(c, desc_off, keep);
  {
    // reads the input windows (and u for the mix), writes y (and ybar and the
    // kept window spectra when keeping)
    ProfScope ps(c, "eq_conv",
                 (double)n * ((keep ? 16.0 : 8.0) * EQ_P * a.nblk + (keep ? 16.0 : 8.0) * c.L + 8.0 * c.L));
    MG_LAUNCH(c, k_eq_fwd, dim3(a.nblk, n), dim3(EQ_NT), 0, c.st, a);
  }
  launch_reduce_lg(c, desc_off, n, a.nblk);
}

void eq_backward(const Ctx& c, int desc_off, int n) {
  EqArgs a = eq_args(c, desc_off, true);
  {
    // reads dL/dy, ybar, u (window each), u again and the kept window spectra;
    // writes dL/du and the block FIR gradients
    ProfScope ps(c, "eq_conv", (double)n * ((32.0 * EQ_P) * a.nblk + 16.0 * c.L + 4.0 * a.N * a.nblk));
    MG_LAUNCH(c, k_eq_bwd, dim3(a.nblk, n, 2), dim3(EQ_BNT), 0, c.st, a);
  }
}

void eq_backward_fir(const Ctx& c, int desc_off, int n) {
  EqArgs a = eq_args(c, desc_off, true);
  MG_LAUNCH(c, k_eq_dh_reduce, dim3((a.N + DH_TAPS - 1) / DH_TAPS, n), dim3(MG_BLOCK), 0, c.st, a);
}

}  // namespace mg
