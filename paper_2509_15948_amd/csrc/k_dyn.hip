// Compressor and noisegate (Sec. 3.5, Sec. 3.6).
//   e[n] = (u_l + u_r)^2;  g[n] = a g[n-1] + (1 - a) e[n];  G = log(g + eps)
//   ybar_c = exp(f(G) - G) u_c  with the quadratic-knee curve f.
// One coefficient (a linear recursion): a chunked scan.  Each 4096-sample
// chunk is summarised (state reached from zero); the second pass chains the
// chunk carries in FP64 (one lane per workgroup, over the chunks before its
// own) and rescans its chunk from that carry with a workgroup-level scan of
// per-thread 16-sample segments.
// Attack/release (a[n] depends on e[n] > g[n-1], not linear): one lane per
// node walks the samples in order; the other lanes of its wave stage inputs
// and outputs through LDS.
// Adjoints: lambda[n] = dL/dg[n] + a[n+1] lambda[n+1] run backwards the same
// ways (the attack/release pattern is recovered from the stored envelope).
#include "mg_device.h"
#include "mg_kernels.h"

namespace mg {

constexpr int DYN_SPT = 16;
constexpr int DYN_CH = MG_BLOCK * DYN_SPT;  // 4096 samples per chunk
constexpr int DYN_PAD = MG_BLOCK + 1;
constexpr float COMP_EPS = 1e-8f;

struct DynParams {
  float a, b, loga;       // a, 1 - a, log a   (single coefficient)
  float aa, ba, ar, br;   // attack / release coefficients
  float T, W, R;
  float dW, dR;           // dW/dtheta_W = W, dR/dtheta_R = R - 1
};

__device__ __forceinline__ float softplusf_(float x) { return x > 20.f ? x : log1pf(expf(x)); }

__device__ __forceinline__ DynParams dyn_params(const float* p, int ar_mode) {
  DynParams q;
  int o = 0;
  if (ar_mode) {
    q.aa = 1.0f / (1.0f + expf(-p[0]));
    q.ba = 1.0f / (1.0f + expf(p[0]));
    q.ar = 1.0f / (1.0f + expf(-p[1]));
    q.br = 1.0f / (1.0f + expf(p[1]));
    q.a = q.b = q.loga = 0.f;
    o = 2;
  } else {
    q.a = 1.0f / (1.0f + expf(-p[0]));
    q.b = 1.0f / (1.0f + expf(p[0]));
    q.loga = -softplusf_(-p[0]);
    q.aa = q.ba = q.ar = q.br = 0.f;
    o = 1;
  }
  q.T = p[o];
  q.W = expf(p[o + 1]);
  q.R = 1.0f + expf(p[o + 2]);
  q.dW = q.W;
  q.dR = q.R - 1.0f;
  return q;
}

// curve f(G) and its partials; GATE selects Sec. 3.6
template <int GATE>
__device__ __forceinline__ float curve(float G, const DynParams& q, float& dG, float& dT, float& dWv, float& dRv) {
  const float T = q.T, W = q.W, R = q.R;
  if (!GATE) {
    if (G >= T + W) {
      dG = 1.0f / R;
      dT = 1.0f - 1.0f / R;
      dWv = 0.f;
      dRv = -(G - T) / (R * R);
      return T + (G - T) / R;
    }
    if (G >= T - W) {
      const float x = G - T + W, k = 1.0f / R - 1.0f;
      dG = 1.0f + k * x / (2.0f * W);
      dT = -k * x / (2.0f * W);
      dWv = k * (x / (2.0f * W) - x * x / (4.0f * W * W));
      dRv = -x * x / (4.0f * W * R * R);
      return G + k * x * x / (4.0f * W);
    }
    dG = 1.f;
    dT = dWv = dRv = 0.f;
    return G;
  } else {
    if (G >= T + W) {
      dG = 1.f;
      dT = dWv = dRv = 0.f;
      return G;
    }
    if (G >= T - W) {
      const float x = G - T - W, k = 1.0f - R;
      dG = 1.0f + k * x / (2.0f * W);
      dT = -k * x / (2.0f * W);
      dWv = k * (-x / (2.0f * W) - x * x / (4.0f * W * W));
      dRv = -x * x / (4.0f * W);
      return G + k * x * x / (4.0f * W);
    }
    dG = R;
    dT = 1.0f - R;
    dWv = 0.f;
    dRv = G - T;
    return T + R * (G - T);
  }
}

struct DynView {
  const NodeDesc* desc;
  const float* dry;
  float* U;
  float* G;
  float* env;         // [row][L]
  const float* theta;
  const float* wet;
  const float* mask;
  int64_t L;
  int C;
  int env0;           // env row of type row 0
  float* part;
  int PB;
};

__device__ __forceinline__ const float* dyn_input(const DynView& v, const NodeDesc& d, int64_t& cs) {
  if (d.in_kind == 0) {
    cs = (v.C == 1) ? 0 : v.L;
    return v.dry + (int64_t)d.in_slot * v.C * v.L;
  }
  cs = v.L;
  return v.U + (int64_t)d.in_slot * 2 * v.L;
}

// The loops over a chunk's samples (DYN_SPT per thread, MG_BLOCK apart)
// fetch a batch of samples' operands from global memory before the first is
// used; the arithmetic and its order are those of one sample after another.
// Two-operand loops take 8 samples per batch, the wider ones 4, so the
// registers stay near 64 (eight workgroups per CU; the backward apply takes
// 65, seven workgroups, as held to 64 it spilled).
constexpr int DYN_B2 = 8;
constexpr int DYN_B6 = 4;
static_assert(DYN_SPT % DYN_B2 == 0 && DYN_SPT % DYN_B6 == 0, "whole batches");

// Stage the chunk's energy into LDS (padded transpose: sample s of thread t
// at i * DYN_PAD + t) so each thread walks 16 consecutive samples.
__device__ __forceinline__ void stage_energy(float* le, const float* u, int64_t cs, int64_t s0, int64_t L) {
#pragma unroll 1
  for (int k0 = 0; k0 < DYN_SPT; k0 += DYN_B2) {
    float ul[DYN_B2], ur[DYN_B2];
#pragma unroll
    for (int k = 0; k < DYN_B2; ++k) {
      const int64_t n = s0 + threadIdx.x + (k0 + k) * MG_BLOCK;
      ul[k] = n < L ? u[n] : 0.f;
      ur[k] = n < L ? u[cs + n] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < DYN_B2; ++k) {
      const int idx = threadIdx.x + (k0 + k) * MG_BLOCK;
      float e = 0.f;
      if (s0 + idx < L) {
        const float m = ul[k] + ur[k];
        e = m * m;
      }
      le[(idx % DYN_SPT) * DYN_PAD + idx / DYN_SPT] = e;
    }
  }
}

// -------------------------------------------------------------- single-coefficient forward
// pass 1: per chunk, the state reached from zero
__global__ __launch_bounds__(MG_BLOCK) void k_dyn_sum(DynView v, float* __restrict__ sums, int nchunks) {
  __shared__ float le[DYN_SPT * DYN_PAD];
  __shared__ float red[MG_BLOCK];
  const NodeDesc d = v.desc[blockIdx.y];
  const DynParams q = dyn_params(v.theta + d.theta_off, 0);
  int64_t cs;
  const float* u = dyn_input(v, d, cs);
  const int64_t s0 = (int64_t)blockIdx.x * DYN_CH;
  stage_energy(le, u, cs, s0, v.L);
  __syncthreads();
  const int t = threadIdx.x;
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < DYN_SPT; ++i) s = fmaf(q.a, s, q.b * le[i * DYN_PAD + t]);
  red[t] = s;
  __syncthreads();
  // tree: combine(left, right) = left * a^{len(right)} + right
  for (int st = 1; st < MG_BLOCK; st <<= 1) {
    if ((t % (2 * st)) == 0) red[t] = red[t] * expf(q.loga * (float)(DYN_SPT * st)) + red[t + st];
    __syncthreads();
  }
  if (t == 0) sums[(int64_t)blockIdx.y * nchunks + blockIdx.x] = red[0];
}

// The FP64 carry entering this workgroup's chunk (node blockIdx.y, chunk
// blockIdx.x), chained by one lane over the chunk states in order: forward
// over the chunks before it, reverse over the chunks after it.  Every
// workgroup of a node runs the same chain, so all of them see the carries a
// separate chaining pass would produce, without its launch.  slot: one
// double of LDS.
__device__ __forceinline__ float chunk_carry(const DynView& v, const NodeDesc& d, const float* __restrict__ sums,
                                             int nchunks, bool reverse, double* slot) {
  if (threadIdx.x == 0) {
    const float* p = v.theta + d.theta_off;
    const double loga = -log1p(exp(-(double)p[0]));
    const double aC = exp(loga * DYN_CH);
    const float* sr = sums + (int64_t)blockIdx.y * nchunks;
    const int k0 = (int)blockIdx.x;
    double c = 0.0;
    if (!reverse) {
#pragma unroll 4
      for (int k = 0; k < k0; ++k) c = aC * c + (double)sr[k];
    } else {
#pragma unroll 4
      for (int k = nchunks - 1; k > k0; --k) c = (double)sr[k] + aC * c;
    }
    *slot = c;
  }
  __syncthreads();
  return (float)*slot;
}

// exclusive scan across threads of per-thread segment states (uniform decay
// a^DYN_SPT per segment) and the incoming chunk state
__device__ __forceinline__ float seg_entry(float seg, float carry_in, float loga, float* red) {
  const int t = threadIdx.x;
  red[t] = seg;
  __syncthreads();
  for (int st = 1; st < MG_BLOCK; st <<= 1) {
    const float other = (t >= st) ? red[t - st] : 0.f;
    __syncthreads();
    if (t >= st) red[t] = fmaf(other, expf(loga * (float)(DYN_SPT * st)), red[t]);
    __syncthreads();
  }
  const float excl = (t > 0) ? red[t - 1] : 0.f;
  __syncthreads();
  return fmaf(carry_in, expf(loga * (float)(DYN_SPT * t)), excl);
}

template <int GATE>
__global__ __launch_bounds__(MG_BLOCK) void k_dyn_apply(DynView v, const float* __restrict__ sums, int nchunks) {
  __shared__ float le[DYN_SPT * DYN_PAD];
  __shared__ float red[MG_BLOCK];
  __shared__ double cslot;
  const NodeDesc d = v.desc[blockIdx.y];
  const DynParams q = dyn_params(v.theta + d.theta_off, 0);
  int64_t cs;
  const float* u = dyn_input(v, d, cs);
  const int64_t s0 = (int64_t)blockIdx.x * DYN_CH;
  stage_energy(le, u, cs, s0, v.L);
  __syncthreads();
  const int t = threadIdx.x;
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < DYN_SPT; ++i) s = fmaf(q.a, s, q.b * le[i * DYN_PAD + t]);
  const float cin = chunk_carry(v, d, sums, nchunks, false, &cslot);
  float gst = seg_entry(s, cin, q.loga, red);
  // envelope into LDS (reuse le in place: each thread owns its column)
#pragma unroll
  for (int i = 0; i < DYN_SPT; ++i) {
    gst = fmaf(q.a, gst, q.b * le[i * DYN_PAD + t]);
    le[i * DYN_PAD + t] = gst;
  }
  __syncthreads();
  float w = node_w(v.wet, v.mask, d);
  float* y = v.U + (int64_t)d.out_slot * 2 * v.L;
  float* env = v.env ? v.env + (int64_t)(v.env0 + d.aux) * v.L : nullptr;
#pragma unroll 1
  for (int k0 = 0; k0 < DYN_SPT; k0 += DYN_B2) {
    float ul[DYN_B2], ur[DYN_B2];
#pragma unroll
    for (int k = 0; k < DYN_B2; ++k) {
      const int64_t n = s0 + threadIdx.x + (k0 + k) * MG_BLOCK;
      ul[k] = n < v.L ? u[n] : 0.f;
      ur[k] = n < v.L ? u[cs + n] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < DYN_B2; ++k) {
      const int idx = threadIdx.x + (k0 + k) * MG_BLOCK;
      const int64_t n = s0 + idx;
      if (n >= v.L) break;
      const float g = le[(idx % DYN_SPT) * DYN_PAD + idx / DYN_SPT];
      const float G = logf(g + COMP_EPS);
      float a0, a1, a2, a3;
      const float f = curve<GATE>(G, q, a0, a1, a2, a3);
      const float gain = expf(f - G);
      const float l = ul[k], r = ur[k];
      y[n] = w * gain * l + (1.0f - w) * l;
      y[v.L + n] = w * gain * r + (1.0f - w) * r;
      if (env) env[n] = g;
    }
  }
}

// -------------------------------------------------------------- single-coefficient backward
// dL/dg[n] from dL/dy, u and the stored envelope (also the parameter partials
// of the curve and the dry/wet partial when acc is set)
template <int GATE>
__device__ __forceinline__ float dyn_dg(const DynParams& q, float w, float g, float l, float r, float dl, float dr,
                                        float* acc) {
  const float G = logf(g + COMP_EPS);
  float fG, fT, fW, fR;
  const float f = curve<GATE>(G, q, fG, fT, fW, fR);
  const float gain = expf(f - G);
  const float da = w * (dl * l + dr * r);  // dL/dgain
  if (acc) {
    acc[0] += dl * (gain * l - l) + dr * (gain * r - r);  // dry/wet
    acc[1] += da * gain * fT;
    acc[2] += da * gain * fW * q.dW;
    acc[3] += da * gain * fR * q.dR;
  }
  return da * gain * (fG - 1.0f) / (g + COMP_EPS);
}

struct DynBwdView {
  DynView v;
  const float* dyb;  // unused placeholder
};

// dL/dg of the chunk's samples into LDS (layout of stage_energy); acc as in dyn_dg
template <int GATE>
__device__ __forceinline__ void stage_dg(float* lg, const DynParams& q, float w, const float* env, const float* u,
                                         int64_t cs, const float* dy, int64_t L, int64_t s0, float* acc) {
#pragma unroll 1
  for (int k0 = 0; k0 < DYN_SPT; k0 += DYN_B6) {
    float ge[DYN_B6], ul[DYN_B6], ur[DYN_B6], dl[DYN_B6], dr[DYN_B6];
#pragma unroll
    for (int k = 0; k < DYN_B6; ++k) {
      const int64_t n = s0 + threadIdx.x + (k0 + k) * MG_BLOCK;
      const bool ok = n < L;
      ge[k] = ok ? env[n] : 0.f;
      ul[k] = ok ? u[n] : 0.f;
      ur[k] = ok ? u[cs + n] : 0.f;
      dl[k] = ok ? dy[n] : 0.f;
      dr[k] = ok ? dy[L + n] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < DYN_B6; ++k) {
      const int idx = threadIdx.x + (k0 + k) * MG_BLOCK;
      float dg = 0.f;
      if (s0 + idx < L) dg = dyn_dg<GATE>(q, w, ge[k], ul[k], ur[k], dl[k], dr[k], acc);
      lg[(idx % DYN_SPT) * DYN_PAD + idx / DYN_SPT] = dg;
    }
  }
}

// pass 1 (reverse): per chunk, lambda at the chunk's first sample from zero
template <int GATE>
__global__ __launch_bounds__(MG_BLOCK) void k_dyn_bsum(DynView v, float* __restrict__ sums, int nchunks) {
  __shared__ float lg[DYN_SPT * DYN_PAD];
  __shared__ float red[MG_BLOCK];
  const NodeDesc d = v.desc[blockIdx.y];
  const DynParams q = dyn_params(v.theta + d.theta_off, 0);
  float w = node_w(v.wet, v.mask, d);
  int64_t cs;
  const float* u = dyn_input(v, d, cs);
  const float* dy = v.G + (int64_t)d.gout * 2 * v.L;
  const float* env = v.env + (int64_t)(v.env0 + d.aux) * v.L;
  const int64_t s0 = (int64_t)blockIdx.x * DYN_CH;
  stage_dg<GATE>(lg, q, w, env, u, cs, dy, v.L, s0, nullptr);
  __syncthreads();
  const int t = threadIdx.x;
  float s = 0.f;
#pragma unroll
  for (int i = DYN_SPT - 1; i >= 0; --i) s = fmaf(q.a, s, lg[i * DYN_PAD + t]);
  red[t] = s;
  __syncthreads();
  // combine(left, right) = left + a^{len(left)} right
  for (int st = 1; st < MG_BLOCK; st <<= 1) {
    if ((t % (2 * st)) == 0) red[t] = red[t] + expf(q.loga * (float)(DYN_SPT * st)) * red[t + st];
    __syncthreads();
  }
  if (t == 0) sums[(int64_t)blockIdx.y * nchunks + blockIdx.x] = red[0];
}

template <int GATE>
__global__ __launch_bounds__(MG_BLOCK) void k_dyn_bapply(DynView v, const float* __restrict__ sums, int nchunks) {
  __shared__ float lg[DYN_SPT * DYN_PAD];
  __shared__ float red[MG_BLOCK];
  __shared__ double cslot;
  const NodeDesc d = v.desc[blockIdx.y];
  const DynParams q = dyn_params(v.theta + d.theta_off, 0);
  float w = node_w(v.wet, v.mask, d);
  int64_t cs;
  const float* u = dyn_input(v, d, cs);
  const float* dy = v.G + (int64_t)d.gout * 2 * v.L;
  const float* env = v.env + (int64_t)(v.env0 + d.aux) * v.L;
  float* gin = d.gin >= 0 ? v.G + (int64_t)d.gin * 2 * v.L : nullptr;
  const int64_t s0 = (int64_t)blockIdx.x * DYN_CH;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  stage_dg<GATE>(lg, q, w, env, u, cs, dy, v.L, s0, acc);
  __syncthreads();
  const int t = threadIdx.x;
  float s = 0.f;
#pragma unroll
  for (int i = DYN_SPT - 1; i >= 0; --i) s = fmaf(q.a, s, lg[i * DYN_PAD + t]);
  // reverse exclusive scan: state entering thread t's segment from the right
  red[t] = s;
  __syncthreads();
  for (int st = 1; st < MG_BLOCK; st <<= 1) {
    const float other = (t + st < MG_BLOCK) ? red[t + st] : 0.f;
    __syncthreads();
    if (t + st < MG_BLOCK) red[t] = fmaf(other, expf(q.loga * (float)(DYN_SPT * st)), red[t]);
    __syncthreads();
  }
  const float excl = (t + 1 < MG_BLOCK) ? red[t + 1] : 0.f;
  __syncthreads();
  const float cin = chunk_carry(v, d, sums, nchunks, true, &cslot);
  float lam = fmaf(cin, expf(q.loga * (float)(DYN_SPT * (MG_BLOCK - 1 - t))), excl);
#pragma unroll
  for (int i = DYN_SPT - 1; i >= 0; --i) {
    lam = fmaf(q.a, lam, lg[i * DYN_PAD + t]);
    lg[i * DYN_PAD + t] = lam;
  }
  __syncthreads();
  float dth = 0.f;
#pragma unroll 1
  for (int k0 = 0; k0 < DYN_SPT; k0 += DYN_B6) {
    float ul[DYN_B6], ur[DYN_B6], gp[DYN_B6], ge[DYN_B6], dl[DYN_B6], dr[DYN_B6];
#pragma unroll
    for (int k = 0; k < DYN_B6; ++k) {
      const int64_t n = s0 + threadIdx.x + (k0 + k) * MG_BLOCK;
      const bool ok = n < v.L;
      ul[k] = ok ? u[n] : 0.f;
      ur[k] = ok ? u[cs + n] : 0.f;
      gp[k] = (ok && n > 0) ? env[n - 1] : 0.f;
      ge[k] = (ok && gin) ? env[n] : 0.f;
      dl[k] = (ok && gin) ? dy[n] : 0.f;
      dr[k] = (ok && gin) ? dy[v.L + n] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < DYN_B6; ++k) {
      const int idx = threadIdx.x + (k0 + k) * MG_BLOCK;
      const int64_t n = s0 + idx;
      if (n >= v.L) break;
      const float lm = lg[(idx % DYN_SPT) * DYN_PAD + idx / DYN_SPT];
      const float l = ul[k], r = ur[k];
      const float um = l + r;
      const float e = um * um;
      const float gprev = gp[k];
      dth += lm * (gprev - e);
      if (gin) {
        const float g = ge[k];
        const float G = logf(g + COMP_EPS);
        float a0, a1, a2, a3;
        const float gain = expf(curve<GATE>(G, q, a0, a1, a2, a3) - G);
        const float de2 = q.b * lm * 2.0f * um;
        gin[n] = (1.0f - w) * dl[k] + w * gain * dl[k] + de2;
        gin[v.L + n] = (1.0f - w) * dr[k] + w * gain * dr[k] + de2;
      }
    }
  }
  float* pr = v.part + ((int64_t)blockIdx.y * v.PB + blockIdx.x) * PK;
  const float s_dw = block_sum<MG_BLOCK>(acc[0], red);
  const float s_th = block_sum<MG_BLOCK>(dth * q.a * q.b, red);
  const float s_T = block_sum<MG_BLOCK>(acc[1], red);
  const float s_W = block_sum<MG_BLOCK>(acc[2], red);
  const float s_R = block_sum<MG_BLOCK>(acc[3], red);
  if (threadIdx.x == 0) {
    pr[2] = s_dw;
    pr[3] = s_th;
    pr[4] = s_T;
    pr[5] = s_W;
    pr[6] = s_R;
  }
}

// -------------------------------------------------------------- attack/release
constexpr int AR_CH = 1024;

// one wave per node; lane 0 runs the recursion over each staged chunk
template <int GATE>
__global__ __launch_bounds__(64) void k_dyn_ar_fwd(DynView v) {
  __shared__ float le[AR_CH];
  const NodeDesc d = v.desc[blockIdx.x];
  const DynParams q = dyn_params(v.theta + d.theta_off, 1);
  float w = node_w(v.wet, v.mask, d);
  int64_t cs;
  const float* u = dyn_input(v, d, cs);
  float* y = v.U + (int64_t)d.out_slot * 2 * v.L;
  float* env = v.env ? v.env + (int64_t)(v.env0 + d.aux) * v.L : nullptr;
  float gprev = 0.f;
  for (int64_t s0 = 0; s0 < v.L; s0 += AR_CH) {
    const int len = (int)((v.L - s0) < AR_CH ? (v.L - s0) : AR_CH);
    for (int i = threadIdx.x; i < len; i += 64) {
      const float m = u[s0 + i] + u[cs + s0 + i];
      le[i] = m * m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      float g = gprev;
      for (int i = 0; i < len; ++i) {
        const float e = le[i];
        g = (e > g) ? fmaf(q.aa, g, q.ba * e) : fmaf(q.ar, g, q.br * e);
        le[i] = g;
      }
      gprev = g;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < len; i += 64) {
      const int64_t n = s0 + i;
      const float g = le[i];
      const float G = logf(g + COMP_EPS);
      float a0, a1, a2, a3;
      const float gain = expf(curve<GATE>(G, q, a0, a1, a2, a3) - G);
      const float l = u[n], r = u[cs + n];
      y[n] = w * gain * l + (1.0f - w) * l;
      y[v.L + n] = w * gain * r + (1.0f - w) * r;
      if (env) env[n] = g;
    }
    __syncthreads();
    gprev = __shfl(gprev, 0);
  }
}

template <int GATE>
__global__ __launch_bounds__(64) void k_dyn_ar_bwd(DynView v) {
  __shared__ float lg[AR_CH];
  __shared__ float red[64];
  const NodeDesc d = v.desc[blockIdx.x];
  const DynParams q = dyn_params(v.theta + d.theta_off, 1);
  float w = node_w(v.wet, v.mask, d);
  int64_t cs;
  const float* u = dyn_input(v, d, cs);
  const float* dy = v.G + (int64_t)d.gout * 2 * v.L;
  const float* env = v.env + (int64_t)(v.env0 + d.aux) * v.L;
  float* gin = d.gin >= 0 ? v.G + (int64_t)d.gin * 2 * v.L : nullptr;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  float s_att = 0.f, s_rel = 0.f;
  float lam_next = 0.f, a_next = 0.f;
  const int64_t nch = (v.L + AR_CH - 1) / AR_CH;
  for (int64_t c = nch - 1; c >= 0; --c) {
    const int64_t s0 = c * AR_CH;
    const int len = (int)((v.L - s0) < AR_CH ? (v.L - s0) : AR_CH);
    for (int i = threadIdx.x; i < len; i += 64) {
      const int64_t n = s0 + i;
      lg[i] = dyn_dg<GATE>(q, w, env[n], u[n], u[cs + n], dy[n], dy[v.L + n], acc);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      float lam = lam_next, an = a_next;
      for (int i = len - 1; i >= 0; --i) {
        const int64_t n = s0 + i;
        lam = fmaf(an, lam, lg[i]);
        const float gp = (n > 0) ? env[n - 1] : 0.f;
        const float um = u[n] + u[cs + n];
        const float e = um * um;
        if (e > gp) {
          s_att += lam * (gp - e);
          an = q.aa;
          lg[i] = q.ba * lam;
        } else {
          s_rel += lam * (gp - e);
          an = q.ar;
          lg[i] = q.br * lam;
        }
      }
      lam_next = lam;
      a_next = an;
    }
    __syncthreads();
    if (gin) {
      for (int i = threadIdx.x; i < len; i += 64) {
        const int64_t n = s0 + i;
        const float g = env[n];
        const float G = logf(g + COMP_EPS);
        float a0, a1, a2, a3;
        const float gain = expf(curve<GATE>(G, q, a0, a1, a2, a3) - G);
        const float um = u[n] + u[cs + n];
        const float de2 = lg[i] * 2.0f * um;
        gin[n] = (1.0f - w) * dy[n] + w * gain * dy[n] + de2;
        gin[v.L + n] = (1.0f - w) * dy[v.L + n] + w * gain * dy[v.L + n] + de2;
      }
    }
    __syncthreads();
  }
  float* pr = v.part + ((int64_t)blockIdx.x * v.PB) * PK;
  const float s_dw = block_sum<64>(acc[0], red);
  const float sT = block_sum<64>(acc[1], red);
  const float sW = block_sum<64>(acc[2], red);
  const float sR = block_sum<64>(acc[3], red);
  if (threadIdx.x == 0) {
    pr[2] = s_dw;
    pr[3] = s_att * q.aa * q.ba;
    pr[4] = s_rel * q.ar * q.br;
    pr[5] = sT;
    pr[6] = sW;
    pr[7] = sR;
  }
}

// -------------------------------------------------------------- host
static DynView dyn_view(const Ctx& c, int type, int desc_off) {
  const mg_graph* g = c.g;
  DynView v;
  v.desc = c.desc + desc_off;
  v.dry = c.dry;
  v.U = c.U;
  v.G = c.G;
  v.env = (g->mode && !c.trial) ? wsp<float>(c, g->ws.ENV) : nullptr;
  v.theta = c.theta;
  v.wet = c.wet;
  v.mask = c.mask;
  v.L = c.L;
  v.C = c.C;
  v.env0 = (type == MG_COMP) ? 0 : g->type_count[MG_COMP];
  v.part = c.part + (int64_t)desc_off * c.PB * PK;
  v.PB = c.PB;
  return v;
}

void dyn_forward(const Ctx& c, int type, int desc_off, int n) {
  const mg_graph* g = c.g;
  DynView v = dyn_view(c, type, desc_off);
  ProfScope ps(c, "dyn", (double)n * 20.0 * c.L);
  const bool ar = (type == MG_COMP && g->cfg.comp_mode == 1);
  if (ar) {
    if (type == MG_COMP) MG_LAUNCH(c, k_dyn_ar_fwd<0>, dim3(n), dim3(64), 0, c.st, v);
    return;
  }
  const int nch = g->dyn_chunks;
  float* sums = wsp<float>(c, g->ws.cmp_sum);
  MG_LAUNCH(c, k_dyn_sum, dim3(nch, n), dim3(MG_BLOCK), 0, c.st, v, sums, nch);
  if (type == MG_GATE) MG_LAUNCH(c, k_dyn_apply<1>, dim3(nch, n), dim3(MG_BLOCK), 0, c.st, v, sums, nch);
  else MG_LAUNCH(c, k_dyn_apply<0>, dim3(nch, n), dim3(MG_BLOCK), 0, c.st, v, sums, nch);
}

void dyn_backward(const Ctx& c, int type, int desc_off, int n) {
  const mg_graph* g = c.g;
  DynView v = dyn_view(c, type, desc_off);
  ProfScope ps(c, "dyn", (double)n * 28.0 * c.L);
  const bool ar = (type == MG_COMP && g->cfg.comp_mode == 1);
  if (ar) {
    MG_LAUNCH(c, k_dyn_ar_bwd<0>, dim3(n), dim3(64), 0, c.st, v);
    return;
  }
  const int nch = g->dyn_chunks;
  float* sums = wsp<float>(c, g->ws.cmp_sum);
  if (type == MG_GATE) {
    MG_LAUNCH(c, k_dyn_bsum<1>, dim3(nch, n), dim3(MG_BLOCK), 0, c.st, v, sums, nch);
    MG_LAUNCH(c, k_dyn_bapply<1>, dim3(nch, n), dim3(MG_BLOCK), 0, c.st, v, sums, nch);
  } else {
    MG_LAUNCH(c, k_dyn_bsum<0>, dim3(nch, n), dim3(MG_BLOCK), 0, c.st, v, sums, nch);
    MG_LAUNCH(c, k_dyn_bapply<0>, dim3(nch, n), dim3(MG_BLOCK), 0, c.st, v, sums, nch);
  }
}

}  // namespace mg
