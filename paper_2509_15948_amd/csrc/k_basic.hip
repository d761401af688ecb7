// Memory-bound kernels of the mixgraph library:
//  * segmented sums of node outputs (mix / output nodes, Sec. 3 eq. for u_i;
//    Alg. 1 Gather + Aggregate) and of gradient contributions (backward);
//  * the fused elementwise processors with the dry/wet mix (Sec. 3.1 gain/pan,
//    Sec. 3.2 stereo imager, tanh waveshaper) and their adjoints;
//  * fixed-order reductions of per-block partial sums; loss finalisation;
//  * Adam.
// Every stage launch covers all nodes of the stage: grid.y = node, grid.x =
// blocks along time.  HBM traffic per stereo sample is one read of the input
// and one write of the output (8 + 8 bytes) in the forward.
#include <algorithm>

#include "mg_device.h"
#include "mg_kernels.h"

namespace mg {

__device__ __forceinline__ const float* resolve_in(const NodeDesc& d, const float* dry, const float* U, int64_t L,
                                                   int C, int64_t& cs) {
  if (d.in_kind == 0) {
    cs = (C == 1) ? 0 : L;
    return dry + (int64_t)d.in_slot * C * L;
  }
  cs = L;
  return U + (int64_t)d.in_slot * 2 * L;
}

__device__ __forceinline__ float wet_of(const NodeDesc& d, const float* wet, const float* mask) {
  float w = node_w(wet, mask, d);
  return w;
}

// ---------------------------------------------------------------- sums
// out[slot] = sum of sources, fixed order.  Sources: dry tracks, U slots or
// gradient slots.  dest_kind 0: the node's output slot; 1: its gradient
// slot; 2: its input-sum slot (processors with several predecessors).
__global__ __launch_bounds__(MG_BLOCK) void k_sum(const NodeDesc* __restrict__ desc, const SrcRef* __restrict__ srcs,
                                                   const float* __restrict__ dry, const float* __restrict__ U,
                                                   const float* __restrict__ G, float* __restrict__ out_base,
                                                   int64_t L, int C, int dest_kind) {
  constexpr int MAXS = 64;  // sources resolved once per block (more are read directly)
  __shared__ const float* sp[MAXS];
  __shared__ int64_t sc[MAXS];
  const NodeDesc d = desc[blockIdx.y];
  if (d.src_count == 0) return;
  const int ns = d.src_count;
  for (int s = threadIdx.x; s < ns && s < MAXS; s += MG_BLOCK) {
    const SrcRef r = srcs[d.src_begin + s];
    if (r.kind == 0) {
      sp[s] = dry + (int64_t)r.slot * C * L;
      sc[s] = (C == 1) ? 0 : L;
    } else {
      sp[s] = (r.kind == 1 ? U : G) + (int64_t)r.slot * 2 * L;
      sc[s] = L;
    }
  }
  __syncthreads();
  const int64_t slot = dest_kind == 0 ? d.out_slot : (dest_kind == 1 ? d.gout : d.in_slot);
  float* out = out_base + slot * 2 * L;
  const int64_t n2 = 2 * L;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x) {
    const int ch = (int)(i / L);
    const int64_t t = i - (int64_t)ch * L;
    float acc = 0.0f;
    for (int s = 0; s < ns; ++s) {
      float v;
      if (s < MAXS) {
        v = sp[s][ch * sc[s] + t];
      } else {
        const SrcRef r = srcs[d.src_begin + s];
        if (r.kind == 0) v = dry[(int64_t)r.slot * C * L + (C == 1 ? 0 : ch * L) + t];
        else if (r.kind == 1) v = U[(int64_t)r.slot * 2 * L + i];
        else v = G[(int64_t)r.slot * 2 * L + i];
      }
      acc += v;
    }
    out[i] = acc;
  }
}

void launch_sum(const Ctx& c, int desc_off, int n, const SrcRef* srcs, float* out_base, int dest_kind) {
  if (n <= 0) return;
  dim3 grid(256, n);
  ProfScope ps(c, "sum", (double)n * 8.0 * c.L * 2);
  hipLaunchKernelGGL(k_sum, grid, dim3(MG_BLOCK), 0, c.st, c.desc + desc_off, srcs, c.dry, c.U, c.G, out_base, c.L,
                     c.C, dest_kind);
}

// ---------------------------------------------------------------- pointwise processors
template <int T>
struct PW;

// Sec. 3.1 gain/panning: ybar_c = exp(p_c) u_c
template <>
struct PW<MG_GAINPAN> {
  float a0, a1;
  __device__ void init(const float* p) {
    a0 = expf(p[0]);
    a1 = expf(p[1]);
  }
  __device__ void fwd(float l, float r, float& yl, float& yr) const {
    yl = a0 * l;
    yr = a1 * r;
  }
  // dl, dr: dL/dybar.  returns dL/du and accumulates parameter partials
  __device__ void bwd(float l, float r, float dl, float dr, float& gl, float& gr, float* pp) const {
    gl = a0 * dl;
    gr = a1 * dr;
    pp[0] += dl * a0 * l;
    pp[1] += dr * a1 * r;
  }
};

// Sec. 3.2 stereo imager: ym = l + r, ys = exp(p)(l - r), ybar = ((ym + ys)/2, (ym - ys)/2)
template <>
struct PW<MG_IMAGER> {
  float s;
  __device__ void init(const float* p) { s = expf(p[0]); }
  __device__ void fwd(float l, float r, float& yl, float& yr) const {
    const float ym = l + r, ys = s * (l - r);
    yl = 0.5f * (ym + ys);
    yr = 0.5f * (ym - ys);
  }
  __device__ void bwd(float l, float r, float dl, float dr, float& gl, float& gr, float* pp) const {
    const float dm = 0.5f * (dl + dr), ds = 0.5f * (dl - dr);
    gl = dm + s * ds;
    gr = dm - s * ds;
    pp[0] += ds * s * (l - r);
  }
};

// tanh waveshaper: ybar = exp(p_o) tanh(exp(p_i) u)
template <>
struct PW<MG_DIST> {
  float gi, go;
  __device__ void init(const float* p) {
    gi = expf(p[0]);
    go = expf(p[1]);
  }
  __device__ void fwd(float l, float r, float& yl, float& yr) const {
    yl = go * tanhf(gi * l);
    yr = go * tanhf(gi * r);
  }
  __device__ void bwd(float l, float r, float dl, float dr, float& gl, float& gr, float* pp) const {
    const float tl = tanhf(gi * l), tr = tanhf(gi * r);
    const float sl = go * gi * (1.0f - tl * tl), sr = go * gi * (1.0f - tr * tr);
    gl = dl * sl;
    gr = dr * sr;
    pp[0] += dl * sl * l + dr * sr * r;   // d/dp_i = ybar'(u) * u
    pp[1] += dl * go * tl + dr * go * tr; // d/dp_o = ybar
  }
};

template <int T>
__global__ __launch_bounds__(MG_BLOCK) void k_pointwise_fwd(const NodeDesc* __restrict__ desc,
                                                             const float* __restrict__ dry, float* __restrict__ U,
                                                             const float* __restrict__ theta,
                                                             const float* __restrict__ wet,
                                                             const float* __restrict__ mask, int64_t L, int C) {
  const NodeDesc d = desc[blockIdx.y];
  PW<T> f;
  f.init(theta + d.theta_off);
  const float w = wet_of(d, wet, mask);
  int64_t cs;
  const float* u = resolve_in(d, dry, U, L, C, cs);
  float* y = U + (int64_t)d.out_slot * 2 * L;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < L; t += (int64_t)gridDim.x * blockDim.x) {
    const float l = u[t], r = u[cs + t];
    float yl, yr;
    f.fwd(l, r, yl, yr);
    y[t] = w * yl + (1.0f - w) * l;
    y[L + t] = w * yr + (1.0f - w) * r;
  }
}

template <int T>
__global__ __launch_bounds__(MG_BLOCK) void k_pointwise_bwd(const NodeDesc* __restrict__ desc,
                                                             const float* __restrict__ dry,
                                                             const float* __restrict__ U, float* __restrict__ G,
                                                             const float* __restrict__ theta,
                                                             const float* __restrict__ wet,
                                                             const float* __restrict__ mask, int64_t L, int C,
                                                             float* __restrict__ part, int PB) {
  __shared__ float red[MG_BLOCK];
  const NodeDesc d = desc[blockIdx.y];
  PW<T> f;
  f.init(theta + d.theta_off);
  const float w = wet_of(d, wet, mask);
  int64_t cs;
  const float* u = resolve_in(d, dry, U, L, C, cs);
  const float* dy = G + (int64_t)d.gout * 2 * L;
  float* gin = d.gin >= 0 ? G + (int64_t)d.gin * 2 * L : nullptr;
  float pp[2] = {0.0f, 0.0f};
  float dw = 0.0f;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < L; t += (int64_t)gridDim.x * blockDim.x) {
    const float l = u[t], r = u[cs + t];
    const float dl = dy[t], dr = dy[L + t];
    float yl, yr;
    f.fwd(l, r, yl, yr);
    dw += dl * (yl - l) + dr * (yr - r);
    float gl, gr;
    f.bwd(l, r, w * dl, w * dr, gl, gr, pp);
    if (gin) {
      gin[t] = gl + (1.0f - w) * dl;
      gin[L + t] = gr + (1.0f - w) * dr;
    }
  }
  float* pr = part + ((int64_t)(blockIdx.y) * PB + blockIdx.x) * PK;
  const float s_dw = block_sum<MG_BLOCK>(dw, red);
  const float s0 = block_sum<MG_BLOCK>(pp[0], red);
  const float s1 = block_sum<MG_BLOCK>(pp[1], red);
  if (threadIdx.x == 0) {
    pr[2] = s_dw;
    pr[3] = s0;
    pr[4] = s1;
  }
}

void launch_pointwise_fwd(const Ctx& c, int type, int desc_off, int n) {
  dim3 grid(128, n), blk(MG_BLOCK);
  ProfScope ps(c, "pointwise", (double)n * 16.0 * c.L);
  const NodeDesc* d = c.desc + desc_off;
  switch (type) {
    case MG_GAINPAN:
      hipLaunchKernelGGL(k_pointwise_fwd<MG_GAINPAN>, grid, blk, 0, c.st, d, c.dry, c.U, c.theta, c.wet, c.mask, c.L, c.C);
      break;
    case MG_IMAGER:
      hipLaunchKernelGGL(k_pointwise_fwd<MG_IMAGER>, grid, blk, 0, c.st, d, c.dry, c.U, c.theta, c.wet, c.mask, c.L, c.C);
      break;
    case MG_DIST:
      hipLaunchKernelGGL(k_pointwise_fwd<MG_DIST>, grid, blk, 0, c.st, d, c.dry, c.U, c.theta, c.wet, c.mask, c.L, c.C);
      break;
  }
}

void launch_pointwise_bwd(const Ctx& c, int type, int desc_off, int n) {
  dim3 grid(128, n), blk(MG_BLOCK);
  ProfScope ps(c, "pointwise", (double)n * 24.0 * c.L);
  const NodeDesc* d = c.desc + desc_off;
  float* part = c.part + (int64_t)desc_off * c.PB * PK;
  switch (type) {
    case MG_GAINPAN:
      hipLaunchKernelGGL(k_pointwise_bwd<MG_GAINPAN>, grid, blk, 0, c.st, d, c.dry, c.U, c.G, c.theta, c.wet, c.mask,
                         c.L, c.C, part, c.PB);
      break;
    case MG_IMAGER:
      hipLaunchKernelGGL(k_pointwise_bwd<MG_IMAGER>, grid, blk, 0, c.st, d, c.dry, c.U, c.G, c.theta, c.wet, c.mask,
                         c.L, c.C, part, c.PB);
      break;
    case MG_DIST:
      hipLaunchKernelGGL(k_pointwise_bwd<MG_DIST>, grid, blk, 0, c.st, d, c.dry, c.U, c.G, c.theta, c.wet, c.mask,
                         c.L, c.C, part, c.PB);
      break;
  }
}

// ---------------------------------------------------------------- reductions
// One workgroup per node: sums partial k over nblocks in FP64 (fixed order:
// strided per thread, then a tree), then writes dL/d(wet logit) (with the
// sigmoid chain, the mask and the l1 regulariser of Sec. 6.3) and nparams
// direct parameter gradients.
__global__ __launch_bounds__(MG_BLOCK) void k_finish_grads(const NodeDesc* __restrict__ desc,
                                                            const float* __restrict__ part, int PB, int nblocks,
                                                            int nparams, const float* __restrict__ wet,
                                                            const float* __restrict__ mask, float alpha_p,
                                                            float* __restrict__ grad_theta,
                                                            float* __restrict__ grad_wet) {
  __shared__ double red[MG_BLOCK];
  const NodeDesc d = desc[blockIdx.x];
  const float* pr = part + (int64_t)blockIdx.x * PB * PK;
  for (int q = 0; q < 1 + nparams; ++q) {
    const int kk = (q == 0) ? 2 : 2 + q;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += MG_BLOCK) s += (double)pr[b * PK + kk];
    s = block_sum<MG_BLOCK>(s, red);
    if (threadIdx.x == 0) {
      if (q == 0) {
        const double sg = 1.0 / (1.0 + exp(-(double)wet[d.proc]));
        const double m = mask ? (double)mask[d.mrow] : 1.0;
        grad_wet[d.proc] = (float)((s + (double)alpha_p) * sg * (1.0 - sg) * m);
      } else {
        grad_theta[d.theta_off + (q - 1)] = (float)s;
      }
    }
  }
}

void launch_finish_grads(const Ctx& c, int desc_off, int n, int nblocks, int nparams, float* grad_theta,
                         float* grad_wet) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_finish_grads, dim3(n), dim3(MG_BLOCK), 0, c.st, c.desc + desc_off,
                     c.part + (int64_t)desc_off * c.PB * PK, c.PB, nblocks, nparams, c.wet, c.mask, c.alpha_p,
                     grad_theta, grad_wet);
}

// The same for every processor of the graph in one launch: fin[j] holds the
// partial-sum blocks and the direct parameter count of descriptor j (0, 0
// for mix/output nodes).  Every block reads only its own node's partials.
__global__ __launch_bounds__(MG_BLOCK) void k_finish_all(const NodeDesc* __restrict__ desc,
                                                          const float* __restrict__ part, int PB,
                                                          const int2* __restrict__ fin,
                                                          const float* __restrict__ wet,
                                                          const float* __restrict__ mask, float alpha_p,
                                                          float* __restrict__ grad_theta,
                                                          float* __restrict__ grad_wet) {
  __shared__ double red[MG_BLOCK];
  const int j = blockIdx.x;
  const NodeDesc d = desc[j];
  if (d.proc < 0) return;
  const int2 f = fin[j];
  const float* pr = part + (int64_t)j * PB * PK;
  for (int q = 0; q < 1 + f.y; ++q) {
    const int kk = (q == 0) ? 2 : 2 + q;
    double s = 0.0;
    for (int b = threadIdx.x; b < f.x; b += MG_BLOCK) s += (double)pr[b * PK + kk];
    s = block_sum<MG_BLOCK>(s, red);
    if (threadIdx.x == 0) {
      if (q == 0) {
        const double sg = 1.0 / (1.0 + exp(-(double)wet[d.proc]));
        const double m = mask ? (double)mask[d.mrow] : 1.0;
        grad_wet[d.proc] = (float)((s + (double)alpha_p) * sg * (1.0 - sg) * m);
      } else {
        grad_theta[d.theta_off + (q - 1)] = (float)s;
      }
    }
  }
}

void launch_finish_all(const Ctx& c, int n_desc, const int2* fin, float* grad_theta, float* grad_wet) {
  if (n_desc <= 0) return;
  hipLaunchKernelGGL(k_finish_all, dim3(n_desc), dim3(MG_BLOCK), 0, c.st, c.desc, c.part, c.PB, fin, c.wet, c.mask,
                     c.alpha_p, grad_theta, grad_wet);
}

// L_g energies: lg[desc] = (sum over blocks of partial 0, of partial 1)
__global__ __launch_bounds__(MG_BLOCK) void k_reduce_lg(const float* __restrict__ part, int PB, int nblocks,
                                                         double* __restrict__ lg) {
  __shared__ double red[MG_BLOCK];
  const float* pr = part + (int64_t)blockIdx.x * PB * PK;
  for (int k = 0; k < 2; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += MG_BLOCK) s += (double)pr[b * PK + k];
    s = block_sum<MG_BLOCK>(s, red);
    if (threadIdx.x == 0) lg[2 * blockIdx.x + k] = s;
  }
}

void launch_reduce_lg(const Ctx& c, int desc_off, int n, int nblocks) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_reduce_lg, dim3(n), dim3(MG_BLOCK), 0, c.st, c.part + (int64_t)desc_off * c.PB * PK, c.PB,
                     nblocks, c.lg + 2 * desc_off);
}

// losses[7] = L, La, Llr, Lm, Ls, Lg, Lp.
// lstats per (resolution, combo): [0] sum |Y|^2, [1] sum |Y - Yh|^2,
// [2] sum |log diff| / cells.
// One block per loss record b (the graph itself: one block, sub = nullptr).
// L_g and L_p run over the graph's nodes in descriptor order; a trial takes
// node j's energies from lg row sub[j] (its copy, or j itself), so the sums
// are formed in the same order as for a complete forward with that mask.
__global__ __launch_bounds__(MG_BLOCK) void k_finalize_losses(double* __restrict__ losses,
                                                               const double* __restrict__ lstats, int n_res,
                                                               const NodeDesc* __restrict__ desc, int n_desc,
                                                               const double* __restrict__ lg,
                                                               const float* __restrict__ wet,
                                                               const float* __restrict__ mask, int mask_stride,
                                                               const int* __restrict__ sub, float alpha_g,
                                                               float alpha_p, const int* __restrict__ lg_flag) {
  __shared__ double red[MG_BLOCK];
  const int b = blockIdx.x;
  losses += 7 * b;
  lstats += 128 * b;
  if (mask) mask += (int64_t)mask_stride * b;
  if (sub) sub += (int64_t)n_desc * b;
  double lgs = 0.0, lps = 0.0;
  for (int j = threadIdx.x; j < n_desc; j += MG_BLOCK) {
    const NodeDesc d = desc[j];
    if (d.proc < 0) continue;
    double w = 1.0 / (1.0 + exp(-(double)wet[d.proc]));
    if (mask) w *= (double)mask[d.mrow];
    lps += w;
    const int r = sub ? sub[j] : j;
    if (lg_flag[j]) lgs += fabs(0.5 * log(lg[2 * r] + 1e-12) - 0.5 * log(lg[2 * r + 1] + 1e-12));
  }
  const double Lg = block_sum<MG_BLOCK>(lgs, red);
  const double Lp = block_sum<MG_BLOCK>(lps, red);
  if (threadIdx.x != 0) return;
  double term[4] = {0, 0, 0, 0};
  for (int i = 0; i < n_res; ++i)
    for (int x = 0; x < 4; ++x) {
      const double* s = lstats + (i * 4 + x) * 4;
      const double sc = sqrt(s[1]) / (sqrt(s[0]) + 1e-12);
      term[x] += s[2] + sc;
    }
  const double Llr = 0.5 * (term[0] + term[1]);
  const double La = 0.5 * Llr + 0.25 * term[2] + 0.25 * term[3];
  losses[0] = La + (double)alpha_g * Lg + (double)alpha_p * Lp;
  losses[1] = La;
  losses[2] = Llr;
  losses[3] = term[2];
  losses[4] = term[3];
  losses[5] = Lg;
  losses[6] = Lp;
}

void launch_finalize_losses(const Ctx& c, double* losses, const double* lstats, int n_res, int n_desc) {
  const int* flag = reinterpret_cast<const int*>(c.base + c.g->ws.losses_tmp);
  hipLaunchKernelGGL(k_finalize_losses, dim3(1), dim3(MG_BLOCK), 0, c.st, losses, lstats, n_res, c.desc, n_desc,
                     c.lg, c.wet, c.mask, 0, (const int*)nullptr, c.alpha_g, c.alpha_p, flag);
}

void launch_finalize_trials(const Ctx& c, double* losses, const double* lstats, int n_res, int n_desc,
                            const float* mask, int P, const int* sub, int n_trials) {
  if (n_trials <= 0) return;
  const int* flag = reinterpret_cast<const int*>(c.base + c.g->ws.losses_tmp);
  hipLaunchKernelGGL(k_finalize_losses, dim3(n_trials), dim3(MG_BLOCK), 0, c.st, losses, lstats, n_res, c.desc,
                     n_desc, c.lg, c.wet, mask, P, sub, c.alpha_g, c.alpha_p, flag);
}

// ---------------------------------------------------------------- Adam
__global__ __launch_bounds__(MG_BLOCK) void k_adam(float* __restrict__ th, float* __restrict__ m,
                                                    float* __restrict__ v, const float* __restrict__ g, int64_t n,
                                                    float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

void launch_adam(float* th, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                 int step, hipStream_t st) {
  const float c1 = (float)(1.0 - pow((double)b1, step));
  const float c2 = (float)(1.0 - pow((double)b2, step));
  int64_t blocks = (n + MG_BLOCK - 1) / MG_BLOCK;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(MG_BLOCK), 0, st, th, m, v, g, n, lr, b1, b2, eps, c1, c2);
}

// Trial masks: the mask of the cached forward times each trial's keep flags.
__global__ void k_trial_mask(float* __restrict__ mask, const float* __restrict__ base,
                             const float* __restrict__ keep, int P, int B) {
  const int64_t n = (int64_t)P * B;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    mask[i] = (base ? base[i % P] : 1.0f) * keep[i];
}

void launch_trial_mask(float* mask, const float* base, const float* keep, int P, int B, hipStream_t st) {
  const int64_t n = (int64_t)P * B;
  if (n <= 0) return;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + MG_BLOCK - 1) / MG_BLOCK, 1024);
  hipLaunchKernelGGL(k_trial_mask, dim3(blocks), dim3(MG_BLOCK), 0, st, mask, base, keep, P, B);
}

// Zero fill with a kernel (no memset nodes, so a caller may capture it).
__global__ void k_zero(uint32_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}

void launch_zero(void* p, size_t bytes, hipStream_t st) {
  size_t n = bytes / 4;
  if (!n) return;
  size_t blocks = (n + MG_BLOCK - 1) / MG_BLOCK;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(MG_BLOCK), 0, st, (uint32_t*)p, n);
}

}  // namespace mg
