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

// Sample visiting shared by every pointwise kernel: with vec set (L a
// multiple of 4 and 16-byte aligned rows, decided once per call on the host)
// each thread takes runs of 4 consecutive samples, one float4 per channel
// row, else single samples; the order is the same in the per-stage and the
// fused kernels, so their per-thread partial sums agree bit for bit.
__device__ __forceinline__ void ld4(const float* p, float (&v)[4]) {
  const float4 t = *reinterpret_cast<const float4*>(p);
  v[0] = t.x;
  v[1] = t.y;
  v[2] = t.z;
  v[3] = t.w;
}
__device__ __forceinline__ void st4(float* p, const float (&v)[4]) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}

// ---------------------------------------------------------------- sums
// out[slot] = sum of sources, fixed order.  Sources: dry tracks, U slots or
// gradient slots.  dest_kind 0: the node's output slot; 1: its gradient
// slot; 2: its input-sum slot (processors with several predecessors).  With
// vec (L a multiple of 4, 16-byte aligned rows) each thread adds runs of four
// samples as float4; every sample's sources are added in the same order
// either way.
__global__ __launch_bounds__(MG_BLOCK) void k_sum(const NodeDesc* __restrict__ desc, const SrcRef* __restrict__ srcs,
                                                  const float* __restrict__ dry, const float* __restrict__ U,
                                                  const float* __restrict__ G, float* __restrict__ out_base,
                                                  int64_t L, int C, int dest_kind, int vec) {
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
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t k0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (vec && ns <= MAXS) {
    const int64_t q4 = L / 4;
    for (int64_t k = k0; k < 2 * q4; k += stride) {
      const int ch = k >= q4 ? 1 : 0;
      const int64_t t = (k - ch * q4) * 4;
      float acc[4] = {0.f, 0.f, 0.f, 0.f};
      for (int s = 0; s < ns; ++s) {
        float v[4];
        ld4(sp[s] + ch * sc[s] + t, v);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] += v[e];
      }
      st4(out + ch * L + t, acc);
    }
    return;
  }
  for (int64_t i = k0; i < 2 * L; i += stride) {
    const int ch = i >= L ? 1 : 0;
    const int64_t t = i - ch * L;
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
  // one float4 (or sample) per thread where the grid allows, up to 4096 blocks per node
  const int64_t items = c.vec4 ? (2 * c.L) / 4 : 2 * c.L;
  const unsigned bx = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (items + MG_BLOCK - 1) / MG_BLOCK));
  dim3 grid(bx, n);
  ProfScope ps(c, "sum", (double)n * 8.0 * c.L * 2);
  MG_LAUNCH(c, k_sum, grid, dim3(MG_BLOCK), 0, c.st, c.desc + desc_off, srcs, c.dry, c.U, c.G, out_base, c.L,
            c.C, dest_kind, c.vec4);
}

void launch_grad_sum(const Ctx& c, const NodeDesc* gdesc, int n) {
  if (n <= 0) return;
  const int64_t items = c.vec4 ? (2 * c.L) / 4 : 2 * c.L;
  const unsigned bx = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (items + MG_BLOCK - 1) / MG_BLOCK));
  dim3 grid(bx, n);
  ProfScope ps(c, "sum", (double)n * 8.0 * c.L * 2);
  MG_LAUNCH(c, k_sum, grid, dim3(MG_BLOCK), 0, c.st, gdesc, c.srcs, c.dry, c.U, c.G, c.G, c.L, c.C, 1, c.vec4);
}

// ---------------------------------------------------------------- pointwise processors
// Each processor keeps two numbers (a, b) derived from its raw parameters.
// Contraction is off from here to the end of the fused chains and every
// product that feeds an addition is an explicit fmaf: the per-stage kernels
// and the fused chains below then round identically (the compiler would
// otherwise fuse a product into a later subtraction only where the product
// has no other use, which differs between the two).
#pragma clang fp contract(off)
template <int T>
struct PW;

// Sec. 3.1 gain/panning: ybar_c = exp(p_c) u_c;  a, b = exp(p_l), exp(p_r)
template <>
struct PW<MG_GAINPAN> {
  float a, b;
  __device__ void init(const float* p) {
    a = expf(p[0]);
    b = expf(p[1]);
  }
  __device__ void fwd(float l, float r, float& yl, float& yr) const {
    yl = a * l;
    yr = b * r;
  }
  // dl, dr: dL/dybar.  returns dL/du and accumulates parameter partials
  __device__ void bwd(float l, float r, float dl, float dr, float& gl, float& gr, float* pp) const {
    gl = a * dl;
    gr = b * dr;
    pp[0] = fmaf(dl * a, l, pp[0]);
    pp[1] = fmaf(dr * b, r, pp[1]);
  }
};

// Sec. 3.2 stereo imager: ym = l + r, ys = exp(p)(l - r), ybar = ((ym + ys)/2,
// (ym - ys)/2);  a = exp(p)
template <>
struct PW<MG_IMAGER> {
  float a, b;
  __device__ void init(const float* p) {
    a = expf(p[0]);
    b = 0.0f;
  }
  __device__ void fwd(float l, float r, float& yl, float& yr) const {
    const float ym = l + r, d = l - r;
    yl = 0.5f * fmaf(a, d, ym);
    yr = 0.5f * fmaf(-a, d, ym);
  }
  __device__ void bwd(float l, float r, float dl, float dr, float& gl, float& gr, float* pp) const {
    const float dm = 0.5f * (dl + dr), ds = 0.5f * (dl - dr);
    gl = fmaf(a, ds, dm);
    gr = fmaf(-a, ds, dm);
    pp[0] = fmaf(ds * a, l - r, pp[0]);
  }
};

// tanh waveshaper: ybar = exp(p_o) tanh(exp(p_i) u);  a, b = exp(p_i), exp(p_o)
template <>
struct PW<MG_DIST> {
  float a, b;
  __device__ void init(const float* p) {
    a = expf(p[0]);
    b = expf(p[1]);
  }
  __device__ void fwd(float l, float r, float& yl, float& yr) const {
    yl = b * tanhf(a * l);
    yr = b * tanhf(a * r);
  }
  __device__ void bwd(float l, float r, float dl, float dr, float& gl, float& gr, float* pp) const {
    const float tl = tanhf(a * l), tr = tanhf(a * r);
    const float sl = b * a * fmaf(-tl, tl, 1.0f), sr = b * a * fmaf(-tr, tr, 1.0f);
    gl = dl * sl;
    gr = dr * sr;
    pp[0] = fmaf(dl * sl, l, fmaf(dr * sr, r, pp[0]));   // d/dp_i = ybar'(u) u
    pp[1] = fmaf(dl * b, tl, fmaf(dr * b, tr, pp[1]));   // d/dp_o = ybar
  }
};

// dry/wet mix y = w ybar + (1 - w) u
__device__ __forceinline__ float dw_mix(float w, float yb, float u) { return fmaf(w, yb, (1.0f - w) * u); }

// Adjoint of one processor with its dry/wet mix at one stereo sample: input
// (l, r), wet output (yl, yr), dL/dy (dl, dr) -> dL/du (gl, gr); dry/wet and
// parameter partials accumulated.
template <int T>
__device__ __forceinline__ void pw_level_bwd(const PW<T>& f, float w, float l, float r, float yl, float yr, float dl,
                                             float dr, float& gl, float& gr, float& dw, float* pp) {
  dw = fmaf(dl, yl - l, fmaf(dr, yr - r, dw));
  float bl, br;
  f.bwd(l, r, w * dl, w * dr, bl, br, pp);
  gl = fmaf(1.0f - w, dl, bl);
  gr = fmaf(1.0f - w, dr, br);
}

template <int T>
__global__ __launch_bounds__(MG_BLOCK) void k_pointwise_fwd(const NodeDesc* __restrict__ desc,
                                                             const float* __restrict__ dry, float* __restrict__ U,
                                                             const float* __restrict__ theta,
                                                             const float* __restrict__ wet,
                                                             const float* __restrict__ mask, int64_t L, int C,
                                                             int vec) {
  const NodeDesc d = desc[blockIdx.y];
  PW<T> f;
  f.init(theta + d.theta_off);
  const float w = wet_of(d, wet, mask);
  int64_t cs;
  const float* u = resolve_in(d, dry, U, L, C, cs);
  float* y = U + (int64_t)d.out_slot * 2 * L;
  const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  if (vec) {
    for (int64_t q = start; q < L / 4; q += stride) {
      float l[4], r[4], ol[4], orr[4];
      ld4(u + 4 * q, l);
      ld4(u + cs + 4 * q, r);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        float yl, yr;
        f.fwd(l[k], r[k], yl, yr);
        ol[k] = dw_mix(w, yl, l[k]);
        orr[k] = dw_mix(w, yr, r[k]);
      }
      st4(y + 4 * q, ol);
      st4(y + L + 4 * q, orr);
    }
    return;
  }
  for (int64_t t = start; t < L; t += stride) {
    const float l = u[t], r = u[cs + t];
    float yl, yr;
    f.fwd(l, r, yl, yr);
    y[t] = dw_mix(w, yl, l);
    y[L + t] = dw_mix(w, yr, r);
  }
}

// partial sums of one processor: [2] dry/wet, [3], [4] parameters
__device__ __forceinline__ void pw_partials(float* pr, float dw, float p0, float p1, float* red) {
  const float s_dw = block_sum<MG_BLOCK>(dw, red);
  const float s0 = block_sum<MG_BLOCK>(p0, red);
  const float s1 = block_sum<MG_BLOCK>(p1, red);
  if (threadIdx.x == 0) {
    pr[2] = s_dw;
    pr[3] = s0;
    pr[4] = s1;
  }
}

template <int T>
__global__ __launch_bounds__(MG_BLOCK) void k_pointwise_bwd(const NodeDesc* __restrict__ desc,
                                                             const float* __restrict__ dry,
                                                             const float* __restrict__ U, float* __restrict__ G,
                                                             const float* __restrict__ theta,
                                                             const float* __restrict__ wet,
                                                             const float* __restrict__ mask, int64_t L, int C,
                                                             float* __restrict__ part, int PB, int vec) {
  __shared__ float red[MG_BLOCK / 64];
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
  const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  if (vec) {
    for (int64_t q = start; q < L / 4; q += stride) {
      float l[4], r[4], dl[4], dr[4], gl[4], gr[4];
      ld4(u + 4 * q, l);
      ld4(u + cs + 4 * q, r);
      ld4(dy + 4 * q, dl);
      ld4(dy + L + 4 * q, dr);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        float yl, yr;
        f.fwd(l[k], r[k], yl, yr);
        pw_level_bwd(f, w, l[k], r[k], yl, yr, dl[k], dr[k], gl[k], gr[k], dw, pp);
      }
      if (gin) {
        st4(gin + 4 * q, gl);
        st4(gin + L + 4 * q, gr);
      }
    }
  } else {
    for (int64_t t = start; t < L; t += stride) {
      const float l = u[t], r = u[cs + t];
      float yl, yr, gl, gr;
      f.fwd(l, r, yl, yr);
      pw_level_bwd(f, w, l, r, yl, yr, dy[t], dy[L + t], gl, gr, dw, pp);
      if (gin) {
        gin[t] = gl;
        gin[L + t] = gr;
      }
    }
  }
  pw_partials(part + ((int64_t)(blockIdx.y) * PB + blockIdx.x) * PK, dw, pp[0], pp[1], red);
}

// ---------------------------------------------------------------- fused pointwise chains
// K consecutive pointwise stages whose node j feeds only node j of the next
// stage (x -> s -> g of every console chain) in one launch.  Forward: one
// read of the chain input, every level's output written (the backward, the
// pruning trials and the next stage read them).  Backward: the level inputs
// are recomputed from the chain input, dL/dy of the last level is carried
// back through the levels in registers and only the chain's input gradient
// is written; the per-level partials are those of the per-stage kernels.
struct PwChain {
  const NodeDesc* desc[PW_MAXK];  // descriptors of each level's stage
  float* part[PW_MAXK];           // partial rows of each level's stage
  int type[PW_MAXK];
  int K;
};

__device__ __forceinline__ void pw_init_rt(int type, const float* p, float& a, float& b) {
  if (type == MG_GAINPAN) {
    PW<MG_GAINPAN> f;
    f.init(p);
    a = f.a;
    b = f.b;
  } else if (type == MG_IMAGER) {
    PW<MG_IMAGER> f;
    f.init(p);
    a = f.a;
    b = f.b;
  } else {
    PW<MG_DIST> f;
    f.init(p);
    a = f.a;
    b = f.b;
  }
}

__device__ __forceinline__ void pw_fwd_rt(int type, float a, float b, float l, float r, float& yl, float& yr) {
  if (type == MG_GAINPAN) PW<MG_GAINPAN>{a, b}.fwd(l, r, yl, yr);
  else if (type == MG_IMAGER) PW<MG_IMAGER>{a, b}.fwd(l, r, yl, yr);
  else PW<MG_DIST>{a, b}.fwd(l, r, yl, yr);
}

__device__ __forceinline__ void pw_bwd_rt(int type, float a, float b, float w, float l, float r, float yl, float yr,
                                          float dl, float dr, float& gl, float& gr, float& dw, float* pp) {
  if (type == MG_GAINPAN) pw_level_bwd(PW<MG_GAINPAN>{a, b}, w, l, r, yl, yr, dl, dr, gl, gr, dw, pp);
  else if (type == MG_IMAGER) pw_level_bwd(PW<MG_IMAGER>{a, b}, w, l, r, yl, yr, dl, dr, gl, gr, dw, pp);
  else pw_level_bwd(PW<MG_DIST>{a, b}, w, l, r, yl, yr, dl, dr, gl, gr, dw, pp);
}

__global__ __launch_bounds__(MG_BLOCK) void k_pw_chain_fwd(PwChain ch, const float* __restrict__ dry,
                                                            float* __restrict__ U, const float* __restrict__ theta,
                                                            const float* __restrict__ wet,
                                                            const float* __restrict__ mask, int64_t L, int C,
                                                            int vec) {
  float pa[PW_MAXK], pb[PW_MAXK], pw[PW_MAXK];
  float* y[PW_MAXK];
#pragma unroll
  for (int i = 0; i < PW_MAXK; ++i) {
    if (i >= ch.K) break;
    const NodeDesc d = ch.desc[i][blockIdx.y];
    pw_init_rt(ch.type[i], theta + d.theta_off, pa[i], pb[i]);
    pw[i] = node_w(wet, mask, d);
    y[i] = U + (int64_t)d.out_slot * 2 * L;
  }
  int64_t cs;
  const float* u = resolve_in(ch.desc[0][blockIdx.y], dry, U, L, C, cs);
  const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  if (vec) {
    for (int64_t q = start; q < L / 4; q += stride) {
      float l[4], r[4];
      ld4(u + 4 * q, l);
      ld4(u + cs + 4 * q, r);
#pragma unroll
      for (int i = 0; i < PW_MAXK; ++i) {
        if (i >= ch.K) break;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          float yl, yr;
          pw_fwd_rt(ch.type[i], pa[i], pb[i], l[k], r[k], yl, yr);
          l[k] = dw_mix(pw[i], yl, l[k]);
          r[k] = dw_mix(pw[i], yr, r[k]);
        }
        st4(y[i] + 4 * q, l);
        st4(y[i] + L + 4 * q, r);
      }
    }
    return;
  }
  for (int64_t t = start; t < L; t += stride) {
    float l = u[t], r = u[cs + t];
#pragma unroll
    for (int i = 0; i < PW_MAXK; ++i) {
      if (i >= ch.K) break;
      float yl, yr;
      pw_fwd_rt(ch.type[i], pa[i], pb[i], l, r, yl, yr);
      l = dw_mix(pw[i], yl, l);
      r = dw_mix(pw[i], yr, r);
      y[i][t] = l;
      y[i][L + t] = r;
    }
  }
}

__global__ __launch_bounds__(MG_BLOCK) void k_pw_chain_bwd(PwChain ch, const float* __restrict__ dry,
                                                            const float* __restrict__ U, float* __restrict__ G,
                                                            const float* __restrict__ theta,
                                                            const float* __restrict__ wet,
                                                            const float* __restrict__ mask, int64_t L, int C,
                                                            int PB, int vec) {
  __shared__ float red[MG_BLOCK / 64];
  float pa[PW_MAXK], pb[PW_MAXK], pw[PW_MAXK];
  float dw[PW_MAXK], pp[PW_MAXK][2];
#pragma unroll
  for (int i = 0; i < PW_MAXK; ++i) {
    dw[i] = pp[i][0] = pp[i][1] = 0.0f;
    if (i >= ch.K) continue;
    const NodeDesc d = ch.desc[i][blockIdx.y];
    pw_init_rt(ch.type[i], theta + d.theta_off, pa[i], pb[i]);
    pw[i] = node_w(wet, mask, d);
  }
  const NodeDesc d0 = ch.desc[0][blockIdx.y];
  int64_t cs;
  const float* u = resolve_in(d0, dry, U, L, C, cs);
  const float* dy = G + (int64_t)ch.desc[ch.K - 1][blockIdx.y].gout * 2 * L;
  float* gin = d0.gin >= 0 ? G + (int64_t)d0.gin * 2 * L : nullptr;
  // one sample through the chain and back; returns dL/du
  auto sample = [&](float l, float r, float gl, float gr, float& ol, float& orr) {
    float li[PW_MAXK], ri[PW_MAXK], yl[PW_MAXK], yr[PW_MAXK];
#pragma unroll
    for (int i = 0; i < PW_MAXK; ++i) {
      if (i >= ch.K) break;
      li[i] = l;
      ri[i] = r;
      pw_fwd_rt(ch.type[i], pa[i], pb[i], l, r, yl[i], yr[i]);
      l = dw_mix(pw[i], yl[i], l);
      r = dw_mix(pw[i], yr[i], r);
    }
#pragma unroll
    for (int i = PW_MAXK - 1; i >= 0; --i) {
      if (i >= ch.K) continue;
      float bl, br;
      pw_bwd_rt(ch.type[i], pa[i], pb[i], pw[i], li[i], ri[i], yl[i], yr[i], gl, gr, bl, br, dw[i], pp[i]);
      gl = bl;
      gr = br;
    }
    ol = gl;
    orr = gr;
  };
  const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  if (vec) {
    for (int64_t q = start; q < L / 4; q += stride) {
      float l[4], r[4], dl[4], dr[4], gl[4], gr[4];
      ld4(u + 4 * q, l);
      ld4(u + cs + 4 * q, r);
      ld4(dy + 4 * q, dl);
      ld4(dy + L + 4 * q, dr);
#pragma unroll
      for (int k = 0; k < 4; ++k) sample(l[k], r[k], dl[k], dr[k], gl[k], gr[k]);
      if (gin) {
        st4(gin + 4 * q, gl);
        st4(gin + L + 4 * q, gr);
      }
    }
  }
  for (int64_t t = start; t < L && !vec; t += stride) {
    float li[PW_MAXK], ri[PW_MAXK], yl[PW_MAXK], yr[PW_MAXK];
    float l = u[t], r = u[cs + t];
#pragma unroll
    for (int i = 0; i < PW_MAXK; ++i) {
      if (i >= ch.K) break;
      li[i] = l;
      ri[i] = r;
      pw_fwd_rt(ch.type[i], pa[i], pb[i], l, r, yl[i], yr[i]);
      l = dw_mix(pw[i], yl[i], l);
      r = dw_mix(pw[i], yr[i], r);
    }
    float gl = dy[t], gr = dy[L + t];
#pragma unroll
    for (int i = PW_MAXK - 1; i >= 0; --i) {
      if (i >= ch.K) continue;
      float ol, orr;
      pw_bwd_rt(ch.type[i], pa[i], pb[i], pw[i], li[i], ri[i], yl[i], yr[i], gl, gr, ol, orr, dw[i], pp[i]);
      gl = ol;
      gr = orr;
    }
    if (gin) {
      gin[t] = gl;
      gin[L + t] = gr;
    }
  }
#pragma unroll
  for (int i = 0; i < PW_MAXK; ++i) {
    if (i >= ch.K) break;
    pw_partials(ch.part[i] + ((int64_t)(blockIdx.y) * PB + blockIdx.x) * PK, dw[i], pp[i][0], pp[i][1], red);
  }
}

#pragma clang fp contract(fast)

// forward grids (no per-block partials): 128 blocks per node, more for small
// stages so that a launch has about 2048 blocks
static dim3 pw_fwd_grid(const Ctx& c, int n) {
  const int64_t items = c.vec4 ? (c.L + 3) / 4 : c.L;
  const int64_t want = std::max<int64_t>(128, 2048 / std::max(1, n));
  const int64_t need = std::max<int64_t>(1, (items + MG_BLOCK - 1) / MG_BLOCK);
  return dim3((unsigned)std::min(want, need), n);
}

void launch_pointwise_fwd(const Ctx& c, int type, int desc_off, int n) {
  dim3 grid = pw_fwd_grid(c, n), blk(MG_BLOCK);
  ProfScope ps(c, "pointwise", (double)n * 16.0 * c.L);
  const NodeDesc* d = c.desc + desc_off;
  switch (type) {
    case MG_GAINPAN:
      MG_LAUNCH(c, k_pointwise_fwd<MG_GAINPAN>, grid, blk, 0, c.st, d, c.dry, c.U, c.theta, c.wet, c.mask, c.L, c.C, c.vec4);
      break;
    case MG_IMAGER:
      MG_LAUNCH(c, k_pointwise_fwd<MG_IMAGER>, grid, blk, 0, c.st, d, c.dry, c.U, c.theta, c.wet, c.mask, c.L, c.C, c.vec4);
      break;
    case MG_DIST:
      MG_LAUNCH(c, k_pointwise_fwd<MG_DIST>, grid, blk, 0, c.st, d, c.dry, c.U, c.theta, c.wet, c.mask, c.L, c.C, c.vec4);
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
      MG_LAUNCH(c, k_pointwise_bwd<MG_GAINPAN>, grid, blk, 0, c.st, d, c.dry, c.U, c.G, c.theta, c.wet, c.mask,
                c.L, c.C, part, c.PB, c.vec4);
      break;
    case MG_IMAGER:
      MG_LAUNCH(c, k_pointwise_bwd<MG_IMAGER>, grid, blk, 0, c.st, d, c.dry, c.U, c.G, c.theta, c.wet, c.mask,
                c.L, c.C, part, c.PB, c.vec4);
      break;
    case MG_DIST:
      MG_LAUNCH(c, k_pointwise_bwd<MG_DIST>, grid, blk, 0, c.st, d, c.dry, c.U, c.G, c.theta, c.wet, c.mask,
                c.L, c.C, part, c.PB, c.vec4);
      break;
  }
}

static PwChain pw_chain(const Ctx& c, const int* types, const int* offs, int K) {
  PwChain ch;
  ch.K = K;
  for (int i = 0; i < PW_MAXK; ++i) {
    const int k = i < K ? i : 0;
    ch.desc[i] = c.desc + offs[k];
    ch.part[i] = c.part + (int64_t)offs[k] * c.PB * PK;
    ch.type[i] = types[k];
  }
  return ch;
}

void launch_pw_chain_fwd(const Ctx& c, const int* types, const int* offs, int K, int n) {
  dim3 grid = pw_fwd_grid(c, n), blk(MG_BLOCK);
  ProfScope ps(c, "pointwise", (double)n * (8.0 + 8.0 * K) * c.L);
  MG_LAUNCH(c, k_pw_chain_fwd, grid, blk, 0, c.st, pw_chain(c, types, offs, K), c.dry, c.U, c.theta, c.wet, c.mask,
            c.L, c.C, c.vec4);
}

void launch_pw_chain_bwd(const Ctx& c, const int* types, const int* offs, int K, int n) {
  dim3 grid(128, n), blk(MG_BLOCK);
  ProfScope ps(c, "pointwise", (double)n * 24.0 * c.L);
  MG_LAUNCH(c, k_pw_chain_bwd, grid, blk, 0, c.st, pw_chain(c, types, offs, K), c.dry, c.U, c.G, c.theta, c.wet,
            c.mask, c.L, c.C, c.PB, c.vec4);
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
  MG_LAUNCH(c, k_finish_grads, dim3(n), dim3(MG_BLOCK), 0, c.st, c.desc + desc_off,
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
  MG_LAUNCH(c, k_finish_all, dim3(n_desc), dim3(MG_BLOCK), 0, c.st, c.desc, c.part, c.PB, fin, c.wet, c.mask,
                     c.alpha_p, grad_theta, grad_wet);
}

// L_g energies of one node: out[k] = sum over blocks of partial k, k = 0, 1
// (E_ybar, E_u), strided per thread then the block sum
__device__ __forceinline__ void reduce_lg_row(const float* pr, int nblocks, double* out, double* red) {
  for (int k = 0; k < 2; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += MG_BLOCK) s += (double)pr[b * PK + k];
    s = block_sum<MG_BLOCK>(s, red);
    if (threadIdx.x == 0) out[k] = s;
  }
}

__global__ __launch_bounds__(MG_BLOCK) void k_reduce_lg(const float* __restrict__ part, int PB, int nblocks,
                                                         double* __restrict__ lg) {
  __shared__ double red[MG_BLOCK / 64];
  reduce_lg_row(part + (int64_t)blockIdx.x * PB * PK, nblocks, lg + 2 * blockIdx.x, red);
}

// every FIR node of the graph in one launch (fin[j].x partial blocks, flag[j]
// set for FIR nodes); the same sums as one k_reduce_lg per stage
__global__ __launch_bounds__(MG_BLOCK) void k_reduce_lg_all(const float* __restrict__ part, int PB,
                                                             const int2* __restrict__ fin,
                                                             const int* __restrict__ flag,
                                                             double* __restrict__ lg) {
  __shared__ double red[MG_BLOCK / 64];
  const int j = blockIdx.x;
  if (!flag[j]) return;
  reduce_lg_row(part + (int64_t)j * PB * PK, fin[j].x, lg + 2 * j, red);
}

void launch_reduce_lg(const Ctx& c, int desc_off, int n, int nblocks) {
  if (n <= 0 || c.defer_lg) return;
  MG_LAUNCH(c, k_reduce_lg, dim3(n), dim3(MG_BLOCK), 0, c.st, c.part + (int64_t)desc_off * c.PB * PK, c.PB,
                     nblocks, c.lg + 2 * desc_off);
}

void launch_reduce_lg_all(const Ctx& c, int n_desc, const int2* fin, const int* flag) {
  if (n_desc <= 0) return;
  MG_LAUNCH(c, k_reduce_lg_all, dim3(n_desc), dim3(MG_BLOCK), 0, c.st, c.part, c.PB, fin, flag, c.lg);
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
  MG_LAUNCH(c, k_finalize_losses, dim3(1), dim3(MG_BLOCK), 0, c.st, losses, lstats, n_res, c.desc, n_desc,
                     c.lg, c.wet, c.mask, 0, (const int*)nullptr, c.alpha_g, c.alpha_p, flag);
}

void launch_finalize_trials(const Ctx& c, double* losses, const double* lstats, int n_res, int n_desc,
                            const float* mask, int P, const int* sub, int n_trials) {
  if (n_trials <= 0) return;
  const int* flag = reinterpret_cast<const int*>(c.base + c.g->ws.losses_tmp);
  MG_LAUNCH(c, k_finalize_losses, dim3(n_trials), dim3(MG_BLOCK), 0, c.st, losses, lstats, n_res, c.desc,
                     n_desc, c.lg, c.wet, mask, P, sub, c.alpha_g, c.alpha_p, flag);
}

// ---------------------------------------------------------------- Adam
// Adam (Kingma & Ba); with decay != 1 the decoupled weight decay of AdamW
// (Loshchilov & Hutter) scales the parameter first: decay = 1 - lr * wd.
// decay = 1 multiplies exactly, so Adam is AdamW with wd = 0 bit for bit.
__global__ __launch_bounds__(MG_BLOCK) void k_adam(float* __restrict__ th, float* __restrict__ m,
                                                    float* __restrict__ v, const float* __restrict__ g, int64_t n,
                                                    float lr, float b1, float b2, float eps, float c1, float c2,
                                                    float decay) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] = th[i] * decay - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

void launch_adam(float* th, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                 int step, hipStream_t st, float weight_decay) {
  const float c1 = (float)(1.0 - pow((double)b1, step));
  const float c2 = (float)(1.0 - pow((double)b2, step));
  const float decay = (float)(1.0 - (double)lr * (double)weight_decay);
  int64_t blocks = (n + MG_BLOCK - 1) / MG_BLOCK;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(MG_BLOCK), 0, st, th, m, v, g, n, lr, b1, b2, eps, c1, c2,
                     decay);
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
