// Launch context and kernel launchers of the mixgraph library.
#pragma once
#include <hip/hip_ext.h>

#include "mg_internal.h"

namespace mg {

constexpr int PW_MAXK = 4;  // pointwise stages fused into one launch at most
// frames of one loss resolution per workgroup of the backward (host and
// kernels agree)
inline int loss_frames_per_block(int nfft) { return nfft >= 1024 ? 1 : 1024 / nfft; }
// the forward's (its partial rows are per block of these)
inline int loss_frames_per_block_fwd(int nfft) { return nfft >= 4096 ? 1 : 4096 / nfft; }
constexpr int PK = 8;  // floats of partial sums per (node, block)
// elements of one column block of the FFT engine (TC = COL_TILE / N2 columns)
constexpr int COL_TILE = 8192;

struct Ctx {
  const mg_graph* g;
  hipStream_t st;
  int64_t L;
  int C;                 // channels of the dry tracks (1 or 2)
  float* U;              // node outputs [slot][2][L]
  float* G;              // gradient buffers [slot][2][L]
  const float* dry;
  const float* theta;
  const float* wet;
  const float* mask;
  const NodeDesc* desc;  // device descriptor array
  const SrcRef* srcs;    // device source list
  float* part;           // partial sums [desc][PB][PK]
  int PB;                // blocks per node row of part
  double* lg;            // per desc: E_ybar, E_u (double)
  float alpha_g, alpha_p;
  char* base;            // workspace base
  bool trial = false;    // pruning-trial copies: keep no backward state, reuse
                         // the FIR tables and spectra of the last forward
  int vec4 = 0;          // L a multiple of 4 and the dry rows 16-byte aligned:
                         // the pointwise kernels move float4 runs
  bool defer_lg = false; // L_g energies reduced once after all stages
};

// effective dry/wet weight w = sigmoid(logit) * mask (Sec. 5.1 and the masked
// evaluation of Alg. 2); the same FP32 expression in every kernel
__device__ __forceinline__ float node_w(const float* wet, const float* mask, const NodeDesc& d) {
  float w = 1.0f / (1.0f + expf(-wet[d.proc]));
  if (mask) w *= mask[d.mrow];
  return w;
}

template <typename T>
inline T* wsp(const Ctx& c, size_t off) {
  return reinterpret_cast<T*>(c.base + off);
}

// Measurement scope of kernel class cls moving `bytes` algorithmic bytes: a
// no-op unless the graph's profiler targets cls.  Scopes nest; the innermost
// one names the class of the launches made inside it.  Timed launches carry
// their own start/stop events (hipExtLaunchKernelGGL stamps the dispatch
// itself), so timing adds no packets between kernels.
struct ProfScope {
  Profiler* q;
  const char* prev;
  ProfScope(const Ctx& c, const char* cls, double bytes) : q(const_cast<Profiler*>(&c.g->prof)), prev(q->cur) {
    q->cur = cls;
    if (q->cls.empty() || q->cls != cls) return;
    q->bytes += bytes;
    q->launches += 1;
  }
  ~ProfScope() { q->cur = prev; }
};

// the event pair of the next launch when it is timed; false otherwise
inline bool prof_pair(const Ctx& c, hipEvent_t& a, hipEvent_t& b) {
  Profiler* p = const_cast<Profiler*>(&c.g->prof);
  if (p->cls.empty() || !p->cur || p->cls != p->cur) return false;
  if (p->used + 2 > (int)p->ev.size()) {
    p->overflow = true;
    return false;
  }
  a = p->ev[p->used];
  b = p->ev[p->used + 1];
  p->used += 2;
  return true;
}

#define MG_LAUNCH(C, K, GRID, BLOCK, SHMEM, STREAM, ...)                                \
  do {                                                                                  \
    hipEvent_t ev_a_, ev_b_;                                                            \
    if (prof_pair(C, ev_a_, ev_b_))                                                     \
      hipExtLaunchKernelGGL(K, GRID, BLOCK, SHMEM, STREAM, ev_a_, ev_b_, 0, __VA_ARGS__); \
    else                                                                                \
      hipLaunchKernelGGL(K, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);                   \
  } while (0)

// mg_api.hip
Ctx make_ctx(const mg_graph* g, hipStream_t st);
int bind_workspace(mg_graph* g, void* workspace, size_t workspace_bytes, int32_t mode, const float* reverb_noise,
                   const float* target, hipStream_t st, bool make_side);
// mg_static.hip: MG_OK, or MG_ERR_STATE when the graph was bound to a static
// scratch that another graph has bound since
int check_binding(const mg_graph* g);
void forward_stage(const Ctx& c, int t, int off, int n, bool keep, const NodeDesc* hd);

// k_basic.hip
void launch_sum(const Ctx& c, int desc_off, int n, const SrcRef* srcs, float* out_base, int dest_kind);
// backward fan-out sums: dL/dy of each gdesc node from its consumers' slots
void launch_grad_sum(const Ctx& c, const NodeDesc* gdesc, int n);
void launch_pointwise_fwd(const Ctx& c, int type, int desc_off, int n);
void launch_pointwise_bwd(const Ctx& c, int type, int desc_off, int n);
// K (<= PW_MAXK) consecutive pointwise stages of n nodes each (types[i], descriptor offsets offs[i])
void launch_pw_chain_fwd(const Ctx& c, const int* types, const int* offs, int K, int n);
void launch_pw_chain_bwd(const Ctx& c, const int* types, const int* offs, int K, int n);
void launch_finish_grads(const Ctx& c, int desc_off, int n, int nblocks, int nparams, float* grad_theta,
                         float* grad_wet);
void launch_finish_all(const Ctx& c, int n_desc, const int2* fin, float* grad_theta, float* grad_wet);
void launch_reduce_lg(const Ctx& c, int desc_off, int n, int nblocks);
// all FIR nodes at once (fin: partial blocks per descriptor, flag: FIR node)
void launch_reduce_lg_all(const Ctx& c, int n_desc, const int2* fin, const int* flag);
void launch_finalize_losses(const Ctx& c, double* losses, const double* lstats, int n_res, int n_desc);
// one block per trial b: losses + 7 b, lstats + 128 b, mask + P b, sub + n_desc b
void launch_finalize_trials(const Ctx& c, double* losses, const double* lstats, int n_res, int n_desc,
                            const float* mask, int P, const int* sub, int n_trials);
void launch_adam(float* th, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                 int step, hipStream_t st, float weight_decay = 0.0f);
void launch_zero(void* p, size_t bytes, hipStream_t st);
// mask[b][p] = (base ? base[p] : 1) * keep[b][p]
void launch_trial_mask(float* mask, const float* base, const float* keep, int P, int B, hipStream_t st);

// k_fft.hip: the FIR convolution engine
void fft_init_tables(const Ctx& c, float2* tw, float2* twhi, float2* twlo, int N, hipStream_t st);
// FIR spectra of the stage's nodes -> ZH (T: column-pass temporary); the
// forward conv of stage nodes needs them ready
void conv_fir_spectrum(const Ctx& c, int type, int desc_off, int n, float2* T);
void conv_forward(const Ctx& c, int type, int desc_off, int n, bool keep_input_spectrum);
// backward in two parts: the input gradient (leaves the FIR-gradient
// spectrum in T3) and the FIR gradient at the FIR's lags (reads T3)
void conv_backward(const Ctx& c, int type, int desc_off, int n, float2* T3);
void conv_backward_fir(const Ctx& c, int type, int desc_off, int n, const float2* T3);

// k_eq.hip: equalizer by overlap-save in LDS
int eq_blocks(const mg_graph* g);
void eq_spectrum(const Ctx& c, int desc_off, int n);            // H_P of the stage's nodes
void eq_forward(const Ctx& c, int desc_off, int n, bool keep);  // needs H_P ready
void eq_backward(const Ctx& c, int desc_off, int n);      // input gradient and per-block FIR gradients
void eq_backward_fir(const Ctx& c, int desc_off, int n);  // FIR gradient: fixed-order sum over blocks

// k_fir.hip: FIR synthesis and adjoints
void fir_setup(const Ctx& c, const float* reverb_noise);
void fir_synth(const Ctx& c, int type, int desc_off, int n);
void fir_adjoint(const Ctx& c, int type, int desc_off, int n, float* grad_theta);

// k_dyn.hip
void dyn_forward(const Ctx& c, int type, int desc_off, int n);
void dyn_backward(const Ctx& c, int type, int desc_off, int n);

// k_loss.hip
void loss_setup(const Ctx& c, const float* target);
// the resident target features of a new target mix (tables already set up)
void loss_target(const Ctx& c, const float* target);
// stats: per-resolution statistics output (nullptr: the graph's own, which
// the backward reads)
void loss_forward(const Ctx& c, const float* yhat, double* stats = nullptr);
void loss_backward(const Ctx& c, const float* yhat, float* dyhat);

}  // namespace mg
