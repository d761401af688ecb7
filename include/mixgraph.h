/* mixgraph: batched mixing-console forward/backward, MRSTFT loss and masked
 * pruning evaluation on one MI355X (gfx950).
 *
 * The calls follow the problem statement of "Reverse Engineering of Music
 * Mixing Graphs with Differentiable Processors and Iterative Pruning"
 * (arxiv 2509.15948): given dry tracks S, a graph G = (T, E) (Sec. 1.1,
 * Sec. 4: node-type vector and 2 x |E| edge tensor), parameters
 * P = (P_bar, w) and dry/wet masks, compute the mix y_hat = G(S; P)
 * (Alg. 1), the audio loss L_a and regularisers (Sec. 5.1, Sec. 6.3), and
 * gradients of L with respect to P_bar and the dry/wet logits.
 *
 * Conventions shared by every call
 *  - Return value: MG_OK (0) or one of the MG_ERR_* codes below; after a
 *    failure mg_last_error() returns a message (thread-local, valid until the
 *    next call on the same thread).  Nothing is thrown across the ABI.
 *  - "dev" pointers are HIP device memory owned by the caller; "host"
 *    pointers are ordinary host memory owned by the caller.  The library owns
 *    only the mg_graph object (host memory) and never allocates device memory:
 *    every device buffer it uses lives in the caller's workspace.
 *  - stream is a hipStream_t passed as void*; compute calls only enqueue
 *    work on it and return.  Results are valid after the stream completes.
 *    Asynchronous device faults surface as MG_ERR_HIP on a later call.
 *  - Audio is FP32, planar [channel][sample]; a track is [C][L] with C = 1
 *    (mono, used for both channels) or C = 2.
 *  - Parameters: theta is one flat FP32 vector; for each processor type t in
 *    the order e c n x s g d r it holds the block P[t] of shape [|V_t|][N_t],
 *    rows in the library's node order sigma (Alg. 1 "Reorder").  The offset
 *    of every node's row is reported by mg_graph_layout.  The dry/wet logits
 *    are a separate FP32 vector wet[P] over processors in sigma order
 *    (w = sigmoid(logit) * mask, Sec. 5.1 initialisation).
 */
#ifndef MIXGRAPH_H
#define MIXGRAPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum mg_status {
  MG_OK = 0,
  MG_ERR_INVALID_ARG = 1, /* null pointer, bad size or unsupported option  */
  MG_ERR_GRAPH = 2,       /* cycle, bad arity, unknown type, != 1 output    */
  MG_ERR_SHAPE = 3,       /* sizes inconsistent with the graph or workspace */
  MG_ERR_STATE = 4,       /* call order violated (e.g. backward w/o forward) */
  MG_ERR_HIP = 5,         /* a HIP runtime call failed                      */
  MG_ERR_BUDGET = 6,      /* the request does not fit the memory it is given */
  MG_ERR_OOM = 7,         /* the HIP runtime ran out of device memory       */
  MG_ERR_NONFINITE = 8    /* a loss handed to a decision rule is NaN or inf */
};

/* Node types (Sec. 1.1): auxiliary input i, mix m, output o; processors
 * equalizer e, compressor c, noisegate n, tanh waveshaper x, stereo imager s,
 * gain/panning g, multitap delay d, reverb r. */
enum mg_type {
  MG_IN = 0, MG_MIX = 1, MG_OUT = 2, MG_EQ = 3, MG_COMP = 4, MG_GATE = 5,
  MG_DIST = 6, MG_IMAGER = 7, MG_GAINPAN = 8, MG_DELAY = 9, MG_REVERB = 10
};

/* Per-graph configuration.  Sizes of the processors (Sec. 3) and the loss
 * (Sec. 5.1). */
typedef struct mg_config {
  int64_t length;          /* L: samples per channel                          */
  int32_t sample_rate;     /* fs in Hz                                        */
  int32_t eq_taps;         /* N of the zero-phase EQ FIR, odd (Sec. 3.3)      */
  int32_t comp_mode;       /* 0: one coefficient (Sec. 3.5); 1: attack/release */
  int32_t delay_taps;      /* M delays per channel (Sec. 3.7)                 */
  int32_t delay_range;     /* D: samples per delay range                      */
  int32_t delay_fir_taps;  /* length of each tap's zero-phase FIR, odd        */
  int32_t reverb_length;   /* L_r: reverb FIR length (Sec. 3.4)              */
  int32_t reverb_nfft;     /* STFT size of the reverb mask (384)              */
  int32_t reverb_hop;      /* hop (nfft / 2)                                  */
  int32_t n_loss_ffts;     /* number of MRSTFT resolutions (<= 8)             */
  int32_t loss_ffts[8];    /* FFT sizes, powers of two in [64, 4096]          */
  int32_t n_mels;          /* Mel bands (96)                                  */
  int32_t loss_skip;       /* leading samples excluded from the loss          */
  int32_t max_trials;      /* pruning trials per mg_forward_trials call (0:
                              none); reserves the trial tables              */
  int32_t trial_slots;     /* node outputs [2][L] reserved for trial copies;
                              0 picks max_trials x the largest suffix of one
                              processor, so single-processor trials run as
                              one batch                                      */
  int32_t unfused;         /* 1: one launch per pointwise stage instead of one
                              per chain of consecutive pointwise stages (same
                              results; for checks)                           */
  double alpha_g;          /* gain-staging regulariser weight                 */
  double alpha_p;          /* dry/wet l1 regulariser weight                   */
  int32_t schedule_rule;   /* type schedule (Sec. 4.2): 0 the shortest of the
                              three below; 1 the console walk (the substring
                              of the console type string); 2 greedy (the type
                              with the most computable nodes each step); 3
                              beam search                                   */
  int32_t beam_width;      /* beam of rule 3 (and of rule 0); 0 picks 8      */
} mg_config;

typedef struct mg_graph mg_graph;

/* Sizes derived by mg_graph_create. */
typedef struct mg_info {
  int32_t n_nodes;
  int32_t n_processors;    /* P: length of the dry/wet logit and mask vectors */
  int32_t n_stages;        /* N + 1 of Alg. 1, input stage included          */
  int32_t fft_size;        /* FFT length used for the FIR convolutions        */
  int64_t n_theta;         /* length of the flat parameter vector             */
  int32_t n_reverbs;       /* rows of the reverb noise input                  */
  int32_t n_losses;        /* values written per loss record (7)              */
} mg_info;

/* Validate a graph and build its schedule, node order and parameter layout
 * on the host (Alg. 1 ScheduleBatchedProcessing, OptimizeNodeOrder,
 * Reorder, GetReadWriteIndex; Sec. 4.2 type scheduling).
 *   types       host int32[n_nodes], values of enum mg_type
 *   edges       host int32[2][n_edges]: row 0 sources, row 1 destinations
 *   input_track host int32[n_nodes]: dry-track index of each MG_IN node,
 *               ignored for other nodes
 *   n_tracks, track_channels: shape [n_tracks][track_channels][L] of the dry
 *               input; track_channels is 1 or 2
 *   cfg         host, copied
 * Errors: MG_ERR_GRAPH for a cycle, an unknown type, an input with
 * predecessors, a processor or mix without inputs, an output count != 1, a
 * node that cannot reach the output; MG_ERR_INVALID_ARG for bad sizes.     */
int mg_graph_create(int32_t n_nodes, const int32_t* types, int32_t n_edges,
                    const int32_t* edges, const int32_t* input_track,
                    int32_t n_tracks, int32_t track_channels,
                    const mg_config* cfg, mg_graph** out);

int mg_graph_destroy(mg_graph* g);

int mg_graph_info(const mg_graph* g, mg_info* out);

/* Layout of the parameters and schedule (all host arrays of n_nodes, any may
 * be NULL):
 *   param_offset  offset of the node's row in theta, -1 for i/m/o
 *   proc_index    index of the node in wet/mask vectors, -1 for i/m/o
 *   stage         stage (0 = inputs) of Alg. 1's subset sequence
 *   type_row      row of the node inside its type block P[t]
 *   schedule      host char[n_stages + 1]: the type string, NUL-terminated */
int mg_graph_layout(const mg_graph* g, int64_t* param_offset, int32_t* proc_index,
                    int32_t* stage, int32_t* type_row, char* schedule);

/* Device workspace needed by the graph (bytes).  mode 0: forward only;
 * mode 1: forward and backward. */
int mg_workspace_size(const mg_graph* g, int32_t mode, size_t* bytes);

/* Device memory one search on this graph holds (bytes), for admission by a
 * memory budget: *workspace = mg_workspace_size(g, mode); *state = the
 * caller-side buffers the calls read and write: dry tracks, reverb noise,
 * target, mix, theta with its gradient and two optimiser moments, the
 * dry/wet logits likewise, the loss record and (max_trials > 0) the trial
 * losses.  Host only.                                                        */
int mg_footprint(const mg_graph* g, int32_t mode, size_t* workspace, size_t* state);

/* Bind a caller-owned device workspace (>= mg_workspace_size bytes, 256-byte
 * aligned) and prepare per-graph device tables: FFT twiddles, Mel/A-weight
 * tables, the STFT of every reverb's fixed noise, and the Mel spectra of the
 * target mix (Sec. 5.1, "target features are resident").
 *   reverb_noise dev float[n_reverbs][2][L_r], rows in type_row order of the
 *                reverb nodes: uniform noise for the mid and side FIR (Sec. 3.4)
 *   target       dev float[2][L]: the target mix y
 * For signals shorter than 2^21 samples the graph also creates a second
 * stream and its events (once), on which the forward and backward run the
 * FIR synthesis, FIR spectra and parameter gradients beside the chain; for
 * longer ones every launch stays on the caller's stream.  Results are the
 * same either way.                                                          */
int mg_setup(mg_graph* g, void* workspace, size_t workspace_bytes, int32_t mode,
             const float* reverb_noise, const float* target, void* stream);

/* Bytes of the static device scratch behind mg_setup_static (64 MiB). */
#define MG_STATIC_SCRATCH_BYTES (64ull << 20)

/* mg_setup without a caller-owned workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops that
 * must not allocate, harnesses that forbid hipMalloc).  The workspace is a
 * static device array of MG_STATIC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends; this call and the compute
 * calls on the graph afterwards allocate nothing (no hipMalloc, no stream or
 * event is created: the graph's work all runs on the caller's stream, in
 * the same order and with the same results as after mg_setup).
 *   mode, reverb_noise, target, stream: as mg_setup (the current device's
 *   array is used)
 * Errors: MG_ERR_BUDGET when mg_workspace_size(g, mode) exceeds
 * MG_STATIC_SCRATCH_BYTES; otherwise those of mg_setup.
 * One array per GPU: binding another graph on the same device takes it over,
 * and the earlier graph's compute calls return MG_ERR_STATE until it is
 * bound again.  The array keeps the last call's contents (setup clears what
 * the kernels accumulate into).  Calls that overlap on one GPU race. */
int mg_setup_static(mg_graph* g, int32_t mode, const float* reverb_noise, const float* target, void* stream);

/* Alg. 1 forward pass and the loss (Sec. 5.1):
 *   dry      dev float[n_tracks][track_channels][L]
 *   theta    dev float[n_theta]
 *   wet      dev float[P] dry/wet logits
 *   mask     dev float[P] multiplied into w (Alg. 2 Evaluate), or NULL
 *   mix      dev float[2][L] output y_hat, or NULL
 *   losses   dev double[7]: L, L_a, L_lr, L_m, L_s, L_g, L_p, with
 *            L = L_a + alpha_g L_g + alpha_p L_p
 * With mode 1 the forward also keeps what mg_backward needs in the
 * workspace; dry/theta/wet/mask must stay unchanged until mg_backward. */
int mg_forward(mg_graph* g, const float* dry, const float* theta, const float* wet,
               const float* mask, float* mix, double* losses, void* stream);

/* Gradients of L from the last mg_forward (hand-written adjoints of every
 * processor, Sec. 3; delay z entries follow the Sec. 3.7 update rule).
 *   grad_theta dev float[n_theta] (overwritten)
 *   grad_wet   dev float[P]       (overwritten)                              */
int mg_backward(mg_graph* g, float* grad_theta, float* grad_wet, void* stream);

/* Masked evaluation (Alg. 2 Evaluate with w * m * m_cand): a complete forward
 * pass and loss for each of B masks, one after another on the stream (the
 * reference for mg_forward_trials, which recomputes only suffixes).
 *   masks  dev float[B][P];  losses dev double[B][7].                        */
int mg_forward_masked(mg_graph* g, const float* dry, const float* theta, const float* wet,
                      const float* masks, int32_t B, double* losses, void* stream);

/* Pruning trials by suffix recomputation (Alg. 2 Evaluate for a batch of
 * candidate masks, Sec. 4.1 batching).  Trial b uses the mask of the last
 * mg_forward multiplied by keep[b]; a processor with keep 0 is bypassed
 * (w = 0, so y = u, Sec. 1.2).  Only the nodes downstream of a bypassed
 * processor are evaluated again, reading every other node's output from the
 * last mg_forward; the copies of one stage across all trials run in one
 * launch per kernel, then each trial's loss is taken.  The results equal B
 * separate mg_forward calls with those masks bit for bit.
 *   keep    host uint8[B][P] (P = processors, proc_index order); B <= max_trials
 *   losses  dev double[B][7], as mg_forward
 * Requires a preceding mg_forward (MG_ERR_STATE otherwise) whose dry, theta,
 * wet and mask buffers still hold the same values; does not disturb a
 * pending mg_backward.  Trials
 * whose copies exceed trial_slots run in several batches; one trial that
 * alone needs more than trial_slots fails with MG_ERR_SHAPE.                */
int mg_forward_trials(mg_graph* g, const uint8_t* keep, int32_t B, double* losses, void* stream);

/* Decision rule of one pruning round (Alg. 2 with a batched trial step), host
 * only.  Phase 1: candidates are the first max_n processors with alive != 0
 * ordered by (w ascending, index), w = sigmoid(wet[p]) * mask[p] the
 * effective dry/wet weight (Sec. 5.1); cand receives their indices, *n_out
 * the count.  wet, mask (may be NULL: all ones), alive: host arrays of P.    */
int mg_prune_candidates(int32_t P, const float* wet, const float* mask, const uint8_t* alive, int32_t max_n,
                        int32_t* cand, int32_t* n_out);

/* Phase 2: from the single-bypass losses L_cand[i] of cand[i] (i < n), keep
 * those with L_cand - L_min < tol, ordered by (L_cand - L_min, index) into
 * order; *n_out their count.  tol = tau * L_min when relative != 0 (the
 * benchmark configuration's 1e-3), tol = tau otherwise (the paper's absolute
 * tolerance, Sec. 6.1).  The trial masks of phase 3 bypass the prefixes
 * order[0..k-1], k = 1..*n_out.                                            */
int mg_prune_order(int32_t n, const int32_t* cand, const double* L_cand, double L_min, double tau,
                   int32_t relative, int32_t* order, int32_t* n_out);

/* Phase 3: the largest k with L_prefix[k-1] < L_min (1 + tau) (relative) or
 * < L_min + tau (absolute), 0 if none.
 * Phases 2 and 3 return MG_ERR_NONFINITE when L_min is NaN or infinite (the
 * search itself has failed); a non-finite trial loss never passes the test,
 * so such a candidate or prefix is simply not accepted.                      */
int mg_prune_accept(int32_t n, const double* L_prefix, double L_min, double tau, int32_t relative,
                    int32_t* k_out);

/* The dry/wet method (Alg. 3, Sec. 6.2 "Candidate Sampling"), host only: one
 * pruning iteration as a sequence of trials the caller evaluates.
 *   mg_drywet_begin: P processors; proc_type host int32[P] (enum mg_type of
 *     each processor, proc_index order); wet, mask (NULL: ones), alive as
 *     mg_prune_candidates; L_min the threshold; tau with relative as
 *     mg_prune_order; u host double[n_u]: the uniform draws in [0, 1) that
 *     pick the type of each trial (the floor(u |T|)-th remaining type in the
 *     order e c n x s g d r), one per trial.  Per type: N_t = its alive count,
 *     r_t = 0.1.
 *   mg_drywet_next: keep host uint8[P] receives the next trial (0: bypassed:
 *     what is pruned so far plus the floor(N_t r_t + 1/2) least-weight alive
 *     processors of the drawn type, at least one, ties by index); *done = 1
 *     and keep untouched when no type is left.  MG_ERR_SHAPE when the draws
 *     run out, MG_ERR_STATE when the last trial's loss was not reported.
 *   mg_drywet_report: the loss L_a of that trial.  L passing the tolerance
 *     test prunes the candidates and sets L_min = min(L_min, L) (the type
 *     leaves once all its processors are pruned); otherwise r_t is halved if
 *     floor(N_t r_t + 1/2) > 1, else the type leaves.  A NaN loss fails.
 *   mg_drywet_end: keep host uint8[P] (may be NULL) receives the final mask
 *     (1 = kept), *L_min the threshold, *trials the trial count; frees s.   */
typedef struct mg_drywet mg_drywet;
int mg_drywet_begin(int32_t P, const int32_t* proc_type, const float* wet, const float* mask,
                    const uint8_t* alive, double L_min, double tau, int32_t relative, const double* u,
                    int32_t n_u, mg_drywet** out);
int mg_drywet_next(mg_drywet* s, uint8_t* keep, int32_t* done);
int mg_drywet_report(mg_drywet* s, double L);
int mg_drywet_end(mg_drywet* s, uint8_t* keep, double* L_min, int32_t* trials);

/* One Adam step (Kingma & Ba) on n parameters, in place on theta, m, v.
 * step counts from 1.  All pointers dev float[n]. */
int mg_adam_step(float* theta, float* m, float* v, const float* grad, int64_t n,
                 float lr, float beta1, float beta2, float eps, int32_t step, void* stream);

/* AdamW (Loshchilov & Hutter, the optimiser of Sec. 5.1): the decoupled
 * weight decay scales theta by 1 - lr * weight_decay, then the Adam step of
 * mg_adam_step follows (weight_decay = 0 gives mg_adam_step bit for bit).
 * All pointers dev float[n]; step counts from 1.                            */
int mg_adamw_step(float* theta, float* m, float* v, const float* grad, int64_t n, float lr, float beta1,
                  float beta2, float eps, float weight_decay, int32_t step, void* stream);

/* A new target mix for the loss (Sec. 5.1: each step compares the mix of a
 * random segment with the same segment of the target): recomputes the
 * resident target Mel features from target, dev float[2][L] of the graph's
 * length, on the stream.  A pending mg_backward and the cached forward of
 * mg_forward_trials are dropped (MG_ERR_STATE until the next mg_forward).   */
int mg_target_prepare(mg_graph* g, const float* target, void* stream);

/* The regulariser weights alpha_g and alpha_p of L = L_a + alpha_g L_g +
 * alpha_p L_p (Sec. 5.1, Sec. 6.3: alpha_p rises during pruning), used from
 * the next mg_forward on.  MG_ERR_STATE between a forward and its backward
 * (the two must see the same weights); MG_ERR_INVALID_ARG for a negative
 * weight.  Host only.                                                       */
int mg_set_alpha(mg_graph* g, double alpha_g, double alpha_p);

/* Graph surgery for pruning (Sec. 1.2: removing a node and rerouting its
 * edges is equivalent to bypass).  keep: host uint8[P] over processors in
 * proc_index order.  Produces a new graph; old_to_new (host int32[n_nodes],
 * may be NULL) maps old node ids to new ids (-1 for removed nodes).  The new
 * graph has its own layout and needs its own workspace and mg_setup. */
int mg_graph_prune(const mg_graph* g, const uint8_t* keep, mg_graph** out,
                   int32_t* old_to_new);

/* Parameters of a graph made by mg_graph_prune, taken from those of the
 * original: each kept processor keeps its row of theta (its raw parameters,
 * Sec. 3) and its dry/wet logit.  Any vector in theta's layout (Adam moments)
 * maps the same way.
 *   old_to_new  host int32[n_nodes of g], as filled by mg_graph_prune
 *   src_theta   dev float[n_theta of g]      -> dst_theta dev float[n_theta of pruned]
 *   src_wet     dev float[P of g]            -> dst_wet   dev float[P of pruned]
 * Either pair may be NULL.  Device-to-device copies on the stream.          */
int mg_remap_params(const mg_graph* g, const mg_graph* pruned, const int32_t* old_to_new,
                    const float* src_theta, float* dst_theta, const float* src_wet, float* dst_wet,
                    void* stream);

/* Copy node v's output y_v (the store of Alg. 1: every non-input node's
 * output stays in the workspace) into out, dev float[2][L], on the stream.
 * Reads what the last mg_forward (or mg_forward_masked: its last mask) left;
 * trials write their copies elsewhere and leave it unchanged.  For checks and
 * inspection.  Input nodes have no slot (their output is the dry track):
 * MG_ERR_INVALID_ARG; no workspace bound: MG_ERR_STATE. */
int mg_node_output(const mg_graph* g, int32_t node, float* out, void* stream);

/* Measurement of one kernel class (for roofline reporting, not part of the
 * method): after mg_profile_enable(g, cls), every kernel launched for that
 * class ("conv_cols", "conv_rows", "conv_icols", "eq_conv", "eq_spec", "dyn",
 * "pointwise", "sum", "loss", "fir", "reverb_fir"; NULL disables) carries a
 * start/stop HIP event pair stamped by its own dispatch, so timing inserts
 * nothing between kernels.  One launch of a class may be several kernels
 * (the dynamics passes, the loss resolutions); their durations add.  At most
 * 4096 timed kernels between reads, else mg_profile_read fails and resets.
 * mg_profile_read synchronises on the events and returns the summed kernel
 * time in ms, the number of class launches and the algorithmic bytes they
 * move (the reads and writes each kernel is designed to make), then resets. */
int mg_profile_enable(mg_graph* g, const char* kernel_class);
int mg_profile_read(mg_graph* g, double* ms, int64_t* launches, double* bytes);

const char* mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
