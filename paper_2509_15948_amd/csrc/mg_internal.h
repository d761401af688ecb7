// Internal structures of the mixgraph library: the compiled graph (host),
// per-stage node descriptors (device-visible PODs) and kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/mixgraph.h"

namespace mg {

constexpr int NTYPES = 11;
// processor types in parameter-block order
constexpr int kProcOrder[8] = {MG_EQ, MG_COMP, MG_GATE, MG_DIST, MG_IMAGER, MG_GAINPAN, MG_DELAY, MG_REVERB};
inline bool is_proc(int t) { return t >= MG_EQ && t <= MG_REVERB; }
inline bool is_conv(int t) { return t == MG_EQ || t == MG_DELAY || t == MG_REVERB; }
inline bool is_dyn(int t) { return t == MG_COMP || t == MG_GATE; }
inline char type_char(int t) {
  static const char c[] = "imoecnxsgdr";
  return (t >= 0 && t < NTYPES) ? c[t] : '?';
}

// One node of a stage, as the kernels see it.  Pointers are resolved from
// slots: U slot -> U + slot * 2L; dry track -> dry + slot * C * L.
struct NodeDesc {
  int32_t node;       // user node id
  int32_t proc;       // processor index (sigma order), -1 for m/o
  int32_t in_kind;    // 0: dry track, 1: U slot
  int32_t in_slot;
  int32_t out_slot;   // U slot of the output
  int32_t aux;        // row inside the type block (ybar/env/conv/fir tables)
  int32_t gin;        // gradient slot receiving dL/du (-1: not needed)
  int32_t gout;       // gradient slot holding dL/dy
  int64_t theta_off;  // offset of the parameter row in theta
  int32_t src_begin;  // m/o/sum: range in the source list
  int32_t src_count;
  int32_t mrow;       // index of the node's entry in the mask vector (proc for
                      // the graph itself, trial * P + proc for a trial copy)
};

// One source of a sum: kind 0 dry track, 1 U slot, 2 gradient slot
struct SrcRef {
  int32_t kind;
  int32_t slot;
};

struct Stage {
  int type;
  std::vector<int> nodes;       // user ids, in sigma order
  int desc_off = 0;             // offset (elements) in the device descriptor array
};

// FFT plan for the FIR convolutions: N = N1 * N2, x[n1 + N1 n2].
struct FftPlan {
  int N = 0, N1 = 0, N2 = 0, log2N = 0;
};

// Offsets (bytes) of everything carved out of the caller's workspace.
struct WsPlan {
  size_t total = 0;
  size_t desc = 0, srcs = 0, gdesc = 0;
  size_t U = 0, YB = 0, ENV = 0, G = 0;
  size_t ZU = 0, ZH = 0, T1 = 0, T1s = 0, T2 = 0, T3 = 0;
  size_t tw = 0, twd = 0, twdl = 0, twhi = 0, twlo = 0;
  size_t eq_h = 0, eq_dh = 0, eq_cos = 0, eq_HP = 0, eq_dhp = 0, eq_XU = 0;
  size_t dl_tab = 0, dl_h = 0, dl_dh = 0, dl_cos = 0, dl_zp = 0;
  size_t rv_U = 0, rv_fr = 0, rv_h = 0, rv_dh = 0, rv_dM = 0, rv_cs = 0, rv_win = 0, rv_wsum = 0;
  size_t cmp_sum = 0;
  size_t part = 0;           // per (node, block) partial sums
  size_t pgrad = 0;          // per node parameter gradient staging (double)
  size_t ls_tgt = 0, ls_part = 0, ls_norm = 0, ls_tab = 0, ls_aw = 0, ls_win = 0;
  size_t ls_stats = 0;       // double: per (res, combo): |Y|^2, |Y-Yh|^2, sum|dlog|
  size_t lg = 0;             // double per node: E_ybar, E_u
  size_t losses_tmp = 0;
  size_t fin = 0;            // int2 per descriptor: partial blocks, direct parameters
  // pruning trials (mg_forward_trials)
  size_t tr_desc = 0;        // staged copy descriptors of every batch
  size_t tr_keep = 0;        // float [max_trials][P] keep flags
  size_t tr_mask = 0;        // float [max_trials][P] trial masks
  size_t tr_sub = 0;         // int [max_trials][n_desc]: lg row used for each node
  size_t tr_stats = 0;       // double [max_trials][8][16] loss statistics
};

// Host tables of one mg_forward_trials call.
struct TrialPlan {
  std::vector<NodeDesc> desc;          // copies, batch by batch, stage-major inside a batch
  std::vector<SrcRef> srcs;            // sources of the copies' sums
  std::vector<float> keep;             // [B][P]
  std::vector<int32_t> sub;            // [B][n_desc]
  struct Batch {
    int t0, t1;                        // trials [t0, t1)
    int d0;                            // first copy in desc
    std::vector<int> stage_off, stage_n;  // per stage: copy range inside the batch
    std::vector<int> out_slot;         // per trial: U slot of its mix
  };
  std::vector<Batch> batches;
};

// Optional timing of one kernel class (measurement only): HIP events are
// recorded on the caller's stream around every launch of that class.
struct Profiler {
  std::string cls;                       // empty: disabled
  std::vector<hipEvent_t> ev;            // pool of start/stop pairs
  int used = 0;                          // events used since the last read
  const char* cur = nullptr;             // class of the innermost open scope
  bool overflow = false;                 // launches went untimed (pool full)
  double bytes = 0.0;                    // algorithmic bytes of the timed launches
  int64_t launches = 0;
};

struct LossRes {
  int nfft, hop, frames;
  size_t tgt_off, part_off, tab_off, aw_off, win_off;  // byte offsets in ws
  int n_tab;                                           // CSR entries
};

}  // namespace mg

struct mg_graph {
  // user graph
  int n_nodes = 0;
  std::vector<int> type, track;
  std::vector<std::vector<int>> preds, succs;
  int n_tracks = 0, track_ch = 1;
  mg_config cfg{};
  // schedule and layout
  std::vector<mg::Stage> stages;
  std::vector<int> order, pos;            // sigma: position -> node, node -> position
  std::vector<int> stage_of, proc_idx, type_row;
  std::vector<int64_t> param_off;
  int type_count[mg::NTYPES] = {0};
  int type_np[mg::NTYPES] = {0};
  int64_t type_off[mg::NTYPES] = {0};
  int n_proc = 0;
  int64_t n_theta = 0;
  int output_node = -1;
  // slots
  std::vector<int> uslot;                 // node -> U slot (-1 for inputs)
  std::vector<int> pw_run;                // stage s starts a fused chain of pw_run[s] >= 2
                                          // pointwise stages (0: not fused)
  int n_uslots = 0;
  std::vector<int> gslot, ginslot;        // node -> gradient slot of dL/dy, dL/du
  int n_gslots = 0;
  std::vector<int> fanout_sum;            // nodes whose dL/dy is a sum of contributions
  // device descriptor tables (host copies)
  std::vector<mg::NodeDesc> desc;
  std::vector<mg::SrcRef> srcs;
  std::vector<mg::SrcRef> gsrcs;          // backward fan-out sums
  std::vector<mg::NodeDesc> gdesc;        // one per fan-out node: gout = its dL/dy slot,
                                          // sources in gsrcs (offset by srcs.size())
  std::vector<int> gdesc_off;             // per stage: first gdesc entry (size stages + 1)
  mg::FftPlan fft;
  std::vector<mg::LossRes> lres;
  int max_conv_stage = 0, max_stage = 0;
  int nf_rev = 0;                         // reverb STFT frames
  int64_t dl_len = 0;                     // delay compact FIR length
  int dyn_chunks = 0;
  int part_blocks = 0;                    // blocks per node for partial sums
  // bound workspace
  mg::WsPlan ws;
  char* base = nullptr;
  size_t ws_bytes = 0;
  int mode = 0;
  bool ready = false;
  bool have_forward = false;
  bool have_cache = false;                // node outputs of the last forward are in U
  // bound by mg_setup_static: the device whose static scratch holds the
  // workspace (-1: a caller-owned workspace) and the binding's generation
  int static_dev = -1;
  uint64_t static_gen = 0;
  // pruning trials
  int trial_slots = 0;                    // U slots reserved for copies
  int trial_desc_cap = 0;                 // staged copy descriptors
  int trial_src_cap = 0;                  // staged copy sources
  int n_src_base = 0;                     // srcs + gsrcs of the graph itself
  mg::TrialPlan tplan;
  hipEvent_t trial_ev = nullptr;          // upload of tplan done
  bool trial_ev_pending = false;
  // parameter-gradient work of the backward runs on a second stream that
  // forks from and joins the caller's stream through events
  hipStream_t side = nullptr;
  std::vector<hipEvent_t> sev;
  mg::Profiler prof;
  // last forward's inputs (for backward)
  const float* f_dry = nullptr;
  const float* f_theta = nullptr;
  const float* f_wet = nullptr;
  const float* f_mask = nullptr;
};
