// Host-side graph compiler of the mixgraph library.
//
// Validates a processing graph (Sec. 1.1), builds a node subset sequence that
// is a partition, causal and homogeneous (Sec. 4.1), chooses the type
// schedule (Sec. 4.2: the console order walk and the greedy rule, whichever
// is shorter), reorders nodes so that every stage's nodes, parameter rows and
// outputs are contiguous (Alg. 1 OptimizeNodeOrder / Reorder), and assigns the
// read/write slots (Alg. 1 GetReadWriteIndex).  No device code here.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <queue>
#include <string>

#include "mg_internal.h"

using namespace mg;

namespace mg {
thread_local std::string g_err;
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
}  // namespace mg

extern "C" const char* mg_last_error(void) { return mg::g_err.c_str(); }

namespace {

// chain order used by the console walk and as the greedy tie-break
const int kCycle[] = {MG_EQ, MG_COMP, MG_GATE, MG_DIST, MG_IMAGER, MG_GAINPAN, MG_DELAY, MG_REVERB, MG_MIX};
constexpr int kCycleLen = 9;

int params_of(int t, const mg_config& c) {
  switch (t) {
    case MG_GAINPAN: return 2;
    case MG_IMAGER: return 1;
    case MG_DIST: return 2;
    case MG_EQ: return (c.eq_taps + 1) / 2;
    case MG_COMP: return c.comp_mode == 1 ? 5 : 4;
    case MG_GATE: return 4;
    case MG_DELAY: return 2 * c.delay_taps * (2 + (c.delay_fir_taps + 1) / 2);
    case MG_REVERB: return 2 * 2 * (c.reverb_nfft / 2);
    default: return 0;
  }
}

// Returns the stage list (types and nodes) for one scheduling rule.
std::vector<Stage> schedule(const mg_graph& g, bool greedy) {
  std::vector<Stage> st;
  std::vector<int> left(g.n_nodes, 0);
  std::vector<char> done(g.n_nodes, 0);
  Stage s0;
  s0.type = MG_IN;
  for (int v = 0; v < g.n_nodes; ++v) {
    left[v] = (int)g.preds[v].size();
    if (g.type[v] == MG_IN) s0.nodes.push_back(v);
  }
  st.push_back(s0);
  int remaining = g.n_nodes;
  auto finish = [&](const std::vector<int>& nodes) {
    for (int v : nodes) {
      done[v] = 1;
      --remaining;
      for (int d : g.succs[v]) --left[d];
    }
  };
  finish(s0.nodes);
  int cyc = 0;
  while (remaining > 0) {
    std::vector<int> ready[NTYPES];
    for (int v = 0; v < g.n_nodes; ++v)
      if (!done[v] && left[v] == 0) ready[g.type[v]].push_back(v);
    int pick = -1;
    if (!ready[MG_OUT].empty()) {
      bool only_out = true;
      for (int t = 0; t < NTYPES; ++t)
        if (t != MG_OUT && !ready[t].empty()) only_out = false;
      if (only_out) pick = MG_OUT;
    }
    if (pick < 0) {
      if (greedy) {
        size_t best = 0;
        for (int i = 0; i < kCycleLen; ++i) {
          int t = kCycle[i];
          if (ready[t].size() > best) {
            best = ready[t].size();
            pick = t;
          }
        }
      } else {
        for (int i = 0; i < kCycleLen; ++i) {
          int t = kCycle[(cyc + i) % kCycleLen];
          if (!ready[t].empty()) {
            pick = t;
            cyc = (cyc + i + 1) % kCycleLen;
            break;
          }
        }
      }
    }
    if (pick < 0) break;  // cannot happen for a validated DAG
    Stage s;
    s.type = pick;
    s.nodes = ready[pick];
    finish(s.nodes);
    st.push_back(s);
  }
  return st;
}

// Beam search over type strings (Sec. 4.2: the search tree of the shortest
// node subset sequence grows exponentially; a beam keeps it bounded).  A
// state is the set of processed nodes after some stages; a step takes one
// type and processes every computable node of it (the maximal subset).
// States of equal depth are ranked by processed nodes (more first), then by
// their type string; duplicates (the same processed set) are dropped; the
// first depth at which a state is complete gives the schedule.
std::vector<Stage> beam_schedule(const mg_graph& g, int width) {
  struct State {
    std::vector<char> done;
    int n_done = 0;
    std::vector<Stage> st;
    std::string key;   // type string, for a deterministic order
  };
  auto ready_of = [&](const std::vector<char>& done, std::vector<int>* ready) {
    for (int v = 0; v < g.n_nodes; ++v) {
      if (done[v]) continue;
      bool ok = true;
      for (int p : g.preds[v])
        if (!done[p]) ok = false;
      if (ok) ready[g.type[v]].push_back(v);
    }
  };
  State s0;
  s0.done.assign(g.n_nodes, 0);
  Stage in;
  in.type = MG_IN;
  for (int v = 0; v < g.n_nodes; ++v)
    if (g.type[v] == MG_IN) {
      in.nodes.push_back(v);
      s0.done[v] = 1;
      ++s0.n_done;
    }
  s0.st.push_back(in);
  s0.key = "i";
  std::vector<State> beam{s0};
  while (true) {
    for (const State& s : beam)
      if (s.n_done == g.n_nodes) return s.st;
    std::vector<State> next;
    for (const State& s : beam) {
      std::vector<int> ready[NTYPES];
      ready_of(s.done, ready);
      bool other = false;
      for (int t = 0; t < NTYPES; ++t)
        if (t != MG_OUT && !ready[t].empty()) other = true;
      for (int t = 0; t < NTYPES; ++t) {
        if (ready[t].empty() || (t == MG_OUT && other)) continue;  // the output stage comes last
        State c = s;
        Stage st;
        st.type = t;
        st.nodes = ready[t];
        for (int v : st.nodes) c.done[v] = 1;
        c.n_done += (int)st.nodes.size();
        c.st.push_back(st);
        c.key += type_char(t);
        next.push_back(std::move(c));
      }
    }
    if (next.empty()) return {};  // cannot happen for a validated DAG
    std::stable_sort(next.begin(), next.end(), [](const State& a, const State& b) {
      return a.n_done > b.n_done || (a.n_done == b.n_done && a.key < b.key);
    });
    std::vector<State> kept;
    for (State& c : next) {
      bool dup = false;
      for (const State& k : kept)
        if (k.n_done == c.n_done && k.done == c.done) dup = true;
      if (!dup) kept.push_back(std::move(c));
      if ((int)kept.size() >= width) break;
    }
    beam = std::move(kept);
  }
}

int64_t next_pow2(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

}  // namespace

namespace mg {

// Build schedule, layout and slots of a validated graph.
int compile(mg_graph& g) {
  const mg_config& c = g.cfg;
  const int rule = c.schedule_rule;
  const int width = c.beam_width > 0 ? c.beam_width : 8;
  if (rule < 0 || rule > 3) return fail(MG_ERR_INVALID_ARG, "schedule_rule must be 0..3");
  if (rule == 1) g.stages = schedule(g, false);
  else if (rule == 2) g.stages = schedule(g, true);
  else if (rule == 3) g.stages = beam_schedule(g, width);
  else {
    // the shortest of the three; ties keep the earlier rule
    g.stages = schedule(g, false);
    auto b = schedule(g, true);
    if (b.size() < g.stages.size()) g.stages = b;
    auto m = beam_schedule(g, width);
    if (!m.empty() && m.size() < g.stages.size()) g.stages = m;
  }
  // sigma: stage by stage, ascending node id inside a stage
  g.order.clear();
  g.pos.assign(g.n_nodes, -1);
  g.stage_of.assign(g.n_nodes, -1);
  for (size_t s = 0; s < g.stages.size(); ++s) {
    std::sort(g.stages[s].nodes.begin(), g.stages[s].nodes.end());
    for (int v : g.stages[s].nodes) {
      g.pos[v] = (int)g.order.size();
      g.order.push_back(v);
      g.stage_of[v] = (int)s;
    }
  }
  if ((int)g.order.size() != g.n_nodes) return fail(MG_ERR_GRAPH, "schedule does not cover every node");
  // parameter layout
  g.proc_idx.assign(g.n_nodes, -1);
  g.type_row.assign(g.n_nodes, -1);
  g.param_off.assign(g.n_nodes, -1);
  std::memset(g.type_count, 0, sizeof(g.type_count));
  for (int v : g.order) g.type_row[v] = g.type_count[g.type[v]]++;
  int64_t off = 0;
  for (int t : kProcOrder) {
    g.type_np[t] = params_of(t, c);
    g.type_off[t] = off;
    off += (int64_t)g.type_count[t] * g.type_np[t];
  }
  g.n_theta = off;
  g.n_proc = 0;
  for (int v : g.order)
    if (is_proc(g.type[v])) {
      g.proc_idx[v] = g.n_proc++;
      g.param_off[v] = g.type_off[g.type[v]] + (int64_t)g.type_row[v] * g.type_np[g.type[v]];
    }
  // output slots (U): every non-input node in sigma order, then input-sum
  // slots for processors with several predecessors
  g.uslot.assign(g.n_nodes, -1);
  g.n_uslots = 0;
  for (int v : g.order)
    if (g.type[v] != MG_IN) g.uslot[v] = g.n_uslots++;
  std::vector<int> insum(g.n_nodes, -1);
  for (int v : g.order)
    if (is_proc(g.type[v]) && g.preds[v].size() > 1) insum[v] = g.n_uslots++;
  // gradient slots.  dL/dy of a node with one successor aliases the
  // successor's dL/du (processor) or dL/dy (m / o); fan-out nodes own a slot
  // filled by a sum of their successors' contributions.
  g.gslot.assign(g.n_nodes, -1);
  g.ginslot.assign(g.n_nodes, -1);
  g.n_gslots = 0;
  g.fanout_sum.clear();
  for (int i = g.n_nodes - 1; i >= 0; --i) {
    int v = g.order[i];
    int t = g.type[v];
    if (t == MG_OUT) {
      g.gslot[v] = g.n_gslots++;
      continue;
    }
    if (t == MG_IN) continue;
    if (g.succs[v].size() == 1) {
      int s = g.succs[v][0];
      if (g.type[s] == MG_MIX || g.type[s] == MG_OUT) g.gslot[v] = g.gslot[s];
      else {
        if (g.ginslot[s] < 0) g.ginslot[s] = g.n_gslots++;
        g.gslot[v] = g.ginslot[s];
      }
    } else {
      g.gslot[v] = g.n_gslots++;
      g.fanout_sum.push_back(v);
    }
  }
  // processors whose input is a multi-predecessor sum or whose single
  // predecessor has fan-out need their own dL/du slot
  for (int v : g.order) {
    if (!is_proc(g.type[v])) continue;
    bool need = false;
    for (int p : g.preds[v])
      if (g.type[p] != MG_IN) need = true;
    if (need && g.ginslot[v] < 0) g.ginslot[v] = g.n_gslots++;
  }
  // descriptors
  g.desc.clear();
  g.srcs.clear();
  g.gsrcs.clear();
  g.max_conv_stage = 0;
  g.max_stage = 0;
  for (size_t s = 1; s < g.stages.size(); ++s) {
    Stage& S = g.stages[s];
    S.desc_off = (int)g.desc.size();
    g.max_stage = std::max(g.max_stage, (int)S.nodes.size());
    if (S.type == MG_DELAY || S.type == MG_REVERB)
      g.max_conv_stage = std::max(g.max_conv_stage, (int)S.nodes.size());
    for (int v : S.nodes) {
      NodeDesc d{};
      d.node = v;
      d.proc = g.proc_idx[v];
      d.mrow = d.proc;
      d.out_slot = g.uslot[v];
      d.aux = g.type_row[v];
      d.theta_off = g.param_off[v] < 0 ? 0 : g.param_off[v];
      d.gout = g.gslot[v];
      d.gin = -1;
      d.src_begin = (int)g.srcs.size();
      d.src_count = 0;
      bool sum_node = (S.type == MG_MIX || S.type == MG_OUT || g.preds[v].size() > 1);
      if (sum_node) {
        std::vector<int> ps = g.preds[v];
        std::sort(ps.begin(), ps.end());
        for (int p : ps) {
          SrcRef r;
          if (g.type[p] == MG_IN) {
            r.kind = 0;
            r.slot = g.track[p];
          } else {
            r.kind = 1;
            r.slot = g.uslot[p];
          }
          g.srcs.push_back(r);
        }
        d.src_count = (int)ps.size();
      }
      if (is_proc(S.type)) {
        if (g.preds[v].size() > 1) {
          d.in_kind = 1;
          d.in_slot = insum[v];
        } else {
          int p = g.preds[v][0];
          if (g.type[p] == MG_IN) {
            d.in_kind = 0;
            d.in_slot = g.track[p];
          } else {
            d.in_kind = 1;
            d.in_slot = g.uslot[p];
          }
        }
        d.gin = g.ginslot[v];
      }
      g.desc.push_back(d);
    }
  }
  // backward fan-out sums: a node with several consumers gets dL/dy as the
  // sum of what each consumer passes back (its dL/du, or the dL/dy of a mix);
  // one sum descriptor per such node, grouped by stage so the backward runs
  // them before the stage's own adjoints
  g.gdesc.clear();
  g.gdesc_off.assign(g.stages.size() + 1, 0);
  std::vector<char> fan(g.n_nodes, 0);
  for (int v : g.fanout_sum) fan[v] = 1;
  for (size_t s = 0; s < g.stages.size(); ++s) {
    g.gdesc_off[s] = (int)g.gdesc.size();
    for (int v : g.stages[s].nodes) {
      if (!fan[v] || g.type[v] == MG_IN) continue;
      NodeDesc d{};
      d.node = v;
      d.proc = -1;
      d.mrow = -1;
      d.gout = g.gslot[v];
      d.gin = -1;
      d.src_begin = (int)(g.srcs.size() + g.gsrcs.size());
      std::vector<int> ss = g.succs[v];
      std::sort(ss.begin(), ss.end());
      for (int s2 : ss) {
        SrcRef r;
        r.kind = 2;
        r.slot = (g.type[s2] == MG_MIX || g.type[s2] == MG_OUT) ? g.gslot[s2] : g.ginslot[s2];
        g.gsrcs.push_back(r);
      }
      d.src_count = (int)ss.size();
      g.gdesc.push_back(d);
    }
  }
  g.gdesc_off[g.stages.size()] = (int)g.gdesc.size();
  // FFT plan for the FIR convolutions
  int64_t ext = 0;
  bool any_conv = false;
  for (int v = 0; v < g.n_nodes; ++v) {
    int t = g.type[v];
    if (t == MG_DELAY)
      ext = std::max<int64_t>(ext, (int64_t)c.delay_taps * c.delay_range + (c.delay_fir_taps - 1) / 2), any_conv = true;
    if (t == MG_REVERB) ext = std::max<int64_t>(ext, c.reverb_length), any_conv = true;
  }
  g.fft = FftPlan{};
  if (any_conv) {
    const int64_t need = c.length + ext;
    int64_t N = std::max<int64_t>(next_pow2(need), 8192);
    int64_t N2 = std::min<int64_t>(std::max<int64_t>(N / 2048, 16), 1024);
    int64_t N1 = N / N2;
    // rows of 3072 points (3 x 1024) where N = 3072 N2 suffices and is
    // smaller than the power of two (up to a quarter fewer points)
    const int64_t N2r = next_pow2((need + 3071) / 3072);
    if (N2r >= 16 && N2r <= 1024 && 3072 * N2r < N) {
      N = 3072 * N2r;
      N1 = 3072;
      N2 = N2r;
    }
    if (N1 > 4096) return fail(MG_ERR_INVALID_ARG, "signal too long for the FFT engine (N > 2^22)");
    g.fft.N = (int)N;
    g.fft.N1 = (int)N1;
    g.fft.N2 = (int)N2;
    g.fft.log2N = 0;
    while ((1LL << g.fft.log2N) < N) ++g.fft.log2N;
  }
  g.dl_len = (int64_t)c.delay_taps * c.delay_range + c.delay_fir_taps - 1;
  g.nf_rev = c.reverb_hop > 0 ? (c.reverb_length - 1) / c.reverb_hop + 2 : 0;
  // loss resolutions
  g.lres.clear();
  for (int i = 0; i < c.n_loss_ffts; ++i) {
    LossRes r{};
    r.nfft = c.loss_ffts[i];
    r.hop = r.nfft / 4;
    r.frames = (int)(1 + (c.length - c.loss_skip - r.nfft) / r.hop);
    g.lres.push_back(r);
  }
  return MG_OK;
}

int validate_config(const mg_config& c, const std::vector<int>& type) {
  bool has[NTYPES] = {false};
  for (int t : type) has[t] = true;
  if (c.length < 64) return fail(MG_ERR_INVALID_ARG, "length must be >= 64");
  if ((has[MG_COMP] || has[MG_GATE]) && c.length > (int64_t)4096 * 4096)
    return fail(MG_ERR_INVALID_ARG, "compressor/noisegate signals are limited to 4096 chunks of 4096 samples");
  if (c.sample_rate <= 0) return fail(MG_ERR_INVALID_ARG, "sample_rate must be > 0");
  if (has[MG_EQ] && (c.eq_taps < 3 || (c.eq_taps & 1) == 0 || c.eq_taps > 4095))
    return fail(MG_ERR_INVALID_ARG, "eq_taps must be odd in [3, 4095]");
  if (has[MG_COMP] && c.comp_mode != 0 && c.comp_mode != 1)
    return fail(MG_ERR_INVALID_ARG, "comp_mode must be 0 or 1");
  if (has[MG_DELAY]) {
    if (c.delay_taps < 1 || c.delay_taps > 64 || c.delay_range < 2 || c.delay_fir_taps < 1 ||
        (c.delay_fir_taps & 1) == 0 || c.delay_fir_taps > 255)
      return fail(MG_ERR_INVALID_ARG, "bad delay sizes");
  }
  if (has[MG_REVERB]) {
    if (c.reverb_nfft != 384 || c.reverb_hop != 192 || c.reverb_length < 2)
      return fail(MG_ERR_INVALID_ARG, "reverb STFT must be 384/192 and length >= 2");
  }
  if (c.n_loss_ffts < 1 || c.n_loss_ffts > 8) return fail(MG_ERR_INVALID_ARG, "1..8 loss resolutions");
  for (int i = 0; i < c.n_loss_ffts; ++i) {
    int n = c.loss_ffts[i];
    if (n < 256 || n > 4096 || (n & (n - 1))) return fail(MG_ERR_INVALID_ARG, "loss FFT sizes must be powers of two in [256, 4096]");
    if (c.length - c.loss_skip < n) return fail(MG_ERR_INVALID_ARG, "signal shorter than a loss frame");
  }
  if (c.n_mels < 1 || c.n_mels > 128) return fail(MG_ERR_INVALID_ARG, "n_mels must be in [1, 128]");
  if (c.loss_skip < 0) return fail(MG_ERR_INVALID_ARG, "loss_skip must be >= 0");
  if (c.max_trials < 0 || c.max_trials > 4096) return fail(MG_ERR_INVALID_ARG, "max_trials must be in [0, 4096]");
  if (c.trial_slots < 0) return fail(MG_ERR_INVALID_ARG, "trial_slots must be >= 0");
  return MG_OK;
}

int build_graph(int32_t n_nodes, const int32_t* types, int32_t n_edges, const int32_t* edges,
                const int32_t* input_track, int32_t n_tracks, int32_t track_channels,
                const mg_config* cfg, mg_graph** out) {
  if (!out) return fail(MG_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n_nodes < 2 || !types || !cfg || (n_edges > 0 && !edges) || !input_track)
    return fail(MG_ERR_INVALID_ARG, "bad graph arguments");
  if (track_channels != 1 && track_channels != 2) return fail(MG_ERR_INVALID_ARG, "track_channels must be 1 or 2");
  mg_graph* g = new mg_graph();
  g->n_nodes = n_nodes;
  g->cfg = *cfg;
  g->n_tracks = n_tracks;
  g->track_ch = track_channels;
  g->type.assign(types, types + n_nodes);
  g->track.assign(n_nodes, -1);
  g->preds.assign(n_nodes, {});
  g->succs.assign(n_nodes, {});
  auto bad = [&](int code, const std::string& m) {
    delete g;
    return fail(code, m);
  };
  int n_out = 0;
  for (int v = 0; v < n_nodes; ++v) {
    int t = g->type[v];
    if (t < 0 || t >= NTYPES) return bad(MG_ERR_GRAPH, "unknown node type at node " + std::to_string(v));
    if (t == MG_OUT) {
      ++n_out;
      g->output_node = v;
    }
    if (t == MG_IN) {
      int k = input_track[v];
      if (k < 0 || k >= n_tracks) return bad(MG_ERR_GRAPH, "input node with bad track index");
      g->track[v] = k;
    }
  }
  if (n_out != 1) return bad(MG_ERR_GRAPH, "graph must have exactly one output node");
  for (int e = 0; e < n_edges; ++e) {
    int s = edges[e], d = edges[n_edges + e];
    if (s < 0 || s >= n_nodes || d < 0 || d >= n_nodes || s == d) return bad(MG_ERR_GRAPH, "bad edge");
    g->succs[s].push_back(d);
    g->preds[d].push_back(s);
  }
  for (int v = 0; v < n_nodes; ++v) {
    int t = g->type[v];
    if (t == MG_IN && !g->preds[v].empty()) return bad(MG_ERR_GRAPH, "input node with predecessors");
    if (t != MG_IN && g->preds[v].empty()) return bad(MG_ERR_GRAPH, "node without inputs");
    if (t == MG_OUT && !g->succs[v].empty()) return bad(MG_ERR_GRAPH, "output node with successors");
    if (t != MG_OUT && g->succs[v].empty()) return bad(MG_ERR_GRAPH, "node cannot reach the output");
  }
  // acyclic (Kahn)
  {
    std::vector<int> indeg(n_nodes);
    std::queue<int> q;
    for (int v = 0; v < n_nodes; ++v) {
      indeg[v] = (int)g->preds[v].size();
      if (!indeg[v]) q.push(v);
    }
    int seen = 0;
    while (!q.empty()) {
      int v = q.front();
      q.pop();
      ++seen;
      for (int d : g->succs[v])
        if (--indeg[d] == 0) q.push(d);
    }
    if (seen != n_nodes) return bad(MG_ERR_GRAPH, "graph has a cycle");
  }
  int rc = validate_config(g->cfg, g->type);
  if (rc) {
    delete g;
    return rc;
  }
  rc = compile(*g);
  if (rc) {
    delete g;
    return rc;
  }
  *out = g;
  return MG_OK;
}

}  // namespace mg

extern "C" int mg_graph_create(int32_t n_nodes, const int32_t* types, int32_t n_edges, const int32_t* edges,
                               const int32_t* input_track, int32_t n_tracks, int32_t track_channels,
                               const mg_config* cfg, mg_graph** out) {
  return mg::build_graph(n_nodes, types, n_edges, edges, input_track, n_tracks, track_channels, cfg, out);
}

extern "C" int mg_graph_destroy(mg_graph* g) {
  if (g) {
    for (auto& e : g->prof.ev) (void)hipEventDestroy(e);
    if (g->trial_ev) (void)hipEventDestroy(g->trial_ev);
    for (auto& e : g->sev) (void)hipEventDestroy(e);
    if (g->side) (void)hipStreamDestroy(g->side);
  }
  delete g;
  return MG_OK;
}

extern "C" int mg_graph_info(const mg_graph* g, mg_info* out) {
  if (!g || !out) return fail(MG_ERR_INVALID_ARG, "NULL argument");
  out->n_nodes = g->n_nodes;
  out->n_processors = g->n_proc;
  out->n_stages = (int32_t)g->stages.size();
  out->fft_size = g->fft.N;
  out->n_theta = g->n_theta;
  out->n_reverbs = g->type_count[MG_REVERB];
  out->n_losses = 7;
  return MG_OK;
}

extern "C" int mg_graph_layout(const mg_graph* g, int64_t* param_offset, int32_t* proc_index, int32_t* stage,
                               int32_t* type_row, char* schedule) {
  if (!g) return fail(MG_ERR_INVALID_ARG, "NULL graph");
  for (int v = 0; v < g->n_nodes; ++v) {
    if (param_offset) param_offset[v] = g->param_off[v];
    if (proc_index) proc_index[v] = g->proc_idx[v];
    if (stage) stage[v] = g->stage_of[v];
    if (type_row) type_row[v] = g->type_row[v];
  }
  if (schedule) {
    size_t i = 0;
    for (; i < g->stages.size(); ++i) schedule[i] = type_char(g->stages[i].type);
    schedule[i] = 0;
  }
  return MG_OK;
}

extern "C" int mg_graph_prune(const mg_graph* g, const uint8_t* keep, mg_graph** out, int32_t* old_to_new) {
  if (!g || !keep || !out) return fail(MG_ERR_INVALID_ARG, "NULL argument");
  // removed processors are bypassed: their predecessors feed their successors
  std::vector<char> drop(g->n_nodes, 0);
  for (int v = 0; v < g->n_nodes; ++v)
    if (g->proc_idx[v] >= 0 && !keep[g->proc_idx[v]]) drop[v] = 1;
  std::vector<int> map(g->n_nodes, -1);
  int n = 0;
  for (int v = 0; v < g->n_nodes; ++v)
    if (!drop[v]) map[v] = n++;
  // resolve each kept node's predecessors through dropped nodes
  std::vector<std::pair<int, int>> edges;
  for (int v = 0; v < g->n_nodes; ++v) {
    if (drop[v]) continue;
    std::vector<int> stack(g->preds[v].begin(), g->preds[v].end());
    std::vector<int> srcs;
    while (!stack.empty()) {
      int p = stack.back();
      stack.pop_back();
      if (drop[p]) {
        for (int q : g->preds[p]) stack.push_back(q);
      } else {
        srcs.push_back(p);
      }
    }
    std::sort(srcs.begin(), srcs.end());
    srcs.erase(std::unique(srcs.begin(), srcs.end()), srcs.end());
    for (int p : srcs) edges.push_back({map[p], map[v]});
  }
  std::vector<int32_t> types(n), tracks(n, -1), ev(2 * edges.size());
  for (int v = 0; v < g->n_nodes; ++v)
    if (map[v] >= 0) {
      types[map[v]] = g->type[v];
      tracks[map[v]] = g->track[v];
    }
  for (size_t e = 0; e < edges.size(); ++e) {
    ev[e] = edges[e].first;
    ev[edges.size() + e] = edges[e].second;
  }
  int rc = mg::build_graph(n, types.data(), (int32_t)edges.size(), ev.data(), tracks.data(), g->n_tracks,
                           g->track_ch, &g->cfg, out);
  if (rc == MG_OK && old_to_new)
    for (int v = 0; v < g->n_nodes; ++v) old_to_new[v] = map[v];
  return rc;
}

extern "C" int mg_remap_params(const mg_graph* g, const mg_graph* pruned, const int32_t* old_to_new,
                               const float* src_theta, float* dst_theta, const float* src_wet, float* dst_wet,
                               void* stream) {
  if (!g || !pruned || !old_to_new) return fail(MG_ERR_INVALID_ARG, "NULL argument");
  if ((src_theta == nullptr) != (dst_theta == nullptr) || (src_wet == nullptr) != (dst_wet == nullptr))
    return fail(MG_ERR_INVALID_ARG, "source and destination must both be given or both be NULL");
  hipStream_t st = (hipStream_t)stream;
  for (int v = 0; v < g->n_nodes; ++v) {
    const int u = old_to_new[v];
    if (u < 0 || g->proc_idx[v] < 0) continue;
    if (u >= pruned->n_nodes || pruned->type[u] != g->type[v] || pruned->proc_idx[u] < 0)
      return fail(MG_ERR_GRAPH, "old_to_new does not match the pruned graph");
    hipError_t e = hipSuccess;
    if (src_theta) {
      const int64_t len = g->type_np[g->type[v]];
      if (len > 0)
        e = hipMemcpyAsync(dst_theta + pruned->param_off[u], src_theta + g->param_off[v], (size_t)len * 4,
                           hipMemcpyDeviceToDevice, st);
    }
    if (e == hipSuccess && src_wet)
      e = hipMemcpyAsync(dst_wet + pruned->proc_idx[u], src_wet + g->proc_idx[v], 4, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return fail(MG_ERR_HIP, std::string("remap copy: ") + hipGetErrorString(e));
  }
  return MG_OK;
}
