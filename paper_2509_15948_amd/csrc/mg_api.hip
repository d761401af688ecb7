// C-ABI entry points that touch the device: workspace planning and binding,
// the forward pass (Alg. 1 stage loop, then the loss of Sec. 5.1), the
// backward pass (stages in reverse with hand-written adjoints), the masked
// pruning evaluation (Alg. 2 Evaluate) and Adam.  All work is enqueued on
// the caller's stream; nothing here allocates device memory.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "mg_device.h"
#include "mg_kernels.h"

namespace mg {
int fail(int code, const std::string& msg);
size_t loss_table_bytes(int N, int nm, int fs, std::vector<char>* blob);

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

static int hip_check(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return fail(MG_ERR_OOM, std::string(what) + ": " + hipGetErrorString(e));
  if (e != hipSuccess) return fail(MG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return MG_OK;
}

// Carve the workspace.  Returns total bytes; fills g.ws when commit is set.
static size_t plan_ws(mg_graph& g, int mode, bool commit) {
  const mg_config& c = g.cfg;
  const int64_t L = c.length;
  WsPlan w;
  size_t o = 0;
  auto take = [&](size_t& field, size_t bytes) {
    field = o;
    o += align256(bytes);
  };
  const int n_desc = (int)g.desc.size();
  const int n_eq = g.type_count[MG_EQ], n_dl = g.type_count[MG_DELAY], n_rv = g.type_count[MG_REVERB];
  const int n_conv = n_eq + n_dl + n_rv;
  const int n_dyn = g.type_count[MG_COMP] + g.type_count[MG_GATE];
  const int64_t N = g.fft.N;
  const int n_win = n_desc + g.trial_slots;   // descriptors incl. the trial window
  const int P = g.n_proc, Bt = c.max_trials;
  take(w.desc, std::max<size_t>(1, n_win) * sizeof(NodeDesc));
  take(w.srcs, std::max<size_t>(1, g.n_src_base + g.trial_src_cap) * sizeof(SrcRef));
  take(w.gdesc, std::max<size_t>(1, g.gdesc.size()) * sizeof(NodeDesc));
  take(w.losses_tmp, std::max(1, n_desc) * sizeof(int));
  take(w.fin, std::max(1, n_desc) * 8);
  take(w.U, (size_t)(g.n_uslots + g.trial_slots) * 2 * L * 4);
  if (Bt > 0) {
    take(w.tr_desc, (size_t)std::max(1, g.trial_desc_cap) * sizeof(NodeDesc));
    take(w.tr_keep, (size_t)Bt * std::max(1, P) * 4);
    take(w.tr_mask, (size_t)Bt * std::max(1, P) * 4);
    take(w.tr_sub, (size_t)Bt * std::max(1, n_desc) * 4);
    take(w.tr_stats, (size_t)Bt * 128 * 8);
  }
  if (mode) {
    take(w.YB, (size_t)n_conv * 2 * L * 4);
    take(w.ENV, (size_t)n_dyn * L * 4);
    take(w.G, (size_t)g.n_gslots * 2 * L * 4);
  }
  if (N > 0) {
    take(w.ZH, (size_t)(n_dl + n_rv) * N * 8);
    if (mode) take(w.ZU, (size_t)(n_dl + n_rv) * N * 8);
    take(w.T1, (size_t)g.max_conv_stage * N * 8);
    take(w.T1s, (size_t)g.max_conv_stage * N * 8);  // FIR spectra on the side stream
    take(w.T2, (size_t)g.max_conv_stage * N * 8);
    if (mode) {
      // FIR-gradient spectra, one row per node of every long-FIR stage: the
      // side stream reads a stage's rows while later stages write their own
      size_t conv_nodes = 0;
      for (const Stage& S : g.stages)
        if (S.type == MG_DELAY || S.type == MG_REVERB) conv_nodes += S.nodes.size();
      take(w.T3, std::max<size_t>(1, conv_nodes) * N * 8);
    }
    take(w.twhi, (size_t)std::max<int64_t>(1, N / 1024) * 8);
    take(w.twlo, 1024 * 8);
  }
  take(w.tw, MG_TWN * 8);
  take(w.twdl, MG_TWN * 8);
  take(w.twd, MG_TWN * 16);
  if (n_eq) {
    take(w.eq_h, (size_t)n_eq * c.eq_taps * 4);
    take(w.eq_HP, (size_t)n_eq * 8192 * 4);
    if (mode) {
      take(w.eq_dh, (size_t)n_eq * c.eq_taps * 4);
      take(w.eq_dhp, (size_t)n_eq * eq_blocks(&g) * c.eq_taps * 4);
      take(w.eq_XU, (size_t)n_eq * eq_blocks(&g) * 8192 * 8);  // input-window spectra for the backward
    }
    take(w.eq_cos, (size_t)c.eq_taps * 4);
  }
  if (n_dl) {
    take(w.dl_tab, (size_t)n_dl * 2 * c.delay_taps * (1 + c.delay_fir_taps) * 4);
    take(w.dl_h, (size_t)n_dl * 2 * g.dl_len * 4);
    if (mode) {
      take(w.dl_dh, (size_t)n_dl * 2 * g.dl_len * 4);
      take(w.dl_zp, (size_t)n_dl * 2 * c.delay_taps * 8 * 16);  // z partial sums, 8 chunks
    }
    take(w.dl_cos, (size_t)c.delay_fir_taps * 4);
  }
  if (n_rv) {
    take(w.rv_U, (size_t)n_rv * 2 * g.nf_rev * 192 * 8);
    take(w.rv_fr, (size_t)n_rv * 2 * g.nf_rev * 384 * 4);
    take(w.rv_h, (size_t)n_rv * 2 * c.reverb_length * 4);
    if (mode) {
      take(w.rv_dh, (size_t)n_rv * 2 * c.reverb_length * 4);
      take(w.rv_dM, (size_t)n_rv * 2 * g.nf_rev * 192 * 4);
    }
    take(w.rv_cs, 384 * 8);
    take(w.rv_win, 384 * 4);
    take(w.rv_wsum, 192 * 4);
  }
  if (n_dyn) {
    take(w.cmp_sum, (size_t)std::max(1, g.max_stage) * g.dyn_chunks * 4);
  }
  take(w.part, (size_t)std::max(1, n_win) * g.part_blocks * PK * 4);
  take(w.lg, (size_t)std::max(1, n_win) * 2 * 8);
  take(w.ls_stats, 8 * 16 * 8);
  for (auto& r : g.lres) {
    const int FPB = loss_frames_per_block_fwd(r.nfft);  // partial rows: one per forward block
    const int blocks = (r.frames + FPB - 1) / FPB;
    size_t tgt, part, tab;
    take(tgt, (size_t)r.frames * 4 * c.n_mels * 8);
    take(part, (size_t)blocks * 8 * 8);
    take(tab, loss_table_bytes(r.nfft, c.n_mels, c.sample_rate, nullptr));
    if (commit) {
      r.tgt_off = tgt;
      r.part_off = part;
      r.tab_off = tab;
    }
  }
  if (mode) {
    size_t s = 0;
    for (auto& r : g.lres) s += align256((size_t)r.frames * r.nfft * 2 * 4);
    take(w.ls_part, s);
  }
  w.total = o;
  if (commit) g.ws = w;
  return o;
}

// U slots that bypassing processor v costs a trial: every node downstream of
// v, plus an input sum for each downstream processor with several inputs.
static int suffix_slots(const mg_graph& g, int v) {
  std::vector<char> seen(g.n_nodes, 0);
  std::vector<int> stack(g.succs[v].begin(), g.succs[v].end());
  int n = 0;
  while (!stack.empty()) {
    const int u = stack.back();
    stack.pop_back();
    if (seen[u]) continue;
    seen[u] = 1;
    n += 1 + ((is_proc(g.type[u]) && g.preds[u].size() > 1) ? 1 : 0);
    for (int s : g.succs[u]) stack.push_back(s);
  }
  return n;
}

static bool is_pointwise(int t) { return t == MG_GAINPAN || t == MG_IMAGER || t == MG_DIST; }

// stage B continues a pointwise chain of stage A: node j of A feeds node j of
// B and nothing else, B has no other input, and B's dL/du is A's dL/dy
static bool pw_link(const mg_graph& g, const Stage& A, const Stage& B) {
  if (A.nodes.size() != B.nodes.size() || A.nodes.empty()) return false;
  for (size_t j = 0; j < A.nodes.size(); ++j) {
    const int va = A.nodes[j], vb = B.nodes[j];
    const NodeDesc& da = g.desc[A.desc_off + j];
    const NodeDesc& db = g.desc[B.desc_off + j];
    if (g.succs[va].size() != 1 || g.succs[va][0] != vb || g.preds[vb].size() != 1) return false;
    if (db.in_kind != 1 || db.in_slot != da.out_slot || db.src_count != 0 || db.gin != da.gout) return false;
  }
  return true;
}

// maximal runs of up to PW_MAXK linked pointwise stages
static void plan_pointwise_chains(mg_graph& g) {
  const size_t S = g.stages.size();
  g.pw_run.assign(S, 0);
  if (g.cfg.unfused) return;
  for (size_t s = 1; s < S;) {
    const Stage& A = g.stages[s];
    bool ok = is_pointwise(A.type);
    for (size_t j = 0; ok && j < A.nodes.size(); ++j)
      if (g.desc[A.desc_off + j].src_count != 0) ok = false;
    size_t k = ok ? 1 : 0;
    while (ok && s + k < S && k < (size_t)PW_MAXK && is_pointwise(g.stages[s + k].type) &&
           pw_link(g, g.stages[s + k - 1], g.stages[s + k]))
      ++k;
    if (k >= 2) {
      g.pw_run[s] = (int)k;
      s += k;
    } else {
      s += 1;
    }
  }
}

static void finish_compile(mg_graph& g) {
  plan_pointwise_chains(g);
  g.n_src_base = (int)(g.srcs.size() + g.gsrcs.size());
  const int Bt = std::max(0, g.cfg.max_trials);
  if (Bt > 0) {
    int per = 1;
    for (int v = 0; v < g.n_nodes; ++v)
      if (is_proc(g.type[v])) per = std::max(per, suffix_slots(g, v));
    g.trial_slots = g.cfg.trial_slots > 0 ? g.cfg.trial_slots : Bt * per;
    int64_t n_edges = 0;
    for (int v = 0; v < g.n_nodes; ++v) n_edges += (int64_t)g.preds[v].size();
    g.trial_desc_cap = Bt * g.n_nodes;
    g.trial_src_cap = (int)(Bt * n_edges);
  } else {
    g.trial_slots = g.trial_desc_cap = g.trial_src_cap = 0;
  }
  g.dyn_chunks = (int)((g.cfg.length + 4095) / 4096);
  int pb = 128;
  if (g.fft.N > 0) pb = std::max(pb, g.fft.N / COL_TILE);
  pb = std::max(pb, g.dyn_chunks);
  if (g.type_count[MG_EQ] > 0) pb = std::max(pb, eq_blocks(&g));
  g.part_blocks = pb;
}

Ctx make_ctx(const mg_graph* g, hipStream_t st) {
  Ctx c;
  c.g = g;
  c.st = st;
  c.L = g->cfg.length;
  c.C = g->track_ch;
  c.base = g->base;
  c.U = (float*)(g->base + g->ws.U);
  c.G = g->mode ? (float*)(g->base + g->ws.G) : nullptr;
  c.dry = g->f_dry;
  c.theta = g->f_theta;
  c.wet = g->f_wet;
  c.mask = g->f_mask;
  c.desc = (const NodeDesc*)(g->base + g->ws.desc);
  c.srcs = (const SrcRef*)(g->base + g->ws.srcs);
  c.part = (float*)(g->base + g->ws.part);
  c.PB = g->part_blocks;
  c.lg = (double*)(g->base + g->ws.lg);
  c.alpha_g = (float)g->cfg.alpha_g;
  c.alpha_p = (float)g->cfg.alpha_p;
  c.vec4 = (c.L % 4 == 0) && ((uintptr_t)c.dry % 16 == 0);
  return c;
}

// Forward of the nodes [off, off + n) of one stage of type t; hd are the host
// copies of those descriptors.  Trial copies (c.trial) reuse the FIR tables
// and spectra of the last forward and run in pieces no larger than the
// graph's own largest stage, which sizes the per-launch temporaries.
void forward_stage(const Ctx& c, int t, int off, int n, bool keep, const NodeDesc* hd) {
  const mg_graph* g = c.g;
  if (n <= 0) return;
  if (t == MG_MIX || t == MG_OUT) {
    launch_sum(c, off, n, c.srcs, c.U, 0);
    return;
  }
  // processors whose input is a sum of several nodes: gather it first
  bool any_sum = false;
  for (int j = 0; j < n; ++j)
    if (hd[j].src_count > 0) any_sum = true;
  if (any_sum) launch_sum(c, off, n, c.srcs, c.U, 2);
  if (t == MG_GAINPAN || t == MG_IMAGER || t == MG_DIST) {
    launch_pointwise_fwd(c, t, off, n);
  } else if (t == MG_COMP || t == MG_GATE) {
    const int cap = std::max(1, g->max_stage);
    for (int j = 0; j < n; j += cap) dyn_forward(c, t, off + j, std::min(cap, n - j));
  } else if (t == MG_EQ) {
    eq_forward(c, off, n, keep);
  } else if (is_conv(t)) {
    const int cap = std::max(1, g->max_conv_stage);
    for (int j = 0; j < n; j += cap) conv_forward(c, t, off + j, std::min(cap, n - j), keep);
  }
}

// FIR synthesis and FIR spectra of one stage (they depend on theta only)
static void fir_stage(const Ctx& c, int t, int off, int n, float2* T) {
  fir_synth(c, t, off, n);
  if (t == MG_EQ) eq_spectrum(c, off, n);
  else conv_fir_spectrum(c, t, off, n, T);
}

static void run_forward(mg_graph* g, hipStream_t st, bool keep, double* losses, float* mix) {
  Ctx c = make_ctx(g, st);
  c.defer_lg = true;  // one L_g reduction for every FIR stage, after the chain
  const int n_desc = (int)g->desc.size();
  // The FIRs of every EQ/delay/reverb stage depend on theta only: they are
  // synthesised on the side stream, ahead of the chain, and each stage waits
  // for its own FIRs.
  std::vector<int> ready(g->stages.size(), -1);
  const bool side = g->side != nullptr;
  if (side) {
    Ctx cs = c;
    cs.st = g->side;
    hipEventRecord(g->sev[0], st);
    hipStreamWaitEvent(g->side, g->sev[0], 0);
    int ev = 1;
    for (size_t s = 1; s < g->stages.size(); ++s) {
      const Stage& S = g->stages[s];
      if (!is_conv(S.type)) continue;
      fir_stage(cs, S.type, S.desc_off, (int)S.nodes.size(), (float2*)(g->base + g->ws.T1s));
      ready[s] = ev;
      hipEventRecord(g->sev[ev], g->side);
      ev = ev + 1 < (int)g->sev.size() ? ev + 1 : 1;
    }
  }
  for (size_t s = 1; s < g->stages.size(); ++s) {
    const Stage& S = g->stages[s];
    if (g->pw_run[s] >= 2) {
      const int K = g->pw_run[s];
      int types[PW_MAXK], offs[PW_MAXK];
      for (int i = 0; i < K; ++i) {
        types[i] = g->stages[s + i].type;
        offs[i] = g->stages[s + i].desc_off;
      }
      launch_pw_chain_fwd(c, types, offs, K, (int)S.nodes.size());
      s += K - 1;
      continue;
    }
    if (is_conv(S.type)) {
      if (ready[s] >= 0) hipStreamWaitEvent(st, g->sev[ready[s]], 0);
      else fir_stage(c, S.type, S.desc_off, (int)S.nodes.size(), (float2*)(g->base + g->ws.T1));
    }
    forward_stage(c, S.type, S.desc_off, (int)S.nodes.size(), keep, g->desc.data() + S.desc_off);
  }
  const float* yhat = c.U + (int64_t)g->uslot[g->output_node] * 2 * c.L;
  launch_reduce_lg_all(c, n_desc, (const int2*)(g->base + g->ws.fin), (const int*)(g->base + g->ws.losses_tmp));
  loss_forward(c, yhat);
  launch_finalize_losses(c, losses, (const double*)(g->base + g->ws.ls_stats), (int)g->lres.size(), n_desc);
  if (mix) hipMemcpyAsync(mix, yhat, (size_t)2 * c.L * 4, hipMemcpyDeviceToDevice, st);
}

}  // namespace mg

using namespace mg;

extern "C" int mg_workspace_size(const mg_graph* g, int32_t mode, size_t* bytes) {
  if (!g || !bytes || (mode != 0 && mode != 1)) return fail(MG_ERR_INVALID_ARG, "bad arguments");
  mg_graph tmp = *g;
  finish_compile(tmp);
  *bytes = plan_ws(tmp, mode, false);
  return MG_OK;
}

namespace mg {
// Bind a workspace and prepare the graph's device tables (the body of
// mg_setup and of mg_setup_static).  With make_side the graph gets its side
// stream and events (created once); without, every launch of the forward and
// backward stays on the caller's stream and nothing is created.
int bind_workspace(mg_graph* g, void* workspace, size_t workspace_bytes, int32_t mode, const float* reverb_noise,
                   const float* target, hipStream_t st, bool make_side) {
  if (!g || !workspace || !target || (mode != 0 && mode != 1)) return fail(MG_ERR_INVALID_ARG, "bad arguments");
  if (((uintptr_t)workspace) & 255) return fail(MG_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (g->type_count[MG_REVERB] > 0 && !reverb_noise) return fail(MG_ERR_INVALID_ARG, "reverb noise required");
  finish_compile(*g);
  const size_t need = plan_ws(*g, mode, true);
  if (workspace_bytes < need) return fail(MG_ERR_SHAPE, "workspace too small: need " + std::to_string(need));
  g->ready = false;
  g->static_dev = -1;
  g->base = (char*)workspace;
  g->ws_bytes = workspace_bytes;
  g->mode = mode;
  g->have_forward = false;
  g->have_cache = false;
  // descriptor tables
  std::vector<SrcRef> all = g->srcs;
  all.insert(all.end(), g->gsrcs.begin(), g->gsrcs.end());
  std::vector<int> flag(std::max<size_t>(1, g->desc.size()), 0);
  for (size_t j = 0; j < g->desc.size(); ++j) {
    const int t = g->type[g->desc[j].node];
    flag[j] = (t == MG_EQ || t == MG_DELAY || t == MG_REVERB) ? 1 : 0;
  }
  int rc;
  if (!g->desc.empty() &&
      (rc = hip_check(hipMemcpyAsync(g->base + g->ws.desc, g->desc.data(), g->desc.size() * sizeof(NodeDesc),
                                     hipMemcpyHostToDevice, st), "descriptor upload")))
    return rc;
  if (!all.empty() && (rc = hip_check(hipMemcpyAsync(g->base + g->ws.srcs, all.data(), all.size() * sizeof(SrcRef),
                                                     hipMemcpyHostToDevice, st), "source upload")))
    return rc;
  if (!g->gdesc.empty() &&
      (rc = hip_check(hipMemcpyAsync(g->base + g->ws.gdesc, g->gdesc.data(), g->gdesc.size() * sizeof(NodeDesc),
                                     hipMemcpyHostToDevice, st), "fan-out descriptor upload")))
    return rc;
  if ((rc = hip_check(hipMemcpyAsync(g->base + g->ws.losses_tmp, flag.data(), flag.size() * sizeof(int),
                                     hipMemcpyHostToDevice, st), "flag upload")))
    return rc;
  // partial-sum blocks and direct parameter counts of every processor, for
  // the one gradient-finishing launch at the end of the backward
  std::vector<int2> fin(std::max<size_t>(1, g->desc.size()), make_int2(0, 0));
  for (size_t j = 0; j < g->desc.size(); ++j) {
    const int t = g->type[g->desc[j].node];
    if (t == MG_GAINPAN || t == MG_IMAGER || t == MG_DIST) fin[j] = make_int2(128, g->type_np[t]);
    else if (t == MG_COMP || t == MG_GATE)
      fin[j] = make_int2((t == MG_COMP && g->cfg.comp_mode == 1) ? 1 : g->dyn_chunks, g->type_np[t]);
    else if (t == MG_EQ) fin[j] = make_int2(eq_blocks(g), 0);
    else if (is_conv(t)) fin[j] = make_int2(g->fft.N1 / (COL_TILE / g->fft.N2), 0);
  }
  if ((rc = hip_check(hipMemcpyAsync(g->base + g->ws.fin, fin.data(), fin.size() * sizeof(int2), hipMemcpyHostToDevice,
                                     st), "finish table upload")))
    return rc;
  if (make_side && !g->side) {
    if ((rc = hip_check(hipStreamCreateWithFlags(&g->side, hipStreamNonBlocking), "side stream"))) return rc;
    g->sev.resize(64);
    for (auto& e : g->sev)
      if ((rc = hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event create"))) return rc;
  }
  Ctx c = make_ctx(g, st);
  fft_init_tables(c, (float2*)(g->base + g->ws.tw), g->fft.N ? (float2*)(g->base + g->ws.twhi) : nullptr,
                  g->fft.N ? (float2*)(g->base + g->ws.twlo) : nullptr, g->fft.N, st);
  launch_zero(g->base + g->ws.part, (size_t)std::max<size_t>(1, g->desc.size()) * g->part_blocks * PK * 4, st);
  launch_zero(g->base + g->ws.lg, (size_t)std::max<size_t>(1, g->desc.size()) * 16, st);
  fir_setup(c, reverb_noise);
  loss_setup(c, target);
  if ((rc = hip_check(hipStreamSynchronize(st), "setup"))) return rc;
  if ((rc = hip_check(hipGetLastError(), "setup launch"))) return rc;
  g->ready = true;
  if (getenv("MG_PRINT_LAYOUT")) {  // diagnostics: byte offsets of the workspace regions
    const WsPlan& w = g->ws;
    const std::pair<const char*, size_t> r[] = {
        {"desc", w.desc}, {"srcs", w.srcs}, {"U", w.U}, {"YB", w.YB}, {"ENV", w.ENV}, {"G", w.G},
        {"ZH", w.ZH}, {"ZU", w.ZU}, {"T1", w.T1}, {"T2", w.T2}, {"T3", w.T3}, {"twhi", w.twhi},
        {"twlo", w.twlo}, {"tw", w.tw}, {"twd", w.twd}, {"eq_h", w.eq_h}, {"eq_HP", w.eq_HP},
        {"eq_dh", w.eq_dh}, {"eq_dhp", w.eq_dhp}, {"eq_XU", w.eq_XU}, {"eq_cos", w.eq_cos}, {"dl_tab", w.dl_tab},
        {"dl_dh", w.dl_dh}, {"dl_cos", w.dl_cos}, {"rv_U", w.rv_U}, {"rv_fr", w.rv_fr}, {"rv_h", w.rv_h},
        {"rv_dh", w.rv_dh}, {"rv_dM", w.rv_dM}, {"rv_cs", w.rv_cs}, {"rv_win", w.rv_win},
        {"rv_wsum", w.rv_wsum}, {"cmp_sum", w.cmp_sum}, {"part", w.part},
        {"lg", w.lg}, {"ls_stats", w.ls_stats}, {"ls_part", w.ls_part}, {"total", w.total}};
    for (const auto& x : r) fprintf(stderr, "mg layout %s %zu\n", x.first, x.second);
  }
  return MG_OK;
}
}  // namespace mg

extern "C" int mg_footprint(const mg_graph* g, int32_t mode, size_t* workspace, size_t* state) {
  if (!g || !workspace || !state || (mode != 0 && mode != 1)) return fail(MG_ERR_INVALID_ARG, "bad arguments");
  if (int rc = mg_workspace_size(g, mode, workspace)) return rc;
  const size_t L = (size_t)g->cfg.length;
  const size_t f = sizeof(float);
  size_t b = (size_t)g->n_tracks * g->track_ch * L * f;                        // dry tracks
  b += (size_t)std::max(1, g->type_count[MG_REVERB]) * 2 * std::max(1, g->cfg.reverb_length) * f;  // noise
  b += 2 * 2 * L * f;                                                          // target, mix
  b += 4 * ((size_t)g->n_theta + (size_t)g->n_proc) * f;                       // values, grads, 2 moments
  b += 7 * sizeof(double) * (1 + (size_t)std::max(0, g->cfg.max_trials));      // loss records
  *state = b;
  return MG_OK;
}

// The side stream takes the FIR synthesis, FIR spectra and parameter-gradient
// kernels off the chain.  That pays while the chain's kernels leave the GPU
// partly idle (441 000 samples, the 16-track console: 2.357 ms per step with
// it, 2.522 without); once every kernel fills the GPU the overlap only slows
// the chain (2 880 000 samples, the 64-track console: 44.40 ms with, 44.02
// without; results bit-identical either way).
constexpr int64_t SIDE_STREAM_MAX_L = (int64_t)1 << 21;

extern "C" int mg_setup(mg_graph* g, void* workspace, size_t workspace_bytes, int32_t mode,
                        const float* reverb_noise, const float* target, void* stream) {
  const bool side = !g || g->cfg.length < SIDE_STREAM_MAX_L;
  return bind_workspace(g, workspace, workspace_bytes, mode, reverb_noise, target, (hipStream_t)stream, side);
}

extern "C" int mg_forward(mg_graph* g, const float* dry, const float* theta, const float* wet, const float* mask,
                          float* mix, double* losses, void* stream) {
  if (!g || !dry || !wet || !losses || (!theta && g->n_theta > 0)) return fail(MG_ERR_INVALID_ARG, "NULL argument");
  if (!g->ready) return fail(MG_ERR_STATE, "mg_setup has not been called");
  if (int rc = check_binding(g)) return rc;
  g->f_dry = dry;
  g->f_theta = theta;
  g->f_wet = wet;
  g->f_mask = mask;
  run_forward(g, (hipStream_t)stream, g->mode == 1, losses, mix);
  int rc = hip_check(hipGetLastError(), "forward launch");
  if (rc) return rc;
  g->have_forward = (g->mode == 1);
  g->have_cache = true;
  return MG_OK;
}

extern "C" int mg_forward_masked(mg_graph* g, const float* dry, const float* theta, const float* wet,
                                 const float* masks, int32_t B, double* losses, void* stream) {
  if (!g || !dry || !wet || !losses || !masks || B < 1) return fail(MG_ERR_INVALID_ARG, "bad arguments");
  if (!g->ready) return fail(MG_ERR_STATE, "mg_setup has not been called");
  if (int rc = check_binding(g)) return rc;
  g->f_dry = dry;
  g->f_theta = theta;
  g->f_wet = wet;
  for (int b = 0; b < B; ++b) {
    g->f_mask = masks + (int64_t)b * g->n_proc;
    run_forward(g, (hipStream_t)stream, false, losses + (int64_t)b * 7, nullptr);
  }
  g->have_forward = false;
  g->have_cache = false;
  return hip_check(hipGetLastError(), "masked forward launch");
}

extern "C" int mg_backward(mg_graph* g, float* grad_theta, float* grad_wet, void* stream) {
  if (!g || !grad_wet || (!grad_theta && g->n_theta > 0)) return fail(MG_ERR_INVALID_ARG, "NULL argument");
  if (!g->ready || g->mode != 1) return fail(MG_ERR_STATE, "graph not set up for backward (mode 1)");
  if (!g->have_forward) return fail(MG_ERR_STATE, "mg_backward needs a preceding mg_forward");
  if (int rc = check_binding(g)) return rc;
  hipStream_t st = (hipStream_t)stream;
  Ctx c = make_ctx(g, st);
  const int o = g->output_node;
  const float* yhat = c.U + (int64_t)g->uslot[o] * 2 * c.L;
  float* dy = c.G + (int64_t)g->gslot[o] * 2 * c.L;
  loss_backward(c, yhat, dy);
  // The input-gradient chain stays on the caller's stream; each FIR stage's
  // parameter-gradient work (FIR-gradient inverse columns, block sums, the
  // adjoints back to the raw parameters) is handed to the side stream after
  // an event, so it overlaps the next stages.  Every long-FIR stage has FIR-
  // gradient spectrum rows of its own, so the caller's stream never waits on
  // the side stream before the join.
  // Without a side stream (a graph bound by mg_setup_static) the same work
  // runs in the same order on the caller's stream.
  const bool side = g->side != nullptr;
  Ctx cs = c;
  if (side) cs.st = g->side;
  int ev = 0;
  auto fork = [&]() {
    if (!side) return;
    hipEventRecord(g->sev[ev], st);
    hipStreamWaitEvent(g->side, g->sev[ev], 0);
    ev = (ev + 1) % (int)g->sev.size();
  };
  size_t t3_row = 0;   // first FIR-gradient spectrum row of the next long-FIR stage
  // the first FIR stage of the schedule is the last one here: nothing on the
  // caller's stream is left to overlap its FIR-gradient work, so it stays there
  size_t last_fir = 0;
  for (size_t s = 1; s < g->stages.size() && !last_fir; ++s)
    if (is_conv(g->stages[s].type)) last_fir = s;
  // stage s ends the fused chain that starts at chain_start[s]
  std::vector<int> chain_start(g->stages.size(), -1);
  for (size_t s = 1; s < g->stages.size(); ++s)
    if (g->pw_run[s] >= 2) chain_start[s + g->pw_run[s] - 1] = (int)s;
  const NodeDesc* gdesc = (const NodeDesc*)(g->base + g->ws.gdesc);
  for (size_t s = g->stages.size() - 1; s >= 1; --s) {
    const Stage& S = g->stages[s];
    const int n = (int)S.nodes.size();
    const int off = S.desc_off;
    const int t = S.type;
    // nodes of this stage with several consumers: dL/dy is the sum of what
    // every consumer (a later stage, done by now) passed back
    if (g->gdesc_off[s + 1] > g->gdesc_off[s])
      launch_grad_sum(c, gdesc + g->gdesc_off[s], g->gdesc_off[s + 1] - g->gdesc_off[s]);
    if (t == MG_MIX || t == MG_OUT) continue;
    if (chain_start[s] >= 0) {
      const int s0 = chain_start[s], K = g->pw_run[s0];
      int types[PW_MAXK], offs[PW_MAXK];
      for (int i = 0; i < K; ++i) {
        types[i] = g->stages[s0 + i].type;
        offs[i] = g->stages[s0 + i].desc_off;
      }
      launch_pw_chain_bwd(c, types, offs, K, n);
      s = (size_t)s0;
      continue;
    }
    if (t == MG_GAINPAN || t == MG_IMAGER || t == MG_DIST) {
      launch_pointwise_bwd(c, t, off, n);
    } else if (t == MG_COMP || t == MG_GATE) {
      dyn_backward(c, t, off, n);
    } else if (t == MG_EQ) {
      eq_backward(c, off, n);
      const Ctx& cf = (s == last_fir) ? c : cs;
      if (s != last_fir) fork();
      eq_backward_fir(cf, off, n);
      fir_adjoint(cf, t, off, n, grad_theta);
    } else if (is_conv(t)) {
      float2* T3 = (float2*)(g->base + g->ws.T3) + t3_row * (size_t)g->fft.N;
      t3_row += (size_t)n;
      conv_backward(c, t, off, n, T3);
      fork();
      conv_backward_fir(cs, t, off, n, T3);
      fir_adjoint(cs, t, off, n, grad_theta);
    }
    // processors with several predecessors: every predecessor's dL/dy is
    // this node's dL/du (aliased slots), nothing to scatter
  }
  // join: the side stream's gradients before anything later on the stream
  if (side) {
    hipEventRecord(g->sev[ev], g->side);
    hipStreamWaitEvent(st, g->sev[ev], 0);
  }
  // dry/wet and direct parameter gradients of every processor from its
  // partial sums (kept per descriptor), in one launch
  launch_finish_all(c, (int)g->desc.size(), (const int2*)(g->base + g->ws.fin), grad_theta, grad_wet);
  g->have_forward = false;
  return hip_check(hipGetLastError(), "backward launch");
}

extern "C" int mg_node_output(const mg_graph* g, int32_t node, float* out, void* stream) {
  if (!g || !out || node < 0 || node >= g->n_nodes) return fail(MG_ERR_INVALID_ARG, "bad arguments");
  if (!g->ready) return fail(MG_ERR_STATE, "mg_setup has not been called");
  if (int rc = check_binding(g)) return rc;
  if (g->uslot[node] < 0) return fail(MG_ERR_INVALID_ARG, "input nodes have no output slot");
  const int64_t L = g->cfg.length;
  const float* src = (const float*)(g->base + g->ws.U) + (int64_t)g->uslot[node] * 2 * L;
  return hip_check(hipMemcpyAsync(out, src, (size_t)2 * L * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream),
                   "node output copy");
}

extern "C" int mg_profile_enable(mg_graph* g, const char* kernel_class) {
  if (!g) return fail(MG_ERR_INVALID_ARG, "NULL graph");
  Profiler& p = g->prof;
  p.cls = kernel_class ? kernel_class : "";
  p.used = 0;
  p.bytes = 0.0;
  p.launches = 0;
  p.overflow = false;
  if (!p.cls.empty() && p.ev.empty()) {
    p.ev.resize(8192);
    for (auto& e : p.ev) {
      int rc = hip_check(hipEventCreate(&e), "event create");
      if (rc) return rc;
    }
  }
  return MG_OK;
}

extern "C" int mg_profile_read(mg_graph* g, double* ms, int64_t* launches, double* bytes) {
  if (!g || !ms || !launches || !bytes) return fail(MG_ERR_INVALID_ARG, "NULL argument");
  Profiler& p = g->prof;
  if (p.overflow) {
    p.used = 0;
    p.bytes = 0.0;
    p.launches = 0;
    p.overflow = false;
    return fail(MG_ERR_INVALID_ARG, "more timed kernels than events between reads");
  }
  double total = 0.0;
  for (int i = 0; i + 1 < p.used; i += 2) {
    int rc = hip_check(hipEventSynchronize(p.ev[i + 1]), "event sync");
    if (rc) return rc;
    float t = 0.f;
    rc = hip_check(hipEventElapsedTime(&t, p.ev[i], p.ev[i + 1]), "event time");
    if (rc) return rc;
    total += t;
  }
  *ms = total;
  *launches = p.launches;
  *bytes = p.bytes;
  p.used = 0;
  p.bytes = 0.0;
  p.launches = 0;
  return MG_OK;
}

extern "C" int mg_adam_step(float* theta, float* m, float* v, const float* grad, int64_t n, float lr, float beta1,
                            float beta2, float eps, int32_t step, void* stream) {
  if (!theta || !m || !v || !grad || n < 0 || step < 1) return fail(MG_ERR_INVALID_ARG, "bad arguments");
  if (n == 0) return MG_OK;
  launch_adam(theta, m, v, grad, n, lr, beta1, beta2, eps, step, (hipStream_t)stream);
  return hip_check(hipGetLastError(), "adam launch");
}
