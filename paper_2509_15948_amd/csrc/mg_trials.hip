// Pruning trials by suffix recomputation, and the decision rule of a pruning
// round (Alg. 2, with the trials of a round evaluated as one batch).
//
// A trial bypasses some processors (w = 0, so y = u: Sec. 1.2).  Every node
// that is not downstream of a bypassed processor keeps the output of the last
// forward; the nodes downstream of one are evaluated again as "copies" that
// share the original node's parameters, FIR tables and spectra but write new
// output slots.  Copies of one stage across all trials of a batch form one
// contiguous descriptor range and run through the same per-stage kernels as
// the graph itself, so each copy computes exactly what a complete forward
// with that mask computes (same kernels, same fixed-order reductions).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "mg_device.h"
#include "mg_kernels.h"

namespace mg {
int fail(int code, const std::string& msg);

// Host planning of one call.  Returns MG_OK or an error code.
static int plan_trials(const mg_graph& g, const uint8_t* keep, int B, TrialPlan& tp) {
  const int P = g.n_proc;
  const int n_desc = (int)g.desc.size();
  std::vector<int> desc_of(g.n_nodes, -1), node_of_proc(std::max(1, P), -1);
  for (int j = 0; j < n_desc; ++j) desc_of[g.desc[j].node] = j;
  for (int v = 0; v < g.n_nodes; ++v)
    if (g.proc_idx[v] >= 0) node_of_proc[g.proc_idx[v]] = v;
  tp.desc.clear();
  tp.srcs.clear();
  tp.batches.clear();
  tp.keep.assign((size_t)B * std::max(1, P), 1.0f);
  tp.sub.resize((size_t)B * std::max(1, n_desc));
  // per trial: bypassed nodes and the copies (sigma order)
  std::vector<std::vector<char>> dropped(B);
  std::vector<std::vector<int>> copies(B);
  std::vector<int> need(B, 0);
  for (int b = 0; b < B; ++b) {
    dropped[b].assign(g.n_nodes, 0);
    std::vector<char> aff(g.n_nodes, 0);
    for (int p = 0; p < P; ++p)
      if (!keep[(size_t)b * P + p]) {
        dropped[b][node_of_proc[p]] = 1;
        tp.keep[(size_t)b * P + p] = 0.0f;
      }
    for (int v : g.order)  // topological: predecessors first
      for (int p : g.preds[v])
        if (dropped[b][p] || aff[p]) aff[v] = 1;
    for (int v : g.order)
      if (aff[v]) {
        copies[b].push_back(v);
        need[b] += 1 + ((is_proc(g.type[v]) && g.preds[v].size() > 1) ? 1 : 0);
      }
    if (need[b] > g.trial_slots)
      return fail(MG_ERR_SHAPE, "trial " + std::to_string(b) + " needs " + std::to_string(need[b]) +
                                    " node slots, more than trial_slots = " + std::to_string(g.trial_slots));
  }
  // batches: consecutive trials while their slots fit
  int t = 0;
  while (t < B) {
    TrialPlan::Batch bt;
    bt.t0 = t;
    int used = 0;
    while (t < B && used + need[t] <= g.trial_slots) used += need[t++];
    bt.t1 = t;
    bt.d0 = (int)tp.desc.size();
    const int nb = bt.t1 - bt.t0;
    // slots of the copies, per trial in sigma order
    std::vector<std::vector<int>> slot(nb), insum(nb);
    int next = g.n_uslots;
    for (int k = 0; k < nb; ++k) {
      const int b = bt.t0 + k;
      slot[k].assign(g.n_nodes, -1);
      insum[k].assign(g.n_nodes, -1);
      for (int v : copies[b]) {
        slot[k][v] = next++;
        if (is_proc(g.type[v]) && g.preds[v].size() > 1) insum[k][v] = next++;
      }
    }
    auto ref = [&](int k, int v) -> SrcRef {
      const int b = bt.t0 + k;
      if (slot[k][v] >= 0) return SrcRef{1, slot[k][v]};
      if (dropped[b][v]) {  // bypassed and not downstream of a change: its input
        const NodeDesc& d = g.desc[desc_of[v]];
        return SrcRef{d.in_kind, d.in_slot};
      }
      if (g.type[v] == MG_IN) return SrcRef{0, g.track[v]};
      return SrcRef{1, g.uslot[v]};
    };
    // descriptors, stage-major; the copy of node v in trial k gets lg row
    // n_desc + (its index inside the batch)
    const int n_stages = (int)g.stages.size();
    bt.stage_off.assign(n_stages, 0);
    bt.stage_n.assign(n_stages, 0);
    for (int k = 0; k < nb; ++k)
      for (int j = 0; j < n_desc; ++j) tp.sub[(size_t)(bt.t0 + k) * n_desc + j] = j;
    for (int s = 1; s < n_stages; ++s) {
      bt.stage_off[s] = (int)tp.desc.size() - bt.d0;
      for (int k = 0; k < nb; ++k) {
        const int b = bt.t0 + k;
        for (int v : copies[b]) {
          if (g.stage_of[v] != s) continue;
          NodeDesc d = g.desc[desc_of[v]];
          d.out_slot = slot[k][v];
          d.gin = -1;
          d.gout = -1;
          d.mrow = d.proc >= 0 ? b * P + d.proc : -1;
          d.src_begin = 0;
          d.src_count = 0;
          const bool sum_node = (g.type[v] == MG_MIX || g.type[v] == MG_OUT || g.preds[v].size() > 1);
          if (sum_node) {
            std::vector<int> ps = g.preds[v];
            std::sort(ps.begin(), ps.end());  // the graph's own summation order
            d.src_begin = g.n_src_base + (int)tp.srcs.size();
            d.src_count = (int)ps.size();
            for (int p : ps) tp.srcs.push_back(ref(k, p));
          }
          if (is_proc(g.type[v])) {
            if (g.preds[v].size() > 1) {
              d.in_kind = 1;
              d.in_slot = insum[k][v];
            } else {
              const SrcRef r = ref(k, g.preds[v][0]);
              d.in_kind = r.kind;
              d.in_slot = r.slot;
            }
          }
          tp.sub[(size_t)b * n_desc + desc_of[v]] = n_desc + ((int)tp.desc.size() - bt.d0);
          tp.desc.push_back(d);
          bt.stage_n[s] += 1;
        }
      }
    }
    bt.out_slot.resize(nb);
    for (int k = 0; k < nb; ++k) bt.out_slot[k] = ref(k, g.output_node).slot;
    tp.batches.push_back(bt);
  }
  if ((int)tp.desc.size() > g.trial_desc_cap || (int)tp.srcs.size() > g.trial_src_cap)
    return fail(MG_ERR_SHAPE, "trial tables exceed the reserved capacity");
  return MG_OK;
}

}  // namespace mg

using namespace mg;

static int hip_ok(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(MG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return MG_OK;
}

extern "C" int mg_forward_trials(mg_graph* g, const uint8_t* keep, int32_t B, double* losses, void* stream) {
  if (!g || !keep || !losses || B < 1) return fail(MG_ERR_INVALID_ARG, "bad arguments");
  if (!g->ready) return fail(MG_ERR_STATE, "mg_setup has not been called");
  if (int rc0 = check_binding(g)) return rc0;
  if (B > g->cfg.max_trials) return fail(MG_ERR_SHAPE, "B exceeds max_trials of the graph's configuration");
  if (!g->have_cache) return fail(MG_ERR_STATE, "mg_forward_trials needs a preceding mg_forward");
  hipStream_t st = (hipStream_t)stream;
  int rc;
  // the host tables of the previous call must have reached the device
  if (g->trial_ev_pending) {
    if ((rc = hip_ok(hipEventSynchronize(g->trial_ev), "trial event"))) return rc;
    g->trial_ev_pending = false;
  }
  TrialPlan& tp = g->tplan;
  if ((rc = plan_trials(*g, keep, B, tp))) return rc;
  if (!g->trial_ev && (rc = hip_ok(hipEventCreateWithFlags(&g->trial_ev, hipEventDisableTiming), "event create")))
    return rc;
  const WsPlan& w = g->ws;
  const int P = g->n_proc;
  const int n_desc = (int)g->desc.size();
  char* base = g->base;
  if (!tp.desc.empty() &&
      (rc = hip_ok(hipMemcpyAsync(base + w.tr_desc, tp.desc.data(), tp.desc.size() * sizeof(NodeDesc),
                                  hipMemcpyHostToDevice, st), "trial descriptors")))
    return rc;
  if (!tp.srcs.empty() &&
      (rc = hip_ok(hipMemcpyAsync(base + w.srcs + (size_t)g->n_src_base * sizeof(SrcRef), tp.srcs.data(),
                                  tp.srcs.size() * sizeof(SrcRef), hipMemcpyHostToDevice, st), "trial sources")))
    return rc;
  if (P > 0 && (rc = hip_ok(hipMemcpyAsync(base + w.tr_keep, tp.keep.data(), (size_t)B * P * 4,
                                           hipMemcpyHostToDevice, st), "trial keep")))
    return rc;
  if (n_desc > 0 && (rc = hip_ok(hipMemcpyAsync(base + w.tr_sub, tp.sub.data(), (size_t)B * n_desc * 4,
                                                hipMemcpyHostToDevice, st), "trial rows")))
    return rc;
  if ((rc = hip_ok(hipEventRecord(g->trial_ev, st), "trial event"))) return rc;
  g->trial_ev_pending = true;
  float* tmask = (float*)(base + w.tr_mask);
  launch_trial_mask(tmask, g->f_mask, (const float*)(base + w.tr_keep), P, B, st);
  Ctx c = make_ctx(g, st);
  c.trial = true;
  c.mask = tmask;
  double* stats = (double*)(base + w.tr_stats);
  const int n_res = (int)g->lres.size();
  for (const auto& bt : tp.batches) {
    // this batch's copies into the descriptor window after the graph's own
    int n_copy = 0;
    for (size_t s = 1; s < bt.stage_n.size(); ++s) n_copy += bt.stage_n[s];
    if (n_copy > 0 &&
        (rc = hip_ok(hipMemcpyAsync(base + w.desc + (size_t)n_desc * sizeof(NodeDesc),
                                    base + w.tr_desc + (size_t)bt.d0 * sizeof(NodeDesc), (size_t)n_copy * sizeof(NodeDesc),
                                    hipMemcpyDeviceToDevice, st), "trial window")))
      return rc;
    for (size_t s = 1; s < bt.stage_n.size(); ++s) {
      if (!bt.stage_n[s]) continue;
      forward_stage(c, g->stages[s].type, n_desc + bt.stage_off[s], bt.stage_n[s], false,
                    tp.desc.data() + bt.d0 + bt.stage_off[s]);
    }
    for (int k = 0; k < bt.t1 - bt.t0; ++k) {
      const float* yhat = c.U + (int64_t)bt.out_slot[k] * 2 * c.L;
      loss_forward(c, yhat, stats + (size_t)(bt.t0 + k) * 128);
    }
    launch_finalize_trials(c, losses + (size_t)bt.t0 * 7, stats + (size_t)bt.t0 * 128, n_res, n_desc,
                           tmask + (size_t)bt.t0 * P, P, (const int*)(base + w.tr_sub) + (size_t)bt.t0 * n_desc,
                           bt.t1 - bt.t0);
  }
  return hip_ok(hipGetLastError(), "trial launch");
}

// ---------------------------------------------------------------- decision rule
extern "C" int mg_prune_candidates(int32_t P, const float* wet, const float* mask, const uint8_t* alive,
                                   int32_t max_n, int32_t* cand, int32_t* n_out) {
  if (P < 0 || (P > 0 && (!wet || !alive)) || max_n < 0 || (max_n > 0 && !cand) || !n_out)
    return fail(MG_ERR_INVALID_ARG, "bad arguments");
  std::vector<float> w(std::max(1, P));
  for (int p = 0; p < P; ++p) {
    w[p] = 1.0f / (1.0f + expf(-wet[p]));
    if (mask) w[p] *= mask[p];
  }
  std::vector<int> idx;
  for (int p = 0; p < P; ++p)
    if (alive[p]) idx.push_back(p);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return w[a] < w[b] || (w[a] == w[b] && a < b); });
  const int n = std::min<int>(max_n, (int)idx.size());
  for (int i = 0; i < n; ++i) cand[i] = idx[i];
  *n_out = n;
  return MG_OK;
}

extern "C" int mg_prune_order(int32_t n, const int32_t* cand, const double* L_cand, double L_min, double tau,
                              int32_t relative, int32_t* order, int32_t* n_out) {
  if (n < 0 || (n > 0 && (!cand || !L_cand || !order)) || !n_out) return fail(MG_ERR_INVALID_ARG, "bad arguments");
  if (!std::isfinite(L_min)) return fail(MG_ERR_NONFINITE, "L_min is not finite");
  std::vector<int> keep;
  for (int i = 0; i < n; ++i)
    if (L_cand[i] - L_min < (relative ? tau * L_min : tau)) keep.push_back(i);
  std::stable_sort(keep.begin(), keep.end(), [&](int a, int b) {
    const double da = L_cand[a] - L_min, db = L_cand[b] - L_min;
    return da < db || (da == db && cand[a] < cand[b]);
  });
  for (size_t i = 0; i < keep.size(); ++i) order[i] = cand[keep[i]];
  *n_out = (int32_t)keep.size();
  return MG_OK;
}

extern "C" int mg_prune_accept(int32_t n, const double* L_prefix, double L_min, double tau, int32_t relative,
                               int32_t* k_out) {
  if (n < 0 || (n > 0 && !L_prefix) || !k_out) return fail(MG_ERR_INVALID_ARG, "bad arguments");
  if (!std::isfinite(L_min)) return fail(MG_ERR_NONFINITE, "L_min is not finite");
  int k = 0;
  for (int i = 0; i < n; ++i)
    if (L_prefix[i] < (relative ? L_min * (1.0 + tau) : L_min + tau)) k = i + 1;
  *k_out = k;
  return MG_OK;
}
