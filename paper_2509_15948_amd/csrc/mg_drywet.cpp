// Host control of the dry/wet method (Alg. 3, Sec. 6.2 "Candidate
// Sampling"): which processors one pruning trial bypasses, and the update
// after its loss is known.  The caller evaluates each proposed trial (for
// instance with mg_forward_trials, B = 1) and reports its loss.
//
// Per processor type t among the alive processors: V_t the alive processors
// of t, N_t = |V_t| when the iteration starts, r_t = 0.1.  Each trial draws a
// remaining type uniformly (the caller supplies the draws u_i in [0, 1): the
// floor(u_i |T|)-th remaining type in the order e c n x s g d r) and bypasses
// its k = floor(N_t r_t + 1/2) processors of least dry/wet weight (at least
// one, at most |V_t|; ties by index) on top of everything pruned so far.  A
// trial whose loss passes the tolerance test prunes them (they leave V_t,
// L_min <- min(L_min, L), and t leaves the set once V_t is empty);
// otherwise r_t is halved while floor(N_t r_t + 1/2) > 1, and t leaves the
// set when it is not.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "mg_internal.h"

namespace mg {
int fail(int code, const std::string& msg);
}
using namespace mg;

struct mg_drywet {
  int P = 0;
  std::vector<float> w;              // effective dry/wet weight per processor
  std::vector<uint8_t> keep;         // 1: not pruned (so far)
  std::vector<int> types;            // remaining types, in the order e c n x s g d r
  std::vector<std::vector<int>> V;   // per type code: remaining processors, least weight first
  std::vector<int> N;                // per type code: |V_t| at the start
  std::vector<double> r;             // per type code: r_t
  std::vector<double> u;             // the caller's uniform draws
  size_t next_u = 0;
  double L_min = 0.0, tau = 0.0;
  int relative = 0;
  // the proposed trial
  bool pending = false;
  int cur_type = -1, cur_kraw = 0;
  std::vector<int> cur;
  int trials = 0;
};

static int order_pos(int type) {
  for (int i = 0; i < 8; ++i)
    if (kProcOrder[i] == type) return i;
  return -1;
}

extern "C" int mg_drywet_begin(int32_t P, const int32_t* proc_type, const float* wet, const float* mask,
                               const uint8_t* alive, double L_min, double tau, int32_t relative, const double* u,
                               int32_t n_u, mg_drywet** out) {
  if (P < 0 || (P > 0 && (!proc_type || !wet || !alive)) || !out || n_u < 0 || (n_u > 0 && !u) || tau < 0)
    return fail(MG_ERR_INVALID_ARG, "bad arguments");
  if (!std::isfinite(L_min)) return fail(MG_ERR_NONFINITE, "L_min is not finite");
  mg_drywet* s = new mg_drywet();
  s->P = P;
  s->w.resize(P);
  s->keep.assign(alive, alive + P);
  s->V.assign(NTYPES, {});
  s->N.assign(NTYPES, 0);
  s->r.assign(NTYPES, 0.1);
  for (int p = 0; p < P; ++p) {
    s->w[p] = 1.0f / (1.0f + expf(-wet[p]));
    if (mask) s->w[p] *= mask[p];
    s->keep[p] = alive[p] ? 1 : 0;
    if (!is_proc(proc_type[p]) || order_pos(proc_type[p]) < 0) {
      delete s;
      return fail(MG_ERR_INVALID_ARG, "proc_type holds a non-processor type");
    }
    if (alive[p]) s->V[proc_type[p]].push_back(p);
  }
  for (int i = 0; i < 8; ++i) {
    const int t = kProcOrder[i];
    auto& v = s->V[t];
    std::stable_sort(v.begin(), v.end(), [&](int a, int b) {
      return s->w[a] < s->w[b] || (s->w[a] == s->w[b] && a < b);
    });
    s->N[t] = (int)v.size();
    if (!v.empty()) s->types.push_back(t);
  }
  s->u.assign(u, u + n_u);
  s->L_min = L_min;
  s->tau = tau;
  s->relative = relative ? 1 : 0;
  *out = s;
  return MG_OK;
}

extern "C" int mg_drywet_next(mg_drywet* s, uint8_t* keep, int32_t* done) {
  if (!s || !keep || !done) return fail(MG_ERR_INVALID_ARG, "bad arguments");
  if (s->pending) return fail(MG_ERR_STATE, "the loss of the last proposed trial has not been reported");
  if (s->types.empty()) {
    *done = 1;
    return MG_OK;
  }
  if (s->next_u >= s->u.size()) return fail(MG_ERR_SHAPE, "ran out of uniform draws");
  const double ud = s->u[s->next_u++];
  if (!(ud >= 0.0 && ud < 1.0)) return fail(MG_ERR_INVALID_ARG, "uniform draws must lie in [0, 1)");
  const int t = s->types[(size_t)std::floor(ud * (double)s->types.size())];
  const int k_raw = (int)std::floor((double)s->N[t] * s->r[t] + 0.5);
  const int k = std::min<int>(std::max(1, k_raw), (int)s->V[t].size());
  s->cur.assign(s->V[t].begin(), s->V[t].begin() + k);
  s->cur_type = t;
  s->cur_kraw = k_raw;
  for (int p = 0; p < s->P; ++p) keep[p] = s->keep[p];
  for (int p : s->cur) keep[p] = 0;
  s->pending = true;
  *done = 0;
  return MG_OK;
}

extern "C" int mg_drywet_report(mg_drywet* s, double L) {
  if (!s) return fail(MG_ERR_INVALID_ARG, "NULL state");
  if (!s->pending) return fail(MG_ERR_STATE, "no trial is pending");
  s->pending = false;
  s->trials += 1;
  const int t = s->cur_type;
  // a non-finite loss never passes the test
  const bool ok = std::isfinite(L) && L < (s->relative ? s->L_min * (1.0 + s->tau) : s->L_min + s->tau);
  auto drop_type = [&]() { s->types.erase(std::find(s->types.begin(), s->types.end(), t)); };
  if (ok) {
    s->L_min = std::min(s->L_min, L);
    for (int p : s->cur) s->keep[p] = 0;
    s->V[t].erase(s->V[t].begin(), s->V[t].begin() + s->cur.size());
    if (s->V[t].empty()) drop_type();
  } else if (s->cur_kraw > 1) {
    s->r[t] *= 0.5;
  } else {
    drop_type();
  }
  return MG_OK;
}

extern "C" int mg_drywet_end(mg_drywet* s, uint8_t* keep, double* L_min, int32_t* trials) {
  if (!s) return fail(MG_ERR_INVALID_ARG, "NULL state");
  if (keep)
    for (int p = 0; p < s->P; ++p) keep[p] = s->keep[p];
  if (L_min) *L_min = s->L_min;
  if (trials) *trials = s->trials;
  delete s;
  return MG_OK;
}
