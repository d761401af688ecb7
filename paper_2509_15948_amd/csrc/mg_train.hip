// Entry points of the paper's training regime (Sec. 5.1, Sec. 6.3): a new
// target mix for the resident loss features (each step trains on a random
// segment of the song), the regulariser weights (alpha_p is ramped during
// pruning), and AdamW.
#include <string>

#include "mg_device.h"
#include "mg_kernels.h"

namespace mg {
int fail(int code, const std::string& msg);
}
using namespace mg;

static int hip_ok(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return fail(MG_ERR_OOM, std::string(what) + ": " + hipGetErrorString(e));
  if (e != hipSuccess) return fail(MG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return MG_OK;
}

extern "C" int mg_target_prepare(mg_graph* g, const float* target, void* stream) {
  if (!g || !target) return fail(MG_ERR_INVALID_ARG, "bad arguments");
  if (!g->ready) return fail(MG_ERR_STATE, "mg_setup has not been called");
  if (int rc = check_binding(g)) return rc;
  Ctx c = make_ctx(g, (hipStream_t)stream);
  loss_target(c, target);
  // the loss statistics a pending backward would read, and the cached
  // forward the trials compare against, belong to the old target
  g->have_forward = false;
  g->have_cache = false;
  return hip_ok(hipGetLastError(), "target features launch");
}

extern "C" int mg_set_alpha(mg_graph* g, double alpha_g, double alpha_p) {
  if (!g || !(alpha_g >= 0.0) || !(alpha_p >= 0.0)) return fail(MG_ERR_INVALID_ARG, "bad arguments");
  if (g->have_forward) return fail(MG_ERR_STATE, "a forward awaits its backward; change the weights after it");
  g->cfg.alpha_g = alpha_g;
  g->cfg.alpha_p = alpha_p;
  return MG_OK;
}

extern "C" int mg_adamw_step(float* theta, float* m, float* v, const float* grad, int64_t n, float lr, float beta1,
                             float beta2, float eps, float weight_decay, int32_t step, void* stream) {
  if (!theta || !m || !v || !grad || n < 0 || step < 1 || !(weight_decay >= 0.0f))
    return fail(MG_ERR_INVALID_ARG, "bad arguments");
  if (n == 0) return MG_OK;
  launch_adam(theta, m, v, grad, n, lr, beta1, beta2, eps, step, (hipStream_t)stream, weight_decay);
  return hip_ok(hipGetLastError(), "adamw launch");
}
