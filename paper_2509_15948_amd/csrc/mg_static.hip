// mg_setup_static: bind a graph to a workspace the library holds in a static
// device array, for callers that cannot allocate device memory themselves
// (code under HIP graph capture, serving loops that must not allocate,
// harnesses that forbid hipMalloc).
//
// The array (`scratch`, MG_STATIC_SCRATCH_BYTES) is a file-scope __device__
// variable: every GPU the library runs on holds one copy of it, at its own
// address, from the library's load until the process ends.  Its device
// address is looked up once per device with hipGetSymbolAddress (the array's
// name is a host-side stand-in in host code and is never passed to a kernel
// or a copy) and cached per device.
//
// One array per GPU means one bound graph per GPU at a time: a second
// mg_setup_static on the same device takes the array over, and the earlier
// graph's compute calls then fail with MG_ERR_STATE until it is bound again.
// Calls that overlap on one GPU (two graphs, or two host threads driving the
// same graph) race on the array.
#include <mutex>
#include <string>
#include <vector>

#include "mg_device.h"
#include "mg_kernels.h"

namespace mg {
int fail(int code, const std::string& msg);
}

namespace {

static __device__ __align__(256) char scratch[MG_STATIC_SCRATCH_BYTES];

struct DeviceScratch {
  void* ptr = nullptr;   // device address of this device's copy of scratch
  uint64_t gen = 0;      // bindings made so far on this device
};

std::mutex g_mu;
std::vector<DeviceScratch> g_dev;

}  // namespace

namespace mg {

int check_binding(const mg_graph* g) {
  if (g->static_dev < 0) return MG_OK;
  std::lock_guard<std::mutex> lock(g_mu);
  if ((size_t)g->static_dev >= g_dev.size() || g_dev[g->static_dev].gen != g->static_gen)
    return fail(MG_ERR_STATE, "the static scratch of device " + std::to_string(g->static_dev) +
                                  " has been bound to another graph since; call mg_setup_static again");
  return MG_OK;
}

}  // namespace mg

using namespace mg;

extern "C" int mg_setup_static(mg_graph* g, int32_t mode, const float* reverb_noise, const float* target,
                               void* stream) {
  if (!g || !target || (mode != 0 && mode != 1)) return fail(MG_ERR_INVALID_ARG, "bad arguments");
  size_t need = 0;
  if (int rc = mg_workspace_size(g, mode, &need)) return rc;
  if (need > (size_t)MG_STATIC_SCRATCH_BYTES)
    return fail(MG_ERR_BUDGET, "the graph needs a workspace of " + std::to_string(need) +
                                   " bytes, more than the static scratch holds (" +
                                   std::to_string((size_t)MG_STATIC_SCRATCH_BYTES) + " bytes); use mg_setup");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(MG_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  void* ptr = nullptr;
  uint64_t gen = 0;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if ((size_t)dev >= g_dev.size()) g_dev.resize(dev + 1);
    if (!g_dev[dev].ptr) {
      // once per device, with that device current
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail(MG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      g_dev[dev].ptr = p;
    }
    ptr = g_dev[dev].ptr;
    gen = ++g_dev[dev].gen;  // any graph bound before on this device is now stale
  }
  // the same binding as mg_setup, on the array's device address, without the
  // side stream (nothing is created); every region the kernels accumulate
  // into is cleared there, whatever the array held from the last call
  if (int rc = bind_workspace(g, ptr, (size_t)MG_STATIC_SCRATCH_BYTES, mode, reverb_noise, target,
                              (hipStream_t)stream, false))
    return rc;
  g->static_dev = dev;
  g->static_gen = gen;
  return MG_OK;
}
