// tpo_execute_noalloc: the whole method with the workspace taken from a
// fixed device array of the library instead of a caller buffer, for callers
// that cannot allocate device memory (code under stream capture, tight
// serving loops, harnesses that forbid allocation).
//
// The array `scratch` is a file-scope __device__ variable: each GPU the
// library runs on holds its own copy, of kScratchBytes, until the process
// ends.  Host code never uses the array's name as an address (on the host it
// names a stand-in, not device memory): the first call on a device looks up
// that device's copy with hipGetSymbolAddress and keeps the address, and
// every kernel gets that address as its workspace, as it gets the caller's
// buffer from tpo_execute.  The kernels are those of tpo_execute.
//
// Every call on one GPU shares that GPU's array, and the array keeps the last
// call's contents.  Nothing in it has to start at zero: as with a caller's
// workspace, whose contents on entry are unspecified, each job writes its
// status block from the host first and resets its grid-barrier counters with
// a small kernel before each use.  Calls that overlap on one GPU (two
// threads, two streams) race on the array: callers serialise them.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "dev_common.hpp"
#include "tpo_internal.hpp"

namespace {

constexpr size_t kScratchBytes = TPO_NOALLOC_MAX_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

// The current device's copy of `scratch` (looked up once per device, with
// that device current).
tpo_status scratch_for_current_device(tpo_plan* plan, void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return tpo::plan_fail(plan, TPO_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return tpo::plan_fail(plan, TPO_EDEVICE, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return tpo::plan_fail(plan, TPO_EDEVICE,
                            std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return TPO_OK;
}

}  // namespace

extern "C" {

tpo_status tpo_execute_noalloc(tpo_plan* plan, const tpo_inputs* in, void* stream, const tpo_outputs* out) {
  if (!plan) return TPO_EINVAL;
  if (plan->lay.total > kScratchBytes)
    return tpo::plan_fail(plan, TPO_ENOMEM,
                          "the job needs " + std::to_string(plan->lay.total) +
                              " bytes of workspace; the no-allocation entry point holds " +
                              std::to_string(kScratchBytes));
  if (plan->par.flags & TPO_FLAG_TIMING)
    return tpo::plan_fail(plan, TPO_EINVAL, "a plan with TPO_FLAG_TIMING creates events; use one without");
  void* ws = nullptr;
  const tpo_status st = scratch_for_current_device(plan, &ws);
  if (st != TPO_OK) return st;
  return tpo::execute_plan(plan, in, ws, kScratchBytes, static_cast<hipStream_t>(stream), out, true);
}

}  // extern "C"
