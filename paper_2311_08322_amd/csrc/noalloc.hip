// noalloc.hip -- the batched forward step for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses
// that forbid hipMalloc).  The work list the persistent launch needs (the
// header with its work counter, the per-field prefix sums and argument
// blocks) goes into a fixed device array of this file instead of a
// caller-provided workspace; everything else is stencil_step_batched.
//
// Each device the library runs on holds its own copy of the array for the
// life of the process.  Host code never passes the array's name to a kernel
// (on the host it is only a stand-in for the symbol): the device address is
// looked up once per device with hipGetSymbolAddress, with that device
// current, and kept.  Every call on a device reuses the same array, so two
// calls that may run at the same time on one device race; the table upload
// of each call rewrites the header, whose work counter therefore starts at
// zero every call.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "../../include/stencil.h"
#include "api_internal.hpp"

namespace gt4mi {
namespace {

static __device__ __align__(256) uint8_t scratch[STENCIL_NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` on the current device (looked up on first use).
int scratch_address(void** out) {
  static std::mutex mu;
  static std::vector<void*> addr;  // per device; null until looked up
  int dev = 0;
  TRY(hip_status(hipGetDevice(&dev), "hipGetDevice"));
  std::lock_guard<std::mutex> lk(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    TRY(hip_status(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"));
    if (!p) return fail(STENCIL_E_HIP, "hipGetSymbolAddress returned a null scratch address");
    addr[dev] = p;
  }
  *out = addr[dev];
  return ok();
}

}  // namespace
}  // namespace gt4mi

using namespace gt4mi;

extern "C" int stencil_step_batched_noalloc(stencil_dtype dtype, int n, const stencil_batch_item* items,
                                            const stencil_options* opts, hipStream_t stream) {
  std::vector<ItemSpans> sp;
  TRY(check_step_batch(dtype, n, items, opts, sp));
  const size_t need = stencil_batch_workspace_bytes(dtype, n, items);
  if (need > (size_t)STENCIL_NOALLOC_SCRATCH_BYTES)
    return fail(STENCIL_E_UNSUPPORTED,
                "the batch's work list needs %zu bytes, more than the %d bytes of the fixed scratch array "
                "(use stencil_step_batched with a workspace)",
                need, STENCIL_NOALLOC_SCRATCH_BYTES);
  if (need == 0) return ok();
  TRY(check_device());
  void* ws = nullptr;
  TRY(scratch_address(&ws));
  return launch_step_batch(dtype, n, items, ws, opts, stream);
}
