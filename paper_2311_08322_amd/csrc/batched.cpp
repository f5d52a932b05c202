// batched.cpp -- placeholder entry points of the batched launch.
#include "../../include/stencil.h"
#include "api_internal.hpp"

using namespace gt4mi;

extern "C" {

size_t stencil_batch_workspace_bytes(stencil_dtype, int, const stencil_batch_item*) { return 0; }
size_t stencil_batch_adjoint_workspace_bytes(stencil_dtype, int, const stencil_batch_adjoint_item*) {
  return 0;
}
int stencil_step_batched(stencil_dtype, int, const stencil_batch_item*, void*, size_t,
                         const stencil_options*, hipStream_t) {
  return fail(STENCIL_E_UNSUPPORTED, "batched launch not built");
}
int stencil_step_adjoint_batched(stencil_dtype, int, const stencil_batch_adjoint_item*, void*, size_t,
                                 const stencil_options*, hipStream_t) {
  return fail(STENCIL_E_UNSUPPORTED, "batched launch not built");
}

}  // extern "C"
