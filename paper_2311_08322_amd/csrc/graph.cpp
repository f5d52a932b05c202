// graph.cpp -- a time loop of stencil steps captured once into a HIP graph
// and replayed with one launch (ping-pong state buffers, frozen halo).
#include <hip/hip_runtime.h>

#include "../../include/stencil.h"
#include "api_internal.hpp"

struct stencil_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
  int nsteps;
};

using namespace gt4mi;

extern "C" {

int stencil_graph_capture_steps(stencil_dtype dtype, int nsteps, stencil_field* u_a, stencil_field* u_b,
                                const stencil_field* data, const stencil_field* w,
                                const int64_t domain[3], double coeff, double dt_dz,
                                const stencil_options* opts, hipStream_t stream, stencil_graph** out) {
  if (!out) return fail(STENCIL_E_NULL, "graph output pointer is NULL");
  *out = nullptr;
  if (nsteps <= 0) return fail(STENCIL_E_ARG, "nsteps = %d must be positive", nsteps);
  if (!stream) return fail(STENCIL_E_ARG, "capture needs a non-default stream");
  if (int rc = check_dtype(dtype)) return rc;
  if (int rc = check_domain(domain)) return rc;
  const size_t es = esize(dtype);
  // both ping-pong buffers are read with a halo and written on the interior
  if (int rc = check_field("u_a", u_a, domain, ROLE_HALO, es)) return rc;
  if (int rc = check_field("u_b", u_b, domain, ROLE_HALO, es)) return rc;
  if (int rc = check_no_alias("u_b", span_of(u_b, es), "u_a", span_of(u_a, es))) return rc;
  if (int rc = check_device()) return rc;  // cache the device check outside the capture
  // validate one step eagerly-in-metadata only: stencil_step validates every call below
  hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_status(e, "hipStreamBeginCapture");
  int rc = STENCIL_OK;
  for (int s = 0; s < nsteps && rc == STENCIL_OK; ++s) {
    const stencil_field* src = (s % 2 == 0) ? u_a : u_b;
    stencil_field* dst = (s % 2 == 0) ? u_b : u_a;
    rc = stencil_step(dtype, src, data, w, dst, domain, coeff, dt_dz, nullptr, opts, stream);
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(stream, &g);
  if (rc != STENCIL_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_status(e, "hipStreamEndCapture");
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_status(e, "hipGraphInstantiate");
  }
  stencil_graph* h = new (std::nothrow) stencil_graph;
  if (!h) {
    (void)hipGraphExecDestroy(x);
    (void)hipGraphDestroy(g);
    return fail(STENCIL_E_ARG, "out of host memory");
  }
  h->graph = g;
  h->exec = x;
  h->nsteps = nsteps;
  *out = h;
  return STENCIL_OK;
}

int stencil_graph_launch(stencil_graph* g, hipStream_t stream) {
  if (!g) return fail(STENCIL_E_NULL, "graph is NULL");
  return hip_status(hipGraphLaunch(g->exec, stream), "hipGraphLaunch");
}

int stencil_graph_destroy(stencil_graph* g) {
  if (!g) return STENCIL_OK;
  hipError_t e1 = hipGraphExecDestroy(g->exec);
  hipError_t e2 = hipGraphDestroy(g->graph);
  delete g;
  if (e1 != hipSuccess) return hip_status(e1, "hipGraphExecDestroy");
  return hip_status(e2, "hipGraphDestroy");
}

}  // extern "C"
