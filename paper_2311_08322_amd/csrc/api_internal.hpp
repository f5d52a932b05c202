// api_internal.hpp -- helpers shared by the host-side translation units of
// the C ABI (validation, errors, tuning table).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/stencil.h"
#include "common.hpp"

#define TRY(x)            \
  do {                    \
    int rc_ = (x);        \
    if (rc_) return rc_;  \
  } while (0)

namespace gt4mi {

int fail(int code, const char* fmt, ...);
int ok();
int hip_status(hipError_t e, const char* what);
int check_device();
int check_dtype(stencil_dtype dt);
int check_domain(const int64_t* dom);
int check_opts(const stencil_options* o);
bool domain_empty(const int64_t* dom);
size_t esize(stencil_dtype dt);

struct Span {
  uintptr_t lo, hi;
};
Span span_of(const stencil_field* f, size_t es);
bool overlap(Span a, Span b);
int check_no_alias(const char* oname, Span o, const char* iname, Span in);

enum Role { ROLE_HALO, ROLE_INTERIOR, ROLE_STAGGERED };
int check_field(const char* name, const stencil_field* f, const int64_t* dom, Role role, size_t es);

struct ResolvedOpts {
  int impl;
  int tile_i, tile_j;
  int column_store;
  void* ws;
  size_t ws_bytes;
  int form;                    // stencil_hdiff_form
  const stencil_field* kappa;  // per-point coefficient or null
  int order;                   // stencil_tile_order (resolved: XCD or DISPATCH)
};
// Tile shapes of the fused forward kernels: 256 columns (64x4, 32x8,
// 16x16: 512-lane workgroups in the two-ended step) or, in the two-ended
// step only, 128 columns (64x2, 32x4, 16x8: 256-lane workgroups).
inline bool tile_wide(int ti, int tj) { return (ti == 64 && tj == 4) || (ti == 32 && tj == 8) || (ti == 16 && tj == 16); }
inline bool tile_narrow(int ti, int tj) { return (ti == 64 && tj == 2) || (ti == 32 && tj == 4) || (ti == 16 && tj == 8); }
// options that ask for the generalised diffusion
inline bool variant_opts(const stencil_options* o) {
  return o && (o->hdiff_form != STENCIL_HDIFF_STATED || o->coeff_field != nullptr);
}
// validates opts->coeff_field on the domain (if set) and that `out` does not overlap it
int check_coeff_field(const stencil_options* o, const int64_t* dom, size_t es, const char* oname, Span out);
ResolvedOpts resolve_opts(const stencil_options* o, stencil_dtype dt, int op, const int64_t* dom);
size_t plain_ws_bytes(size_t es, const int64_t* dom);

// kernel argument blocks from field descriptors (pointers at the domain origin)
template <typename T>
inline const T* at_origin(const stencil_field* f) {
  return static_cast<const T*>(f->data) + f->origin[0] + f->origin[1] * f->stride[1] +
         f->origin[2] * f->stride[2];
}
template <typename T>
inline T* at_origin_mut(stencil_field* f) {
  return static_cast<T*>(f->data) + f->origin[0] + f->origin[1] * f->stride[1] +
         f->origin[2] * f->stride[2];
}
template <typename T>
StepArgs<T> step_args(const stencil_field* u, const stencil_field* data, const stencil_field* w,
                      stencil_field* out, const int64_t* dom, double coeff, double dt_dz, void* mask);
template <typename T>
AdjArgs<T> adj_args(const stencil_field* xbar, const stencil_field* w, T* lam, int64_t l_sj,
                    int64_t l_sk, stencil_field* ubar, const int64_t* dom, double coeff,
                    double dt_dz, const void* mask);

// persistent batched forward (batched.cpp).  ItemSpans: the buffers one
// item reads and writes.  check_step_batch validates the arguments and
// every item (not the workspace); launch_step_batch runs a validated,
// non-empty batch with its work list in ws (at least
// stencil_batch_workspace_bytes, 256-byte aligned, device memory).
struct ItemSpans {
  std::vector<Span> rd, wr;
};
int check_step_batch(stencil_dtype dtype, int n, const stencil_batch_item* items, const stencil_options* opts,
                     std::vector<ItemSpans>& spans);
int launch_step_batch(stencil_dtype dtype, int n, const stencil_batch_item* items, void* ws,
                      const stencil_options* opts, hipStream_t stream);

// tuning table (tune.cpp): tile, column store and tile order for (dtype, op,
// size class); the defaults, and false, when the class has no entry
bool tuning_get(stencil_dtype dt, int op, const int64_t* dom, int32_t* tile_i, int32_t* tile_j,
                int32_t* column_store, int32_t* tile_order);

}  // namespace gt4mi
