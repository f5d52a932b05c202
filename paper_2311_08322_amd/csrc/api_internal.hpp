// api_internal.hpp -- helpers shared by the host-side translation units of
// the C ABI (validation, errors, tuning table).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/stencil.h"

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
  int tile_i;
  int column_store;
  void* ws;
  size_t ws_bytes;
};
ResolvedOpts resolve_opts(const stencil_options* o, stencil_dtype dt, int op, const int64_t* dom);
size_t plain_ws_bytes(size_t es, const int64_t* dom);

// tuning table (tune.cpp): tile and column store for (dtype, op, size class)
void tuning_get(stencil_dtype dt, int op, const int64_t* dom, int32_t* tile_i, int32_t* tile_j,
                int32_t* column_store);

}  // namespace gt4mi
