// param.cpp -- the C ABI of the parameter gradients of a step (coeff, w).
#include <hip/hip_runtime.h>
#include <string.h>

#include "../../include/stencil.h"
#include "api_internal.hpp"
#include "launch.hpp"

using namespace gt4mi;

namespace {

int64_t r256(int64_t b) { return MaskLayout::round256(b); }

size_t partial_bytes(const int64_t* dom) {
  if (domain_empty(dom)) return 0;
  return (size_t)r256((int64_t)coeff_partial_count(dom[0], dom[1]) * 8);
}

Span bytes_span(const void* p, size_t n) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  return Span{a, a + n};
}

template <typename T>
int run(const stencil_field* u, const stencil_field* w, const stencil_field* x, const stencil_field* lam,
        stencil_field* w_bar, double* coeff_bar, const int64_t* dom, double dt_dz, int form, void* ws,
        hipStream_t s) {
  StepArgs<T> A = step_args<T>(u, lam, nullptr, nullptr, dom, 0.0, dt_dz, nullptr);
  A.form = form;
  WGradArgs<T> W;
  memset(&W, 0, sizeof W);
  if (w_bar) {
    W.w = at_origin<T>(w);
    W.w_sj = w->stride[1];
    W.w_sk = w->stride[2];
    W.x = at_origin<T>(x);
    W.x_sj = x->stride[1];
    W.x_sk = x->stride[2];
    W.lam = at_origin<T>(lam);
    W.l_sj = lam->stride[1];
    W.l_sk = lam->stride[2];
    W.wbar = at_origin_mut<T>(w_bar);
    W.b_sj = w_bar->stride[1];
    W.b_sk = w_bar->stride[2];
    W.ni = (int)dom[0];
    W.nj = (int)dom[1];
    W.nk = (int)dom[2];
    W.q = (T)(0.25 * dt_dz);
  }
  return hip_status(launch_param_grads<T>(A, w_bar ? &W : nullptr, static_cast<double*>(ws), coeff_bar, s),
                    "step parameter gradients");
}

}  // namespace

extern "C" {

size_t stencil_param_workspace_bytes(stencil_dtype dtype, const int64_t domain[3]) {
  if (check_dtype(dtype) || !domain || check_domain(domain)) return 0;
  return partial_bytes(domain);
}

int stencil_step_param_adjoint(stencil_dtype dtype, const stencil_field* u, const stencil_field* w,
                               const stencil_field* x, const stencil_field* lam, stencil_field* w_bar,
                               double* coeff_bar, const int64_t domain[3], double dt_dz,
                               const stencil_options* opts, void* ws, size_t ws_bytes, hipStream_t stream) {
  TRY(check_dtype(dtype));
  TRY(check_domain(domain));
  TRY(check_opts(opts));
  if (!w_bar && !coeff_bar) return fail(STENCIL_E_NULL, "w_bar and coeff_bar are both NULL");
  if (coeff_bar && opts && opts->coeff_field)
    return fail(STENCIL_E_ARG, "a step with a coefficient field has no scalar coeff_bar (stencil_coeff_field_adjoint)");
  const int form = opts ? opts->hdiff_form : STENCIL_HDIFF_STATED;
  const size_t es = esize(dtype);
  TRY(check_field("lam", lam, domain, ROLE_INTERIOR, es));
  std::vector<Span> in{span_of(lam, es)};
  if (coeff_bar) {
    TRY(check_field("u", u, domain, ROLE_HALO, es));
    in.push_back(span_of(u, es));
    if (reinterpret_cast<uintptr_t>(coeff_bar) % 8) return fail(STENCIL_E_DTYPE, "coeff_bar is not 8-byte aligned");
  }
  if (w_bar) {
    TRY(check_field("w", w, domain, ROLE_STAGGERED, es));
    TRY(check_field("x", x, domain, ROLE_INTERIOR, es));
    TRY(check_field("w_bar", w_bar, domain, ROLE_STAGGERED, es));
    in.push_back(span_of(w, es));
    in.push_back(span_of(x, es));
    const Span sb = span_of(w_bar, es);
    for (const Span& i : in) TRY(check_no_alias("w_bar", sb, "an input", i));
  }
  const size_t need = coeff_bar ? partial_bytes(domain) : 0;
  if (need) {
    if (!ws) return fail(STENCIL_E_WORKSPACE, "coeff_bar needs %zu bytes of workspace (ws is NULL)", need);
    if (ws_bytes < need) return fail(STENCIL_E_WORKSPACE, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(ws) % 8) return fail(STENCIL_E_WORKSPACE, "workspace is not 8-byte aligned");
    const Span sw = bytes_span(ws, need);
    for (const Span& i : in) TRY(check_no_alias("workspace", sw, "an input", i));
    if (w_bar) TRY(check_no_alias("workspace", sw, "w_bar", span_of(w_bar, es)));
  }
  if (coeff_bar) {
    const Span sc = bytes_span(coeff_bar, 8);
    for (const Span& i : in) TRY(check_no_alias("coeff_bar", sc, "an input", i));
    if (w_bar) TRY(check_no_alias("coeff_bar", sc, "w_bar", span_of(w_bar, es)));
    if (need) TRY(check_no_alias("coeff_bar", sc, "the workspace", bytes_span(ws, need)));
  }
  TRY(check_device());
  return dtype == STENCIL_F64
             ? run<double>(u, w, x, lam, w_bar, coeff_bar, domain, dt_dz, form, ws, stream)
             : run<float>(u, w, x, lam, w_bar, coeff_bar, domain, dt_dz, form, ws, stream);
}

int stencil_coeff_field_adjoint(stencil_dtype dtype, const stencil_field* u, const stencil_field* lam,
                                stencil_field* kappa_bar, const int64_t domain[3],
                                const stencil_options* opts, hipStream_t stream) {
  TRY(check_dtype(dtype));
  TRY(check_domain(domain));
  TRY(check_opts(opts));
  const size_t es = esize(dtype);
  TRY(check_field("u", u, domain, ROLE_HALO, es));
  TRY(check_field("lam", lam, domain, ROLE_INTERIOR, es));
  TRY(check_field("kappa_bar", kappa_bar, domain, ROLE_INTERIOR, es));
  const Span sk = span_of(kappa_bar, es);
  TRY(check_no_alias("kappa_bar", sk, "u", span_of(u, es)));
  TRY(check_no_alias("kappa_bar", sk, "lam", span_of(lam, es)));
  if (domain_empty(domain)) return ok();
  TRY(check_device());
  const int form = opts ? opts->hdiff_form : STENCIL_HDIFF_STATED;
  auto go = [&](auto tag) -> int {
    using T = decltype(tag);
    StepArgs<T> A = step_args<T>(u, lam, nullptr, kappa_bar, domain, 0.0, 0.0, nullptr);
    A.form = form;
    return hip_status(launch_coeff_field_grad<T>(A, stream), "coefficient field gradient");
  };
  return dtype == STENCIL_F64 ? go(double(0)) : go(float(0));
}

}  // extern "C"
