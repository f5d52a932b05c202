// api.cpp -- the C ABI (include/stencil.h): O(1) host-side validation of
// field metadata, implementation choice and kernel dispatch.  No call reads
// device memory, allocates or synchronises (the autotuner excepted).
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/stencil.h"
#include "api_internal.hpp"
#include "common.hpp"
#include "launch.hpp"

namespace gt4mi {

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ok() { return STENCIL_OK; }

int hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return STENCIL_OK;
  return fail(STENCIL_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// ------------------------------------------------------------------ device
// The kernels are compiled for gfx950 only; refuse other devices up front.
int check_device() {
  static std::mutex mu;
  static std::vector<int> known;  // per device: 0 unknown, 1 ok, -1 unsupported
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(mu);
  if ((int)known.size() <= dev) known.resize(dev + 1, 0);
  if (known[dev] == 0) {
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, dev);
    if (e != hipSuccess) return hip_status(e, "hipGetDeviceProperties");
    known[dev] = (strncmp(p.gcnArchName, "gfx950", 6) == 0) ? 1 : -1;
    if (known[dev] < 0)
      return fail(STENCIL_E_UNSUPPORTED, "device %d is %s; this library is built for gfx950", dev,
                  p.gcnArchName);
  }
  if (known[dev] < 0) return fail(STENCIL_E_UNSUPPORTED, "device %d is not gfx950", dev);
  return STENCIL_OK;
}

// ------------------------------------------------------------------ validation
size_t esize(stencil_dtype dt) { return dt == STENCIL_F64 ? 8 : 4; }

int check_dtype(stencil_dtype dt) {
  if (dt != STENCIL_F32 && dt != STENCIL_F64) return fail(STENCIL_E_DTYPE, "unknown dtype %d", (int)dt);
  return STENCIL_OK;
}

static const int64_t kMaxExtent = int64_t(1) << 31;

int check_domain(const int64_t* dom) {
  if (!dom) return fail(STENCIL_E_NULL, "domain is NULL");
  for (int d = 0; d < 3; ++d)
    if (dom[d] < 0 || dom[d] >= kMaxExtent)
      return fail(STENCIL_E_SHAPE, "domain[%d] = %lld out of range", d, (long long)dom[d]);
  return STENCIL_OK;
}

bool domain_empty(const int64_t* dom) { return dom[0] == 0 || dom[1] == 0 || dom[2] == 0; }

// Byte range [lo, hi) spanned by a field's allocation.
Span span_of(const stencil_field* f, size_t es) {
  Span s;
  s.lo = reinterpret_cast<uintptr_t>(f->data);
  int64_t last = 0;
  for (int d = 0; d < 3; ++d) last += (f->shape[d] > 0 ? f->shape[d] - 1 : 0) * f->stride[d];
  s.hi = s.lo + (uintptr_t)(last + 1) * es;
  return s;
}

bool overlap(Span a, Span b) { return a.lo < b.hi && b.lo < a.hi; }

int check_field(const char* name, const stencil_field* f, const int64_t* dom, Role role, size_t es) {
  if (!f) return fail(STENCIL_E_NULL, "%s: field is NULL", name);
  if (!f->data) return fail(STENCIL_E_NULL, "%s.data is NULL", name);
  if (reinterpret_cast<uintptr_t>(f->data) % es)
    return fail(STENCIL_E_DTYPE, "%s.data is not aligned to %zu bytes", name, es);
  for (int d = 0; d < 3; ++d) {
    if (f->shape[d] < 0 || f->shape[d] >= kMaxExtent)
      return fail(STENCIL_E_SHAPE, "%s.shape[%d] = %lld out of range", name, d, (long long)f->shape[d]);
    if (f->origin[d] < 0 || f->origin[d] >= kMaxExtent)
      return fail(STENCIL_E_SHAPE, "%s.origin[%d] = %lld out of range", name, d, (long long)f->origin[d]);
  }
  if (f->stride[0] != 1) return fail(STENCIL_E_STRIDE, "%s.stride[0] = %lld, must be 1", name, (long long)f->stride[0]);
  if (f->stride[1] < f->shape[0] || f->stride[1] >= (int64_t(1) << 40))
    return fail(STENCIL_E_STRIDE, "%s.stride[1] = %lld overlaps rows (shape[0] = %lld)", name,
                (long long)f->stride[1], (long long)f->shape[0]);
  if (f->stride[2] < f->stride[1] * f->shape[1] || f->stride[2] >= (int64_t(1) << 46))
    return fail(STENCIL_E_STRIDE, "%s.stride[2] = %lld overlaps planes", name, (long long)f->stride[2]);
  // kernels address within a level with 32-bit byte offsets, and predicate a
  // lane's access off with the offset kOffNone, which must stay outside every
  // window: a level may span at most kOffNone - 16 bytes
  if ((f->stride[1] * f->shape[1] + f->shape[0]) * (int64_t)es > (int64_t)kOffNone - 16)
    return fail(STENCIL_E_UNSUPPORTED, "%s: one level spans %lld bytes, above the 32-bit window limit %lld", name,
                (long long)((f->stride[1] * f->shape[1] + f->shape[0]) * (int64_t)es),
                (long long)((int64_t)kOffNone - 16));
  const int64_t h = (role == ROLE_HALO) ? kHalo : 0;
  for (int d = 0; d < 2; ++d) {
    if (f->origin[d] < h)
      return fail(STENCIL_E_HALO, "%s.origin[%d] = %lld leaves no room for the %lld-point halo", name,
                  d, (long long)f->origin[d], (long long)h);
    if (f->origin[d] + dom[d] + h > f->shape[d])
      return fail(h ? STENCIL_E_HALO : STENCIL_E_SHAPE,
                  "%s: origin[%d] + domain[%d] (+ halo %lld) = %lld exceeds shape %lld", name, d, d,
                  (long long)h, (long long)(f->origin[d] + dom[d] + h), (long long)f->shape[d]);
  }
  const int64_t kext = dom[2] + (role == ROLE_STAGGERED ? 1 : 0);
  if (f->origin[2] + kext > f->shape[2])
    return fail(STENCIL_E_SHAPE, "%s: origin[2] + %lld levels = %lld exceeds shape[2] = %lld", name,
                (long long)kext, (long long)(f->origin[2] + kext), (long long)f->shape[2]);
  return STENCIL_OK;
}

int check_no_alias(const char* oname, Span o, const char* iname, Span in) {
  if (overlap(o, in)) return fail(STENCIL_E_ALIAS, "%s overlaps %s", oname, iname);
  return STENCIL_OK;
}

// ------------------------------------------------------------------ options
// Whether a 128-column tile can run: the fused two-ended step only.
static bool narrow_tile_runs(const ResolvedOpts& r, int op, stencil_dtype dt, const int64_t* dom) {
  return op == STENCIL_OP_STEP && r.impl != STENCIL_IMPL_PLAIN && r.column_store == STENCIL_COLUMN_SPLIT &&
         dom[2] <= split_step_limit((int)esize(dt));
}

ResolvedOpts resolve_opts(const stencil_options* o, stencil_dtype dt, int op, const int64_t* dom) {
  ResolvedOpts r;
  r.impl = o ? o->impl : STENCIL_IMPL_AUTO;
  int32_t ti = 0, tj = 0, col = 0, ord = 0;
  tuning_get(dt, op, dom, &ti, &tj, &col, &ord);
  const bool own_tile = o && o->tile_i;
  r.tile_i = own_tile ? o->tile_i : ti;
  r.tile_j = own_tile ? (o->tile_j ? o->tile_j : kWG / o->tile_i) : tj;
  r.column_store = (o && o->column_store) ? o->column_store : col;
  if (r.column_store == STENCIL_COLUMN_AUTO) {
    if (op == STENCIL_OP_STEP && dom[2] <= split_step_limit((int)esize(dt)))
      r.column_store = STENCIL_COLUMN_SPLIT;
    else
      r.column_store = (dt == STENCIL_F64 && dom[2] > 96) ? STENCIL_COLUMN_OUTBUF : STENCIL_COLUMN_REGISTERS;
  }
  // a tuned 128-column tile where the call does not run the two-ended step
  // (another column store, or columns past its limit) takes the 256-column
  // tile of the same width; a caller's own such tile is refused by the step
  if (!own_tile && !narrow_tile_runs(r, op, dt, dom)) r.tile_j = kWG / r.tile_i;
  r.ws = o ? o->workspace : nullptr;
  r.ws_bytes = o ? o->workspace_bytes : 0;
  r.form = o ? o->hdiff_form : STENCIL_HDIFF_STATED;
  r.kappa = o ? o->coeff_field : nullptr;
  r.order = (o && o->tile_order) ? o->tile_order : ord;
  if (r.order != STENCIL_ORDER_DISPATCH) r.order = STENCIL_ORDER_XCD;
  return r;
}

int check_opts(const stencil_options* o) {
  if (!o) return STENCIL_OK;
  if (o->impl < STENCIL_IMPL_AUTO || o->impl > STENCIL_IMPL_PLAIN)
    return fail(STENCIL_E_ARG, "options.impl = %d unknown", (int)o->impl);
  if (o->tile_i != 0 && !(o->tile_j == 0 && (o->tile_i == 64 || o->tile_i == 32 || o->tile_i == 16)) &&
      !tile_wide(o->tile_i, o->tile_j) && !tile_narrow(o->tile_i, o->tile_j))
    return fail(STENCIL_E_ARG, "options tile %dx%d unsupported (64x4, 32x8, 16x16; 64x2, 32x4, 16x8)",
                (int)o->tile_i, (int)o->tile_j);
  if (o->column_store < 0 || o->column_store > STENCIL_COLUMN_SPLIT)
    return fail(STENCIL_E_ARG, "options.column_store = %d unknown", (int)o->column_store);
  if (o->workspace_bytes && !o->workspace) return fail(STENCIL_E_NULL, "options.workspace is NULL");
  if (o->boundary != STENCIL_BOUNDARY_FROZEN && o->boundary != STENCIL_BOUNDARY_PERIODIC)
    return fail(STENCIL_E_ARG, "options.boundary = %d unknown", (int)o->boundary);
  if (o->hdiff_form != STENCIL_HDIFF_STATED && o->hdiff_form != STENCIL_HDIFF_DAMPING)
    return fail(STENCIL_E_ARG, "options.hdiff_form = %d unknown", (int)o->hdiff_form);
  if (o->tile_order < STENCIL_ORDER_AUTO || o->tile_order > STENCIL_ORDER_DISPATCH)
    return fail(STENCIL_E_ARG, "options.tile_order = %d unknown", (int)o->tile_order);
  return STENCIL_OK;
}

int check_coeff_field(const stencil_options* o, const int64_t* dom, size_t es, const char* oname, Span out) {
  if (!o || !o->coeff_field) return STENCIL_OK;
  TRY(check_field("coeff_field", o->coeff_field, dom, ROLE_INTERIOR, es));
  return check_no_alias(oname, out, "coeff_field", span_of(o->coeff_field, es));
}

// The generalised diffusion in the forward argument block.
template <typename T>
static void apply_variant(StepArgs<T>& A, const ResolvedOpts& r) {
  A.form = r.form;
  if (r.kappa) {
    A.kappa = at_origin<T>(r.kappa);
    A.c_sj = r.kappa->stride[1];
    A.c_sk = r.kappa->stride[2];
  }
}

// ... and in the adjoint's: a scalar coefficient takes the form's sign
// (the damping form is the stated one with the coefficient negated, its
// saved mask already holding the damping decisions); a coefficient field
// leaves the sign in coeff.
template <typename T>
static void apply_variant(AdjArgs<T>& A, const ResolvedOpts& r, double coeff) {
  const double sg = r.form == STENCIL_HDIFF_DAMPING ? -1.0 : 1.0;
  if (r.kappa) {
    A.kappa = at_origin<T>(r.kappa);
    A.c_sj = r.kappa->stride[1];
    A.c_sk = r.kappa->stride[2];
    A.coeff = (T)sg;
  } else {
    A.coeff = (T)(sg * coeff);
  }
}

// Plain-form workspace carve-up: lap, fx, fy, c', d' (each 256-B aligned).
static int64_t r256(int64_t b) { return (b + 255) & ~int64_t(255); }

size_t plain_ws_bytes(size_t es, const int64_t* dom) {
  const int64_t ni = dom[0], nj = dom[1], nk = dom[2];
  return (size_t)(r256((ni + 2) * (nj + 2) * nk * es) + r256((ni + 1) * nj * nk * es) +
                  r256(ni * (nj + 1) * nk * es) + 2 * r256(ni * nj * nk * es));
}

template <typename T>
PlainWs<T> carve_plain(void* ws, const int64_t* dom) {
  const int64_t ni = dom[0], nj = dom[1], nk = dom[2];
  const int64_t es = sizeof(T);
  char* p = static_cast<char*>(ws);
  PlainWs<T> w;
  w.lap = reinterpret_cast<T*>(p);
  p += r256((ni + 2) * (nj + 2) * nk * es);
  w.fx = reinterpret_cast<T*>(p);
  p += r256((ni + 1) * nj * nk * es);
  w.fy = reinterpret_cast<T*>(p);
  p += r256(ni * (nj + 1) * nk * es);
  w.cp = reinterpret_cast<T*>(p);
  p += r256(ni * nj * nk * es);
  w.dp = reinterpret_cast<T*>(p);
  return w;
}

// column-adjoint workspace: lambda (when data_bar is absent) then y and c'
size_t adj_ws_bytes(size_t es, const int64_t* dom, bool need_lam, bool plain) {
  const int64_t n = dom[0] * dom[1] * dom[2];
  return (size_t)((need_lam ? r256(n * es) : 0) + (plain ? 2 * r256(n * es) : 0));
}

// ------------------------------------------------------------------ arg blocks
template <typename T>
StepArgs<T> step_args(const stencil_field* u, const stencil_field* data, const stencil_field* w,
                      stencil_field* out, const int64_t* dom, double coeff, double dt_dz,
                      void* mask) {
  StepArgs<T> A;
  memset(&A, 0, sizeof A);
  if (u) { A.u = at_origin<T>(u); A.u_sj = u->stride[1]; A.u_sk = u->stride[2]; }
  if (data) { A.data = at_origin<T>(data); A.d_sj = data->stride[1]; A.d_sk = data->stride[2]; }
  if (w) { A.w = at_origin<T>(w); A.w_sj = w->stride[1]; A.w_sk = w->stride[2]; }
  if (out) { A.out = at_origin_mut<T>(out); A.o_sj = out->stride[1]; A.o_sk = out->stride[2]; }
  A.mask = static_cast<uint8_t*>(mask);
  A.ml = MaskLayout::make(dom[0], dom[1], dom[2]);
  A.ni = (int)dom[0];
  A.nj = (int)dom[1];
  A.nk = (int)dom[2];
  A.coeff = (T)coeff;
  A.r4 = (T)(0.25 * dt_dz);
  return A;
}

template StepArgs<float> step_args<float>(const stencil_field*, const stencil_field*, const stencil_field*,
                                          stencil_field*, const int64_t*, double, double, void*);
template StepArgs<double> step_args<double>(const stencil_field*, const stencil_field*, const stencil_field*,
                                            stencil_field*, const int64_t*, double, double, void*);

template <typename T>
AdjArgs<T> adj_args(const stencil_field* xbar, const stencil_field* w, T* lam, int64_t l_sj,
                    int64_t l_sk, stencil_field* ubar, const int64_t* dom, double coeff,
                    double dt_dz, const void* mask) {
  AdjArgs<T> A;
  memset(&A, 0, sizeof A);
  if (xbar) { A.xbar = at_origin<T>(xbar); A.x_sj = xbar->stride[1]; A.x_sk = xbar->stride[2]; }
  if (w) { A.w = at_origin<T>(w); A.w_sj = w->stride[1]; A.w_sk = w->stride[2]; }
  A.lam = lam;
  A.l_sj = l_sj;
  A.l_sk = l_sk;
  if (ubar) { A.ubar = at_origin_mut<T>(ubar); A.b_sj = ubar->stride[1]; A.b_sk = ubar->stride[2]; }
  A.mask = static_cast<const uint8_t*>(mask);
  A.ml = MaskLayout::make(dom[0], dom[1], dom[2]);
  A.ni = (int)dom[0];
  A.nj = (int)dom[1];
  A.nk = (int)dom[2];
  A.coeff = (T)coeff;
  A.r4 = (T)(0.25 * dt_dz);
  return A;
}

template AdjArgs<float> adj_args<float>(const stencil_field*, const stencil_field*, float*, int64_t, int64_t,
                                      stencil_field*, const int64_t*, double, double, const void*);
template AdjArgs<double> adj_args<double>(const stencil_field*, const stencil_field*, double*, int64_t, int64_t,
                                        stencil_field*, const int64_t*, double, double, const void*);

// ------------------------------------------------------------------ dispatch
template <typename T>
int run_hdiff(const stencil_field* u, stencil_field* out, const int64_t* dom, double coeff,
              void* mask, const ResolvedOpts& r, hipStream_t s) {
  StepArgs<T> A = step_args<T>(u, nullptr, nullptr, out, dom, coeff, 0.0, mask);
  if (r.impl == STENCIL_IMPL_PLAIN)
    return hip_status(launch_hdiff_plain<T>(A, carve_plain<T>(r.ws, dom), s), "hdiff (plain)");
  apply_variant(A, r);
  return hip_status(launch_hdiff_fused<T>(A, r.tile_i, s), "hdiff (fused)");
}

template <typename T>
int run_vadv(const stencil_field* u, const stencil_field* data, const stencil_field* w,
             stencil_field* out, const int64_t* dom, double dt_dz, const ResolvedOpts& r,
             hipStream_t s) {
  StepArgs<T> A = step_args<T>(u, data, w, out, dom, 0.0, dt_dz, nullptr);
  if (r.impl == STENCIL_IMPL_PLAIN)
    return hip_status(launch_vadv_plain<T>(A, carve_plain<T>(r.ws, dom), s), "vadv (plain)");
  return hip_status(launch_vadv_fused<T>(A, s), "vadv (fused)");
}

template <typename T>
int run_step(const stencil_field* u, const stencil_field* data, const stencil_field* w,
             stencil_field* out, const int64_t* dom, double coeff, double dt_dz, void* mask,
             const ResolvedOpts& r, hipStream_t s) {
  if (r.impl == STENCIL_IMPL_PLAIN) {
    PlainWs<T> ws = carve_plain<T>(r.ws, dom);
    StepArgs<T> A = step_args<T>(u, nullptr, nullptr, out, dom, coeff, 0.0, mask);
    int rc = hip_status(launch_hdiff_plain<T>(A, ws, s), "step (plain hdiff)");
    if (rc) return rc;
    // the diffused field now sits in out's interior: it is the u_k of d_k
    StepArgs<T> B = step_args<T>(out, data, w, out, dom, coeff, dt_dz, nullptr);
    return hip_status(launch_vadv_plain<T>(B, ws, s), "step (plain vadv)");
  }
  StepArgs<T> A = step_args<T>(u, data, w, out, dom, coeff, dt_dz, mask);
  apply_variant(A, r);
  A.order = r.order;
  return hip_status(launch_step_fused<T>(A, r.tile_i, r.tile_j, r.column_store, s), "step (fused)");
}

template <typename T>
int run_hdiff_adjoint(const T* lam, int64_t l_sj, int64_t l_sk, const void* mask,
                      stencil_field* ubar, const int64_t* dom, double coeff, const ResolvedOpts& r,
                      hipStream_t s) {
  AdjArgs<T> A = adj_args<T>(nullptr, nullptr, const_cast<T*>(lam), l_sj, l_sk, ubar, dom, coeff,
                             0.0, (dom[0] == 0 || dom[1] == 0) ? nullptr : mask);
  apply_variant(A, r, coeff);
  return hip_status(launch_hdiff_adjoint<T>(A, s), "hdiff adjoint");
}

template <typename T>
int run_vadv_adjoint(const stencil_field* xbar, const stencil_field* w, T* lam, int64_t l_sj,
                     int64_t l_sk, const int64_t* dom, double dt_dz, const ResolvedOpts& r,
                     void* ws_after_lam, hipStream_t s) {
  AdjArgs<T> A = adj_args<T>(xbar, w, lam, l_sj, l_sk, nullptr, dom, 0.0, dt_dz, nullptr);
  const bool plain = r.impl == STENCIL_IMPL_PLAIN || dom[2] > kMaxFusedNk;
  T* y = nullptr;
  T* c = nullptr;
  if (plain) {
    const int64_t n = dom[0] * dom[1] * dom[2];
    y = static_cast<T*>(ws_after_lam);
    c = reinterpret_cast<T*>(static_cast<char*>(ws_after_lam) + r256(n * (int64_t)sizeof(T)));
  }
  return hip_status(launch_vadv_adjoint<T>(A, plain ? 1 : 0, y, c, s), "vadv adjoint");
}

}  // namespace gt4mi

using namespace gt4mi;

// ====================================================================== C ABI
extern "C" {

int stencil_version(void) { return STENCIL_ABI_VERSION; }

const char* stencil_last_error(void) { return g_err.c_str(); }

int stencil_max_fused_nk(stencil_dtype dtype) {
  (void)dtype;
  return kMaxFusedNk;
}

size_t stencil_mask_bytes(const int64_t domain[3]) {
  if (!domain) return 0;
  for (int d = 0; d < 3; ++d)
    if (domain[d] < 0 || domain[d] >= kMaxExtent) return 0;
  return (size_t)MaskLayout::make(domain[0], domain[1], domain[2]).total;
}

size_t stencil_workspace_bytes(int op, stencil_dtype dtype, const int64_t domain[3],
                               const stencil_options* opts) {
  if (check_dtype(dtype) || check_domain(domain)) return 0;
  const size_t es = esize(dtype);
  const bool plain = (opts && opts->impl == STENCIL_IMPL_PLAIN) || domain[2] > kMaxFusedNk;
  switch (op) {
    case STENCIL_OP_HDIFF:
    case STENCIL_OP_VADV:
    case STENCIL_OP_STEP:
      return plain ? plain_ws_bytes(es, domain) : 0;
    case STENCIL_OP_HDIFF_ADJOINT:
      return 0;
    case STENCIL_OP_VADV_ADJOINT:
      return adj_ws_bytes(es, domain, false, plain);
    case STENCIL_OP_STEP_ADJOINT:
      return adj_ws_bytes(es, domain, true, plain);
    default:
      return 0;
  }
}

static int need_plain_ws(const ResolvedOpts& r, size_t need) {
  if (need == 0) return STENCIL_OK;
  if (!r.ws) return fail(STENCIL_E_WORKSPACE, "this call needs %zu bytes of workspace (options.workspace is NULL)", need);
  if (r.ws_bytes < need)
    return fail(STENCIL_E_WORKSPACE, "workspace of %zu bytes is smaller than the %zu needed", r.ws_bytes, need);
  return STENCIL_OK;
}

static int fused_nk_ok(ResolvedOpts& r, const int64_t* dom) {
  if (r.impl == STENCIL_IMPL_PLAIN) return STENCIL_OK;
  if (dom[2] > kMaxFusedNk) {
    if (r.impl == STENCIL_IMPL_FUSED)
      return fail(STENCIL_E_UNSUPPORTED, "nk = %lld exceeds the fused column limit %d; use STENCIL_IMPL_PLAIN",
                  (long long)dom[2], kMaxFusedNk);
    r.impl = STENCIL_IMPL_PLAIN;
  }
  return STENCIL_OK;
}

int stencil_hdiff(stencil_dtype dtype, const stencil_field* u, stencil_field* out,
                  const int64_t domain[3], double coeff, void* mask, const stencil_options* opts,
                  hipStream_t stream) {
  TRY(check_dtype(dtype));
  TRY(check_domain(domain));
  TRY(check_opts(opts));
  const size_t es = esize(dtype);
  TRY(check_field("u", u, domain, ROLE_HALO, es));
  TRY(check_field("out", out, domain, ROLE_INTERIOR, es));
  TRY(check_no_alias("out", span_of(out, es), "u", span_of(u, es)));
  TRY(check_coeff_field(opts, domain, es, "out", span_of(out, es)));
  if (mask) {
    Span m{reinterpret_cast<uintptr_t>(mask), reinterpret_cast<uintptr_t>(mask) + stencil_mask_bytes(domain)};
    TRY(check_no_alias("mask", m, "u", span_of(u, es)));
    TRY(check_no_alias("mask", m, "out", span_of(out, es)));
    if (opts && opts->coeff_field) TRY(check_no_alias("mask", m, "coeff_field", span_of(opts->coeff_field, es)));
  }
  if (domain_empty(domain)) return ok();
  ResolvedOpts r = resolve_opts(opts, dtype, STENCIL_OP_HDIFF, domain);
  if (variant_opts(opts) && r.impl == STENCIL_IMPL_PLAIN)
    return fail(STENCIL_E_UNSUPPORTED, "the generalised diffusion runs the fused kernels only");
  if (r.impl == STENCIL_IMPL_PLAIN) TRY(need_plain_ws(r, plain_ws_bytes(es, domain)));
  TRY(check_device());
  return dtype == STENCIL_F64 ? run_hdiff<double>(u, out, domain, coeff, mask, r, stream)
                              : run_hdiff<float>(u, out, domain, coeff, mask, r, stream);
}

int stencil_vadv(stencil_dtype dtype, const stencil_field* u, const stencil_field* data,
                 const stencil_field* w, stencil_field* out, const int64_t domain[3], double dt_dz,
                 const stencil_options* opts, hipStream_t stream) {
  TRY(check_dtype(dtype));
  TRY(check_domain(domain));
  TRY(check_opts(opts));
  const size_t es = esize(dtype);
  TRY(check_field("u", u, domain, ROLE_INTERIOR, es));
  TRY(check_field("data", data, domain, ROLE_INTERIOR, es));
  TRY(check_field("w", w, domain, ROLE_STAGGERED, es));
  const bool periodic = opts && opts->boundary == STENCIL_BOUNDARY_PERIODIC;
  TRY(check_field("out", out, domain, periodic ? ROLE_HALO : ROLE_INTERIOR, es));
  const Span so = span_of(out, es);
  TRY(check_no_alias("out", so, "u", span_of(u, es)));
  TRY(check_no_alias("out", so, "data", span_of(data, es)));
  TRY(check_no_alias("out", so, "w", span_of(w, es)));
  if (domain_empty(domain)) return ok();
  ResolvedOpts r = resolve_opts(opts, dtype, STENCIL_OP_VADV, domain);
  TRY(fused_nk_ok(r, domain));
  if (r.impl == STENCIL_IMPL_PLAIN) TRY(need_plain_ws(r, plain_ws_bytes(es, domain)));
  TRY(check_device());
  return dtype == STENCIL_F64 ? run_vadv<double>(u, data, w, out, domain, dt_dz, r, stream)
                              : run_vadv<float>(u, data, w, out, domain, dt_dz, r, stream);
}

int stencil_step(stencil_dtype dtype, const stencil_field* u, const stencil_field* data,
                 const stencil_field* w, stencil_field* out, const int64_t domain[3], double coeff,
                 double dt_dz, void* mask, const stencil_options* opts, hipStream_t stream) {
  TRY(check_dtype(dtype));
  TRY(check_domain(domain));
  TRY(check_opts(opts));
  const size_t es = esize(dtype);
  TRY(check_field("u", u, domain, ROLE_HALO, es));
  TRY(check_field("data", data, domain, ROLE_INTERIOR, es));
  TRY(check_field("w", w, domain, ROLE_STAGGERED, es));
  const bool periodic = opts && opts->boundary == STENCIL_BOUNDARY_PERIODIC;
  TRY(check_field("out", out, domain, periodic ? ROLE_HALO : ROLE_INTERIOR, es));
  const Span so = span_of(out, es);
  TRY(check_no_alias("out", so, "u", span_of(u, es)));
  TRY(check_no_alias("out", so, "data", span_of(data, es)));
  TRY(check_no_alias("out", so, "w", span_of(w, es)));
  if (mask) {
    Span m{reinterpret_cast<uintptr_t>(mask), reinterpret_cast<uintptr_t>(mask) + stencil_mask_bytes(domain)};
    TRY(check_no_alias("mask", m, "u", span_of(u, es)));
    TRY(check_no_alias("mask", m, "out", so));
    TRY(check_no_alias("mask", m, "data", span_of(data, es)));
    TRY(check_no_alias("mask", m, "w", span_of(w, es)));
    if (opts && opts->coeff_field) TRY(check_no_alias("mask", m, "coeff_field", span_of(opts->coeff_field, es)));
  }
  TRY(check_coeff_field(opts, domain, es, "out", so));
  if (domain_empty(domain)) return ok();
  ResolvedOpts r = resolve_opts(opts, dtype, STENCIL_OP_STEP, domain);
  if (variant_opts(opts)) {
    if (r.impl == STENCIL_IMPL_PLAIN)
      return fail(STENCIL_E_UNSUPPORTED, "the generalised diffusion runs the fused kernels only");
    if (domain[2] > split_step_limit((int)es))
      return fail(STENCIL_E_UNSUPPORTED, "the generalised step takes nk <= %d (nk = %lld)",
                  split_step_limit((int)es), (long long)domain[2]);
  }
  TRY(fused_nk_ok(r, domain));
  if (tile_narrow(r.tile_i, r.tile_j) && !narrow_tile_runs(r, STENCIL_OP_STEP, dtype, domain))
    return fail(STENCIL_E_UNSUPPORTED,
                "the %dx%d tile (128 columns) runs the fused two-ended step only (column store SPLIT, nk <= %d)",
                r.tile_i, r.tile_j, split_step_limit((int)es));
  if (r.impl == STENCIL_IMPL_PLAIN) TRY(need_plain_ws(r, plain_ws_bytes(es, domain)));
  TRY(check_device());
  TRY(dtype == STENCIL_F64 ? run_step<double>(u, data, w, out, domain, coeff, dt_dz, mask, r, stream)
                           : run_step<float>(u, data, w, out, domain, coeff, dt_dz, mask, r, stream));
  return periodic ? stencil_halo_update(dtype, out, domain, STENCIL_BOUNDARY_PERIODIC, stream) : ok();
}

int stencil_halo_update(stencil_dtype dtype, stencil_field* f, const int64_t domain[3], int boundary,
                        hipStream_t stream) {
  TRY(check_dtype(dtype));
  TRY(check_domain(domain));
  if (boundary != STENCIL_BOUNDARY_FROZEN && boundary != STENCIL_BOUNDARY_PERIODIC)
    return fail(STENCIL_E_ARG, "boundary = %d unknown", boundary);
  TRY(check_field("f", f, domain, ROLE_HALO, esize(dtype)));
  if (boundary == STENCIL_BOUNDARY_FROZEN || domain_empty(domain)) return ok();
  TRY(check_device());
  const int ni = (int)domain[0], nj = (int)domain[1], nk = (int)domain[2];
  hipError_t e = dtype == STENCIL_F64
                     ? launch_halo_periodic<double>(at_origin_mut<double>(f), f->stride[1], f->stride[2], ni, nj, nk, stream)
                     : launch_halo_periodic<float>(at_origin_mut<float>(f), f->stride[1], f->stride[2], ni, nj, nk, stream);
  return hip_status(e, "periodic halo update");
}

int stencil_hdiff_adjoint(stencil_dtype dtype, const stencil_field* out_bar, const void* mask,
                          stencil_field* u_bar, const int64_t domain[3], double coeff,
                          const stencil_options* opts, hipStream_t stream) {
  TRY(check_dtype(dtype));
  TRY(check_domain(domain));
  TRY(check_opts(opts));
  const size_t es = esize(dtype);
  TRY(check_field("out_bar", out_bar, domain, ROLE_INTERIOR, es));
  TRY(check_field("u_bar", u_bar, domain, ROLE_HALO, es));
  const Span sb = span_of(u_bar, es);
  TRY(check_no_alias("u_bar", sb, "out_bar", span_of(out_bar, es)));
  TRY(check_coeff_field(opts, domain, es, "u_bar", sb));
  if (domain[2] == 0) return ok();
  const bool empty = domain_empty(domain);
  if (!mask && !empty) return fail(STENCIL_E_NULL, "mask is NULL");
  if (mask) {
    Span m{reinterpret_cast<uintptr_t>(mask), reinterpret_cast<uintptr_t>(mask) + stencil_mask_bytes(domain)};
    TRY(check_no_alias("u_bar", sb, "mask", m));
  }
  ResolvedOpts r = resolve_opts(opts, dtype, STENCIL_OP_HDIFF_ADJOINT, domain);
  TRY(check_device());
  if (dtype == STENCIL_F64) {
    return run_hdiff_adjoint<double>(at_origin<double>(out_bar), out_bar->stride[1], out_bar->stride[2],
                                     mask, u_bar, domain, coeff, r, stream);
  }
  return run_hdiff_adjoint<float>(at_origin<float>(out_bar), out_bar->stride[1], out_bar->stride[2],
                                  mask, u_bar, domain, coeff, r, stream);
}

int stencil_vadv_adjoint(stencil_dtype dtype, const stencil_field* x_bar, const stencil_field* w,
                         stencil_field* d_bar, const int64_t domain[3], double dt_dz,
                         const stencil_options* opts, hipStream_t stream) {
  TRY(check_dtype(dtype));
  TRY(check_domain(domain));
  TRY(check_opts(opts));
  const size_t es = esize(dtype);
  TRY(check_field("x_bar", x_bar, domain, ROLE_INTERIOR, es));
  TRY(check_field("w", w, domain, ROLE_STAGGERED, es));
  TRY(check_field("d_bar", d_bar, domain, ROLE_INTERIOR, es));
  const Span sd = span_of(d_bar, es);
  TRY(check_no_alias("d_bar", sd, "x_bar", span_of(x_bar, es)));
  TRY(check_no_alias("d_bar", sd, "w", span_of(w, es)));
  if (domain_empty(domain)) return ok();
  ResolvedOpts r = resolve_opts(opts, dtype, STENCIL_OP_VADV_ADJOINT, domain);
  const bool plain = r.impl == STENCIL_IMPL_PLAIN || domain[2] > kMaxFusedNk;
  if (r.impl == STENCIL_IMPL_FUSED && domain[2] > kMaxFusedNk)
    return fail(STENCIL_E_UNSUPPORTED, "nk = %lld exceeds the fused column limit %d", (long long)domain[2], kMaxFusedNk);
  TRY(need_plain_ws(r, adj_ws_bytes(es, domain, false, plain)));
  TRY(check_device());
  if (dtype == STENCIL_F64)
    return run_vadv_adjoint<double>(x_bar, w, at_origin_mut<double>(d_bar), d_bar->stride[1], d_bar->stride[2],
                                    domain, dt_dz, r, r.ws, stream);
  return run_vadv_adjoint<float>(x_bar, w, at_origin_mut<float>(d_bar), d_bar->stride[1], d_bar->stride[2],
                                 domain, dt_dz, r, r.ws, stream);
}

int stencil_step_adjoint(stencil_dtype dtype, const stencil_field* x_bar, const stencil_field* w,
                         const void* mask, stencil_field* u_bar, stencil_field* data_bar,
                         const int64_t domain[3], double coeff, double dt_dz,
                         const stencil_options* opts, hipStream_t stream) {
  TRY(check_dtype(dtype));
  TRY(check_domain(domain));
  TRY(check_opts(opts));
  const size_t es = esize(dtype);
  TRY(check_field("x_bar", x_bar, domain, ROLE_INTERIOR, es));
  TRY(check_field("w", w, domain, ROLE_STAGGERED, es));
  TRY(check_field("u_bar", u_bar, domain, ROLE_HALO, es));
  const Span sb = span_of(u_bar, es), sx = span_of(x_bar, es), sw = span_of(w, es);
  TRY(check_no_alias("u_bar", sb, "x_bar", sx));
  TRY(check_no_alias("u_bar", sb, "w", sw));
  if (data_bar) {
    TRY(check_field("data_bar", data_bar, domain, ROLE_INTERIOR, es));
    const Span sd = span_of(data_bar, es);
    TRY(check_no_alias("data_bar", sd, "x_bar", sx));
    TRY(check_no_alias("data_bar", sd, "w", sw));
    TRY(check_no_alias("data_bar", sd, "u_bar", sb));
    TRY(check_coeff_field(opts, domain, es, "data_bar", sd));
  }
  TRY(check_coeff_field(opts, domain, es, "u_bar", sb));
  if (domain[2] == 0) return ok();
  const bool empty = domain_empty(domain);
  if (!mask && !empty) return fail(STENCIL_E_NULL, "mask is NULL");
  if (mask) {
    Span m{reinterpret_cast<uintptr_t>(mask), reinterpret_cast<uintptr_t>(mask) + stencil_mask_bytes(domain)};
    TRY(check_no_alias("u_bar", sb, "mask", m));
  }
  ResolvedOpts r = resolve_opts(opts, dtype, STENCIL_OP_STEP_ADJOINT, domain);
  const bool plain = r.impl == STENCIL_IMPL_PLAIN || domain[2] > kMaxFusedNk;
  if (r.impl == STENCIL_IMPL_FUSED && domain[2] > kMaxFusedNk)
    return fail(STENCIL_E_UNSUPPORTED, "nk = %lld exceeds the fused column limit %d", (long long)domain[2], kMaxFusedNk);
  const size_t need = adj_ws_bytes(es, domain, data_bar == nullptr, plain);
  TRY(need_plain_ws(r, need));
  if (r.ws && need) {
    Span swsp{reinterpret_cast<uintptr_t>(r.ws), reinterpret_cast<uintptr_t>(r.ws) + need};
    TRY(check_no_alias("workspace", swsp, "u_bar", sb));
    TRY(check_no_alias("workspace", swsp, "x_bar", sx));
    TRY(check_no_alias("workspace", swsp, "w", sw));
  }
  TRY(check_device());
  const int64_t n = domain[0] * domain[1] * domain[2];
  auto go = [&](auto tag) -> int {
    using T = decltype(tag);
    T* lam;
    int64_t l_sj, l_sk;
    char* rest = static_cast<char*>(r.ws);
    if (data_bar) {
      lam = at_origin_mut<T>(data_bar);
      l_sj = data_bar->stride[1];
      l_sk = data_bar->stride[2];
    } else if (empty) {
      lam = nullptr;  // no interior: the gather reads no lambda, it only zeroes u_bar
      l_sj = l_sk = 0;
    } else {
      lam = static_cast<T*>(r.ws);
      l_sj = domain[0];
      l_sk = domain[0] * domain[1];
      rest += r256(n * (int64_t)sizeof(T));
    }
    if (!empty) TRY(run_vadv_adjoint<T>(x_bar, w, lam, l_sj, l_sk, domain, dt_dz, r, rest, stream));
    return run_hdiff_adjoint<T>(lam, l_sj, l_sk, mask, u_bar, domain, coeff, r, stream);
  };
  return dtype == STENCIL_F64 ? go(double(0)) : go(float(0));
}

}  // extern "C"
