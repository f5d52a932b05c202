// batched.cpp -- the C ABI of the persistent batched launches: per-item
// validation (the single-field rules plus no output of one field touching
// any buffer of another, since all fields run concurrently), the work list
// (fields sorted longest column first, prefix sums of their work items) and
// its upload into the caller's workspace, then one persistent launch per
// kernel.  Workspace layout, each part 256-byte aligned:
//   forward:  [header + prefix][argument blocks]
//   adjoint:  [column table][horizontal table][lambda of items without data_bar]
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/stencil.h"
#include "api_internal.hpp"
#include "launch.hpp"

namespace gt4mi {
namespace {

constexpr int kMaxBatch = 1024;  // fields per call (keeps the O(n^2) alias check cheap)
constexpr int kWsAlign = 256;

int64_t r256(int64_t b) { return MaskLayout::round256(b); }

// bytes of one table: header and prefix[n + 1], then n argument blocks
int64_t table_head_bytes(int n) { return r256((int64_t)sizeof(BatchHeader) + 4 * ((int64_t)n + 1)); }
int64_t table_bytes(int n, size_t arg_bytes) { return table_head_bytes(n) + r256((int64_t)n * (int64_t)arg_bytes); }

size_t arg_bytes(stencil_dtype dt, bool adj) {
  if (dt == STENCIL_F64) return adj ? sizeof(AdjArgs<double>) : sizeof(StepArgs<double>);
  return adj ? sizeof(AdjArgs<float>) : sizeof(StepArgs<float>);
}

int64_t lam_bytes(size_t es, const int64_t* dom) { return r256(dom[0] * dom[1] * dom[2] * (int64_t)es); }

Span mask_span(const void* mask, const int64_t* dom) {
  const uintptr_t p = reinterpret_cast<uintptr_t>(mask);
  return Span{p, mask ? p + stencil_mask_bytes(dom) : p};
}

// Tile width of one field of a forward batch (tiles of nt columns): the
// caller's for every field, else the tuning table's entry for the field's
// size class, else the width with the least cost: the lanes its tiles span
// on the field (idle lanes on the ragged edges included) times the width's
// cost per lane relative to 64-wide tiles, as the single-field step
// measures it at 512x512x80 (FP64: 32 as fast, 16 6% slower; FP32: 32 8%,
// 16 25% slower).  Ties go to the wider tile.
int field_tile_i(const stencil_options* o, stencil_dtype dt, const int64_t* dom, int nt) {
  if (o && o->tile_i) return o->tile_i;
  int32_t ti = 64, tj = 4, col = 0, ord = 0;
  if (tuning_get(dt, STENCIL_OP_STEP, dom, &ti, &tj, &col, &ord)) return (ti == 16 || ti == 32) ? ti : 64;
  static const int kPerMille[2][3] = {{1000, 1080, 1250}, {1000, 1000, 1060}};  // [FP32, FP64][64, 32, 16]
  const int* fac = kPerMille[dt == STENCIL_F64 ? 1 : 0];
  int best = 64;
  int64_t least = -1;
  for (int c = 0; c < 3; ++c) {
    const int w = 64 >> c, h = nt / w;
    const int64_t cost = (dom[0] + w - 1) / w * w * ((dom[1] + h - 1) / h * h) * fac[c];
    if (least < 0 || cost < least) least = cost, best = w;
  }
  return best;
}

int check_batch_args(stencil_dtype dtype, int n, const void* items, const stencil_options* opts) {
  TRY(check_dtype(dtype));
  if (n < 0 || n > kMaxBatch) return fail(STENCIL_E_ARG, "batch of %d fields (0..%d)", n, kMaxBatch);
  if (n > 0 && !items) return fail(STENCIL_E_NULL, "items is NULL");
  TRY(check_opts(opts));
  if (opts && opts->impl == STENCIL_IMPL_PLAIN)
    return fail(STENCIL_E_UNSUPPORTED, "the batched launch runs the fused kernels only");
  if (opts && opts->boundary != STENCIL_BOUNDARY_FROZEN)
    return fail(STENCIL_E_UNSUPPORTED, "the batched launch leaves halos frozen (use stencil_halo_update)");
  if (variant_opts(opts))
    return fail(STENCIL_E_UNSUPPORTED, "the batched launch runs the stated diffusion with a scalar coefficient");
  return STENCIL_OK;
}

// Writes of one item against every buffer of every other item.
int check_cross_alias(const std::vector<ItemSpans>& sp) {
  const size_t n = sp.size();
  for (size_t a = 0; a < n; ++a)
    for (const Span& w : sp[a].wr) {
      if (w.lo == w.hi) continue;
      for (size_t b = 0; b < n; ++b) {
        if (b == a) continue;
        for (const Span& o : sp[b].wr)
          if (overlap(w, o)) return fail(STENCIL_E_ALIAS, "an output of item %zu overlaps an output of item %zu", a, b);
        for (const Span& o : sp[b].rd)
          if (overlap(w, o)) return fail(STENCIL_E_ALIAS, "an output of item %zu overlaps an input of item %zu", a, b);
      }
    }
  return STENCIL_OK;
}

int check_workspace(void* ws, size_t ws_bytes, size_t need, const std::vector<ItemSpans>& sp) {
  if (need == 0) return STENCIL_OK;
  if (!ws) return fail(STENCIL_E_WORKSPACE, "the batch needs %zu bytes of workspace (ws is NULL)", need);
  if (ws_bytes < need) return fail(STENCIL_E_WORKSPACE, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(ws) % kWsAlign)
    return fail(STENCIL_E_WORKSPACE, "workspace must be %d-byte aligned", kWsAlign);
  const Span s{reinterpret_cast<uintptr_t>(ws), reinterpret_cast<uintptr_t>(ws) + need};
  for (size_t a = 0; a < sp.size(); ++a) {
    for (const Span& o : sp[a].wr)
      if (overlap(s, o)) return fail(STENCIL_E_ALIAS, "the workspace overlaps an output of item %zu", a);
    for (const Span& o : sp[a].rd)
      if (overlap(s, o)) return fail(STENCIL_E_ALIAS, "the workspace overlaps an input of item %zu", a);
  }
  return STENCIL_OK;
}

int check_item_nk(const int64_t* dom) {
  if (dom[2] > kMaxBatchedNk)
    return fail(STENCIL_E_UNSUPPORTED, "nk = %lld exceeds the batched column limit %d", (long long)dom[2],
                kMaxBatchedNk);
  return STENCIL_OK;
}

// Per-item validation of a forward batch; fills the spans.
int check_forward_items(stencil_dtype dtype, int n, const stencil_batch_item* it, std::vector<ItemSpans>& sp) {
  const size_t es = esize(dtype);
  sp.resize(n);
  for (int a = 0; a < n; ++a) {
    const stencil_batch_item& x = it[a];
    const int64_t* dom = x.domain;
    int rc = check_domain(dom);
    if (!rc) rc = check_field("u", &x.u, dom, ROLE_HALO, es);
    if (!rc) rc = check_field("data", &x.data, dom, ROLE_INTERIOR, es);
    if (!rc) rc = check_field("w", &x.w, dom, ROLE_STAGGERED, es);
    if (!rc) rc = check_field("out", &x.out, dom, ROLE_INTERIOR, es);
    if (!rc) rc = check_item_nk(dom);
    ItemSpans& s = sp[a];
    if (!rc) {
      s.rd = {span_of(&x.u, es), span_of(&x.data, es), span_of(&x.w, es)};
      s.wr = {span_of(&x.out, es), mask_span(x.mask, dom)};
      for (const Span& w : s.wr)
        for (const Span& r : s.rd)
          if (!rc && overlap(w, r)) rc = fail(STENCIL_E_ALIAS, "an output of the item overlaps one of its inputs");
      if (!rc && overlap(s.wr[0], s.wr[1])) rc = fail(STENCIL_E_ALIAS, "mask overlaps out");
    }
    if (rc) return fail(rc, "item %d: %s", a, stencil_last_error());
  }
  return check_cross_alias(sp);
}

int check_adjoint_items(stencil_dtype dtype, int n, const stencil_batch_adjoint_item* it, std::vector<ItemSpans>& sp) {
  const size_t es = esize(dtype);
  sp.resize(n);
  for (int a = 0; a < n; ++a) {
    const stencil_batch_adjoint_item& x = it[a];
    const int64_t* dom = x.domain;
    int rc = check_domain(dom);
    if (!rc) rc = check_field("x_bar", &x.x_bar, dom, ROLE_INTERIOR, es);
    if (!rc) rc = check_field("w", &x.w, dom, ROLE_STAGGERED, es);
    if (!rc) rc = check_field("u_bar", &x.u_bar, dom, ROLE_HALO, es);
    if (!rc && x.data_bar.data) rc = check_field("data_bar", &x.data_bar, dom, ROLE_INTERIOR, es);
    if (!rc) rc = check_item_nk(dom);
    if (!rc && !x.mask && dom[2] > 0 && !domain_empty(dom)) rc = fail(STENCIL_E_NULL, "mask is NULL");
    ItemSpans& s = sp[a];
    if (!rc) {
      s.rd = {span_of(&x.x_bar, es), span_of(&x.w, es), mask_span(x.mask, dom)};
      s.wr = {span_of(&x.u_bar, es)};
      if (x.data_bar.data) s.wr.push_back(span_of(&x.data_bar, es));
      for (const Span& w : s.wr)
        for (const Span& r : s.rd)
          if (!rc && overlap(w, r)) rc = fail(STENCIL_E_ALIAS, "an output of the item overlaps one of its inputs");
      if (!rc && s.wr.size() == 2 && overlap(s.wr[0], s.wr[1])) rc = fail(STENCIL_E_ALIAS, "data_bar overlaps u_bar");
    }
    if (rc) return fail(rc, "item %d: %s", a, stencil_last_error());
  }
  return check_cross_alias(sp);
}

// Items with work, longest column first (ties by index, so the order is
// deterministic).
template <typename Item>
std::vector<int> lpt_order(int n, const Item* it, bool (*has_work)(const int64_t*)) {
  std::vector<int> ord;
  for (int a = 0; a < n; ++a)
    if (has_work(it[a].domain)) ord.push_back(a);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return it[x].domain[2] > it[y].domain[2]; });
  return ord;
}

bool interior_work(const int64_t* d) { return !domain_empty(d); }
bool halo_work(const int64_t* d) { return d[2] > 0; }

// Writes one table (header, prefix, argument blocks) into blob at off.
template <typename Args>
int32_t write_table(std::vector<uint8_t>& blob, size_t off, const std::vector<Args>& args,
                    const std::vector<int32_t>& items) {
  const int n = (int)args.size();
  BatchHeader h;
  memset(&h, 0, sizeof h);
  h.n = n;
  std::vector<int32_t> prefix(n + 1, 0);
  for (int e = 0; e < n; ++e) prefix[e + 1] = prefix[e] + items[e];
  h.total = prefix[n];
  uint8_t* p = blob.data() + off;
  memcpy(p, &h, sizeof h);
  memcpy(p + sizeof h, prefix.data(), 4 * (n + 1));
  if (n) memcpy(p + table_head_bytes(n), args.data(), n * sizeof(Args));
  return h.total;
}

// ---------------------------------------------------------------- forward
// FP64 fields whose columns exceed kBatchedShortNk levels run in a launch of
// their own (128-column tiles, e and f in VGPRs); the rest share one launch
// in the 40-level class.  FP32 fields all run in one launch (the 72-level
// class): splitting them by class was measured slower.
bool long_class(stencil_dtype dt, const int64_t* d) { return dt == STENCIL_F64 && d[2] > kBatchedShortNk; }

// Table sizes of the forward batch: [short group, long group].
void forward_groups(stencil_dtype dt, int n, const stencil_batch_item* it, int m[2]) {
  m[0] = m[1] = 0;
  for (int a = 0; a < n; ++a)
    if (interior_work(it[a].domain)) ++m[long_class(dt, it[a].domain) ? 1 : 0];
}

template <typename T>
int run_step_batched(int n, const stencil_batch_item* it, void* ws, const stencil_options* opts, hipStream_t s) {
  constexpr stencil_dtype dt = sizeof(T) == 8 ? STENCIL_F64 : STENCIL_F32;
  const std::vector<int> ord = lpt_order(n, it, interior_work);
  if (ord.empty()) return ok();
  char* base = static_cast<char*>(ws);
  int64_t off = 0;
  // the long group first: its columns are the longest (longest work first)
  for (int g = 1; g >= 0; --g) {
    const bool long_tiles = g == 1;  // FP64 long columns: 128-column tiles
    const int nt = long_tiles ? kSplitLongNT : kWG;
    std::vector<StepArgs<T>> args;
    std::vector<int32_t> items;
    bool any_mask = false;
    int64_t total = 0;
    for (int a : ord) {
      const stencil_batch_item& x = it[a];
      if (long_class(dt, x.domain) != (g == 1)) continue;
      StepArgs<T> A = step_args<T>(&x.u, &x.data, &x.w, const_cast<stencil_field*>(&x.out), x.domain, x.coeff,
                                   x.dt_dz, x.mask);
      A.tile_i = field_tile_i(opts, dt, x.domain, nt);
      const int tile_j = nt / A.tile_i;
      A.tiles_i = (A.ni + A.tile_i - 1) / A.tile_i;
      A.ntiles = A.tiles_i * ((A.nj + tile_j - 1) / tile_j);
      args.push_back(A);
      items.push_back(A.ntiles);
      total += A.ntiles;
      any_mask |= x.mask != nullptr;
    }
    const int m = (int)args.size();
    if (m == 0) continue;
    if (total > INT32_MAX / 2) return fail(STENCIL_E_UNSUPPORTED, "batch of %lld tiles is too large", (long long)total);
    std::vector<uint8_t> blob((size_t)table_bytes(m, sizeof(StepArgs<T>)), 0);
    write_table(blob, 0, args, items);
    TRY(hip_status(launch_upload(base + off, blob.data(), blob.size(), s), "batched table upload"));
    BatchHeader* h = reinterpret_cast<BatchHeader*>(base + off);
    const auto* ent = reinterpret_cast<const StepArgs<T>*>(base + off + table_head_bytes(m));
    if constexpr (sizeof(T) == 8) {
      if (long_tiles) {
        TRY(hip_status(launch_step_batched_long<T>(h, ent, (int)total, any_mask, s), "step (batched, long)"));
        off += (int64_t)blob.size();
        continue;
      }
    }
    TRY(hip_status(launch_step_batched<T>(h, ent, (int)total, any_mask, s), "step (batched)"));
    off += (int64_t)blob.size();
  }
  return ok();
}

// ---------------------------------------------------------------- adjoint
size_t adjoint_ws(stencil_dtype dt, int n, const stencil_batch_adjoint_item* it) {
  int mv = 0, mh = 0;
  int64_t lam = 0;
  for (int a = 0; a < n; ++a) {
    const int64_t* d = it[a].domain;
    if (interior_work(d)) {
      ++mv;
      if (!it[a].data_bar.data) lam += lam_bytes(esize(dt), d);
    }
    if (halo_work(d)) ++mh;
  }
  if (mh == 0) return 0;
  return (size_t)(table_bytes(mv, arg_bytes(dt, false)) + table_bytes(mh, arg_bytes(dt, true)) + lam);
}

template <typename T>
int run_step_adjoint_batched(int n, const stencil_batch_adjoint_item* it, void* ws, hipStream_t s) {
  const std::vector<int> vord = lpt_order(n, it, interior_work);
  const std::vector<int> hord = lpt_order(n, it, halo_work);
  if (hord.empty()) return ok();
  const int mv = (int)vord.size(), mh = (int)hord.size();
  char* base = static_cast<char*>(ws);
  const int64_t vbytes = table_bytes(mv, sizeof(StepArgs<T>));
  const int64_t hbytes = table_bytes(mh, sizeof(AdjArgs<T>));

  // lambda of each item: data_bar, else a workspace slice (dense, ni x nj x nk)
  std::vector<T*> lam(n, nullptr);
  std::vector<int64_t> lsj(n, 0), lsk(n, 0);
  int64_t lam_off = vbytes + hbytes;
  for (int a = 0; a < n; ++a) {
    const stencil_batch_adjoint_item& x = it[a];
    const int64_t* d = x.domain;
    if (!interior_work(d)) continue;
    if (x.data_bar.data) {
      lam[a] = at_origin_mut<T>(const_cast<stencil_field*>(&x.data_bar));
      lsj[a] = x.data_bar.stride[1];
      lsk[a] = x.data_bar.stride[2];
    } else {
      lam[a] = reinterpret_cast<T*>(base + lam_off);
      lsj[a] = d[0];
      lsk[a] = d[0] * d[1];
      lam_off += lam_bytes(sizeof(T), d);
    }
  }

  // column adjoints: 64 x 4 column tiles
  std::vector<StepArgs<T>> vargs(mv);
  std::vector<int32_t> vitems(mv);
  int64_t vtotal = 0;
  for (int e = 0; e < mv; ++e) {
    const int a = vord[e];
    const stencil_batch_adjoint_item& x = it[a];
    StepArgs<T> C = step_args<T>(&x.x_bar, nullptr, &x.w, nullptr, x.domain, 0.0, x.dt_dz, nullptr);
    C.out = lam[a];
    C.o_sj = lsj[a];
    C.o_sk = lsk[a];
    C.tiles_i = (C.ni + 63) / 64;
    C.ntiles = C.tiles_i * ((C.nj + 3) / 4);
    vargs[e] = C;
    vitems[e] = C.ntiles;
    vtotal += C.ntiles;
  }

  // horizontal gathers: groups of strips over the padded domain, one level per item
  std::vector<AdjArgs<T>> hargs(mh);
  for (int e = 0; e < mh; ++e) {
    const int a = hord[e];
    const stencil_batch_adjoint_item& x = it[a];
    const bool empty = domain_empty(x.domain);
    AdjArgs<T> A = adj_args<T>(nullptr, nullptr, lam[a], lsj[a], lsk[a], const_cast<stencil_field*>(&x.u_bar),
                               x.domain, x.coeff, 0.0, empty ? nullptr : x.mask);
    const int out_i = sizeof(T) == 4 ? kStripOut2 : kStripOut;  // FP32: two columns per lane
    A.tiles_i = (A.ni + 4 + out_i - 1) / out_i;
    A.ntiles = A.tiles_i * ((A.nj + 4 + strip_rows<T>() - 1) / strip_rows<T>());  // strips
    hargs[e] = A;
  }
  auto groups = [](const AdjArgs<T>& A) { return (int64_t)(A.ntiles + kStripsPerWG - 1) / kStripsPerWG; };
  std::vector<int32_t> hitems(mh);
  int64_t htotal = 0;
  for (int e = 0; e < mh; ++e) {
    const int64_t c = groups(hargs[e]) * hargs[e].nk;
    if (c > INT32_MAX / 2) return fail(STENCIL_E_UNSUPPORTED, "batch too large");
    hitems[e] = (int32_t)c;
    htotal += c;
  }
  if (vtotal > INT32_MAX / 2 || htotal > INT32_MAX / 2) return fail(STENCIL_E_UNSUPPORTED, "batch too large");

  std::vector<uint8_t> blob((size_t)(vbytes + hbytes), 0);
  write_table(blob, 0, vargs, vitems);
  write_table(blob, (size_t)vbytes, hargs, hitems);
  TRY(hip_status(launch_upload(ws, blob.data(), blob.size(), s), "batched table upload"));
  if (vtotal > 0) {
    BatchHeader* h = reinterpret_cast<BatchHeader*>(base);
    const auto* ent = reinterpret_cast<const StepArgs<T>*>(base + table_head_bytes(mv));
    TRY(hip_status(launch_vadj_batched<T>(h, ent, (int)vtotal, s), "vadv adjoint (batched)"));
  }
  BatchHeader* h = reinterpret_cast<BatchHeader*>(base + vbytes);
  const auto* ent = reinterpret_cast<const AdjArgs<T>*>(base + vbytes + table_head_bytes(mh));
  return hip_status(launch_hadj_batched<T>(h, ent, (int)htotal, s), "hdiff adjoint (batched)");
}

}  // namespace

int check_step_batch(stencil_dtype dtype, int n, const stencil_batch_item* items, const stencil_options* opts,
                     std::vector<ItemSpans>& spans) {
  TRY(check_batch_args(dtype, n, items, opts));
  return check_forward_items(dtype, n, items, spans);
}

int launch_step_batch(stencil_dtype dtype, int n, const stencil_batch_item* items, void* ws,
                      const stencil_options* opts, hipStream_t stream) {
  return dtype == STENCIL_F64 ? run_step_batched<double>(n, items, ws, opts, stream)
                              : run_step_batched<float>(n, items, ws, opts, stream);
}

}  // namespace gt4mi

using namespace gt4mi;

extern "C" {

size_t stencil_batch_workspace_bytes(stencil_dtype dtype, int n, const stencil_batch_item* items) {
  if (check_dtype(dtype) || n <= 0 || n > kMaxBatch || !items) return 0;
  int m[2];
  forward_groups(dtype, n, items, m);
  int64_t b = 0;
  for (int g = 0; g < 2; ++g)
    if (m[g]) b += table_bytes(m[g], arg_bytes(dtype, false));
  return (size_t)b;
}

size_t stencil_batch_adjoint_workspace_bytes(stencil_dtype dtype, int n, const stencil_batch_adjoint_item* items) {
  if (check_dtype(dtype) || n <= 0 || n > kMaxBatch || !items) return 0;
  return adjoint_ws(dtype, n, items);
}

int stencil_step_batched(stencil_dtype dtype, int n, const stencil_batch_item* items, void* ws, size_t ws_bytes,
                         const stencil_options* opts, hipStream_t stream) {
  std::vector<ItemSpans> sp;
  TRY(check_step_batch(dtype, n, items, opts, sp));
  const size_t need = stencil_batch_workspace_bytes(dtype, n, items);
  TRY(check_workspace(ws, ws_bytes, need, sp));
  if (need == 0) return ok();
  TRY(check_device());
  return launch_step_batch(dtype, n, items, ws, opts, stream);
}

int stencil_step_adjoint_batched(stencil_dtype dtype, int n, const stencil_batch_adjoint_item* items, void* ws,
                                 size_t ws_bytes, const stencil_options* opts, hipStream_t stream) {
  TRY(check_batch_args(dtype, n, items, opts));
  std::vector<ItemSpans> sp;
  TRY(check_adjoint_items(dtype, n, items, sp));
  const size_t need = n ? adjoint_ws(dtype, n, items) : 0;
  TRY(check_workspace(ws, ws_bytes, need, sp));
  if (need == 0) return ok();
  TRY(check_device());
  return dtype == STENCIL_F64 ? run_step_adjoint_batched<double>(n, items, ws, stream)
                              : run_step_adjoint_batched<float>(n, items, ws, stream);
}

}  // extern "C"
