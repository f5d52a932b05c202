// tune.cpp -- the autotuner and its process-wide tuning table.
//
// A tuning entry is keyed by (dtype, op, nk class, area class) and holds the
// horizontal tile (64x4, 32x8 or 16x16) and the column store of the fused
// kernels.  stencil_autotune times every candidate on scratch fields of the
// requested size; the table persists as JSON (an analogue of the paper's
// build cache, Sec. 2.3, keyed by size class instead of source fingerprint).
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/stencil.h"
#include "api_internal.hpp"
#include "launch.hpp"

namespace gt4mi {

struct TuneKey {
  int dtype, op, nkc, areac;
  bool operator<(const TuneKey& o) const {
    return std::tie(dtype, op, nkc, areac) < std::tie(o.dtype, o.op, o.nkc, o.areac);
  }
};
struct TuneVal {
  int tile_i, tile_j, col;
  double us;
};

static std::mutex g_mu;
static std::map<TuneKey, TuneVal> g_table;

static int nk_class(int64_t nk) { return (int)((nk + 15) / 16); }
static int area_class(int64_t ni, int64_t nj) {
  const int64_t a = ni * nj;
  return a < 128 * 128 ? 0 : (a < 256 * 256 ? 1 : 2);
}

void tuning_get(stencil_dtype dt, int op, const int64_t* dom, int32_t* ti, int32_t* tj, int32_t* col) {
  TuneKey k{(int)dt, op, nk_class(dom[2]), area_class(dom[0], dom[1])};
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(k);
  if (it != g_table.end()) {
    *ti = it->second.tile_i;
    *tj = it->second.tile_j;
    *col = it->second.col;
  } else {
    *ti = 64;
    *tj = 4;
    *col = STENCIL_COLUMN_AUTO;
  }
}

}  // namespace gt4mi

using namespace gt4mi;

namespace {

struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  void* alloc(size_t b) {
    void* p = nullptr;
    if (hipMalloc(&p, b ? b : 256) != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return p;
  }
};

stencil_field make_field(void* p, int64_t ni, int64_t nj, int64_t nk, int64_t halo, int64_t kextra) {
  stencil_field f;
  f.data = p;
  f.shape[0] = ni + 2 * halo;
  f.shape[1] = nj + 2 * halo;
  f.shape[2] = nk + kextra;
  f.stride[0] = 1;
  f.stride[1] = f.shape[0];
  f.stride[2] = f.shape[0] * f.shape[1];
  f.origin[0] = halo;
  f.origin[1] = halo;
  f.origin[2] = 0;
  return f;
}

}  // namespace

extern "C" {

int stencil_autotune(stencil_dtype dtype, int op, const int64_t domain[3], int reps, double* best_us) {
  if (check_dtype(dtype)) return STENCIL_E_DTYPE;
  if (int rc = check_domain(domain)) return rc;
  if (domain_empty(domain)) return fail(STENCIL_E_SHAPE, "cannot tune an empty domain");
  // the adjoints' gather walks fixed strips and their column solve has no
  // tile: only the forward kernels have a tile to choose
  if (op != STENCIL_OP_STEP && op != STENCIL_OP_HDIFF)
    return fail(STENCIL_E_ARG, "op %d has no tile choice to tune", op);
  if (reps <= 0) reps = 5;
  if (int rc = check_device()) return rc;
  const int64_t ni = domain[0], nj = domain[1], nk = domain[2];
  const size_t es = esize(dtype);
  const size_t padded = (size_t)((ni + 4) * (nj + 4) * nk) * es;
  const size_t inter = (size_t)(ni * nj * nk) * es;
  const size_t stag = (size_t)(ni * nj * (nk + 1)) * es;
  Scratch sc;
  void* pu = sc.alloc(padded);
  void* po = sc.alloc(padded);
  void* pd = sc.alloc(inter);
  void* pw = sc.alloc(stag);
  void* pm = sc.alloc(stencil_mask_bytes(domain));
  const size_t wsb = stencil_workspace_bytes(op, dtype, domain, nullptr);
  void* pws = wsb ? sc.alloc(wsb) : nullptr;
  if (!pu || !po || !pd || !pw || !pm || (wsb && !pws))
    return fail(STENCIL_E_HIP, "autotune: scratch allocation failed");
  hipStream_t s;
  if (hipStreamCreate(&s) != hipSuccess) return fail(STENCIL_E_HIP, "autotune: stream");
  auto fill = [&](void* p, size_t bytes, double lo, double hi, uint32_t seed) {
    const int64_t n = (int64_t)(bytes / es);
    if (dtype == STENCIL_F64) launch_fill_pattern<double>((double*)p, n, lo, hi, seed, s);
    else launch_fill_pattern<float>((float*)p, n, (float)lo, (float)hi, seed, s);
  };
  fill(pu, padded, 0.0, 1.0, 1u);
  fill(po, padded, 0.0, 1.0, 2u);
  fill(pd, inter, -0.1, 0.1, 3u);
  fill(pw, stag, -1.0, 1.0, 4u);
  stencil_field u = make_field(pu, ni, nj, nk, 2, 0), out = make_field(po, ni, nj, nk, 2, 0);
  stencil_field data = make_field(pd, ni, nj, nk, 0, 0), w = make_field(pw, ni, nj, nk, 0, 1);
  int rc = 0;
  struct Cand {
    int ti, tj, col;
  };
  std::vector<Cand> cands;
  for (int t : {64, 32, 16}) {
    if (op == STENCIL_OP_STEP) {
      if (nk <= split_step_limit((int)(dtype == STENCIL_F64 ? 8 : 4))) cands.push_back({t, 256 / t, STENCIL_COLUMN_SPLIT});
      if (dtype == STENCIL_F32 || nk <= 96) cands.push_back({t, 256 / t, STENCIL_COLUMN_REGISTERS});
      if (dtype == STENCIL_F64) cands.push_back({t, 256 / t, STENCIL_COLUMN_OUTBUF});
    } else {
      cands.push_back({t, 256 / t, STENCIL_COLUMN_AUTO});  // hdiff
    }
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  double best = 1e300;
  Cand bc = cands[0];
  for (const Cand& c : cands) {
    stencil_options o;
    memset(&o, 0, sizeof o);
    o.impl = STENCIL_IMPL_FUSED;
    o.tile_i = c.ti;
    o.tile_j = c.tj;
    o.column_store = c.col;
    o.workspace = pws;
    o.workspace_bytes = wsb;
    // the stated hdiff walks fixed strips; the tile is the generalised
    // diffusion's, so that is the form timed
    if (op == STENCIL_OP_HDIFF) o.hdiff_form = STENCIL_HDIFF_DAMPING;
    auto run = [&]() -> int {
      switch (op) {
        case STENCIL_OP_STEP: return stencil_step(dtype, &u, &data, &w, &out, domain, 0.025, 0.5, pm, &o, s);
        default: return stencil_hdiff(dtype, &u, &out, domain, 0.025, pm, &o, s);
      }
    };
    rc = run();  // warm-up
    if (rc) break;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && !rc; ++r) rc = run();
    (void)hipEventRecord(e1, s);
    if (rc) break;
    if (hipEventSynchronize(e1) != hipSuccess) {
      rc = fail(STENCIL_E_HIP, "autotune: event sync");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double us = 1000.0 * ms / reps;
    if (us < best) {
      best = us;
      bc = c;
    }
  }
  (void)hipStreamSynchronize(s);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[TuneKey{(int)dtype, op, nk_class(nk), area_class(ni, nj)}] = TuneVal{bc.ti, bc.tj, bc.col, best};
  }
  if (best_us) *best_us = best;
  return STENCIL_OK;
}

int stencil_tuning_lookup(stencil_dtype dtype, int op, const int64_t domain[3], int32_t* tile_i,
                          int32_t* tile_j, int32_t* column_store) {
  if (int rc = check_dtype(dtype)) return rc;
  if (int rc = check_domain(domain)) return rc;
  if (!tile_i || !tile_j || !column_store) return fail(STENCIL_E_NULL, "output pointer is NULL");
  tuning_get(dtype, op, domain, tile_i, tile_j, column_store);
  return STENCIL_OK;
}

int stencil_clear_tuning(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
  return STENCIL_OK;
}

int stencil_save_tuning(const char* path) {
  if (!path) return fail(STENCIL_E_NULL, "path is NULL");
  FILE* f = fopen(path, "w");
  if (!f) return fail(STENCIL_E_ARG, "cannot open %s for writing", path);
  std::lock_guard<std::mutex> lk(g_mu);
  fprintf(f, "{\"arch\": \"gfx950\", \"version\": %d, \"entries\": [\n", STENCIL_ABI_VERSION);
  size_t n = 0;
  for (const auto& kv : g_table) {
    fprintf(f,
            "  {\"dtype\": %d, \"op\": %d, \"nk_class\": %d, \"area_class\": %d, \"tile_i\": %d, "
            "\"tile_j\": %d, \"column_store\": %d, \"us\": %.3f}%s\n",
            kv.first.dtype, kv.first.op, kv.first.nkc, kv.first.areac, kv.second.tile_i,
            kv.second.tile_j, kv.second.col, kv.second.us, (++n < g_table.size()) ? "," : "");
  }
  fprintf(f, "]}\n");
  fclose(f);
  return STENCIL_OK;
}

static bool read_int(const char* obj, const char* end, const char* key, int* v) {
  char pat[64];
  snprintf(pat, sizeof pat, "\"%s\":", key);
  const char* p = strstr(obj, pat);
  if (!p || p >= end) return false;
  p += strlen(pat);
  char* e = nullptr;
  long x = strtol(p, &e, 10);
  if (e == p) return false;
  *v = (int)x;
  return true;
}

int stencil_load_tuning(const char* path) {
  if (!path) return fail(STENCIL_E_NULL, "path is NULL");
  FILE* f = fopen(path, "r");
  if (!f) return fail(STENCIL_E_ARG, "cannot open %s", path);
  std::string s;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
  fclose(f);
  if (s.find("\"arch\": \"gfx950\"") == std::string::npos)
    return fail(STENCIL_E_ARG, "%s is not a gfx950 tuning table", path);
  const char* p = strstr(s.c_str(), "\"entries\"");
  if (!p) return fail(STENCIL_E_ARG, "%s has no entries", path);
  std::map<TuneKey, TuneVal> t;
  while ((p = strchr(p, '{')) != nullptr) {
    const char* e = strchr(p, '}');
    if (!e) return fail(STENCIL_E_ARG, "%s: unterminated entry", path);
    TuneKey k;
    TuneVal v;
    v.us = 0.0;
    if (!read_int(p, e, "dtype", &k.dtype) || !read_int(p, e, "op", &k.op) ||
        !read_int(p, e, "nk_class", &k.nkc) || !read_int(p, e, "area_class", &k.areac) ||
        !read_int(p, e, "tile_i", &v.tile_i) || !read_int(p, e, "tile_j", &v.tile_j) ||
        !read_int(p, e, "column_store", &v.col))
      return fail(STENCIL_E_ARG, "%s: malformed entry", path);
    if (!((v.tile_i == 64 && v.tile_j == 4) || (v.tile_i == 32 && v.tile_j == 8) ||
          (v.tile_i == 16 && v.tile_j == 16)) ||
        v.col < 0 || v.col > STENCIL_COLUMN_SPLIT)
      return fail(STENCIL_E_ARG, "%s: entry with unsupported tile or column store", path);
    const char* us = strstr(p, "\"us\":");
    if (us && us < e) v.us = strtod(us + 5, nullptr);
    t[k] = v;
    p = e + 1;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& kv : t) g_table[kv.first] = kv.second;
  return STENCIL_OK;
}

}  // extern "C"
