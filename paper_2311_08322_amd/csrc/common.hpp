// common.hpp -- device-side views, kernel argument blocks and small helpers
// shared by the gfx950 kernels of the stencil library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gt4mi {

constexpr int kHalo = 2;
constexpr int kNumXcd = 8;        // MI355X: 8 XCDs, workgroups dispatched round-robin
constexpr int kWG = 256;          // threads per workgroup of every tile kernel
// the two-ended fused step in FP64: columns up to kSplitRegNkF64 levels in
// 256-column tiles with e and f in VGPRs; longer ones (up to 144) in
// kSplitLongNT-column tiles
constexpr int kSplitRegNkF64 = 96;
constexpr int kSplitLongNT = 128;
// the hdiff adjoint's strips: 64 lanes in i (60 outputs; FP32 124, two
// columns per lane), strip_rows<T>() output rows in j, of whose
// strip_rows<T>() + 4 input rows strip_pd<T>() are in flight ahead of their
// use.  Measured on cold buffers (512x512x80 and 256x256x80): FP64 walks
// 8 rows with the whole strip loaded at once, FP32 12 rows likewise.
constexpr int kStripOut = 60;
constexpr int kStripOut2 = 124;
#ifndef GT4MI_STRIP_ROWS_F64
#define GT4MI_STRIP_ROWS_F64 8
#endif
#ifndef GT4MI_STRIP_PD_F64
#define GT4MI_STRIP_PD_F64 12
#endif
#ifndef GT4MI_STRIP_ROWS_F32
#define GT4MI_STRIP_ROWS_F32 12
#endif
#ifndef GT4MI_STRIP_PD_F32
#define GT4MI_STRIP_PD_F32 16
#endif
template <typename T>
constexpr int strip_rows() {
  return sizeof(T) == 8 ? GT4MI_STRIP_ROWS_F64 : GT4MI_STRIP_ROWS_F32;
}
template <typename T>
constexpr int strip_pd() {
  return sizeof(T) == 8 ? GT4MI_STRIP_PD_F64 : GT4MI_STRIP_PD_F32;
}
constexpr int kStripsPerWG = kWG / 64;  // one strip per wave

// ------------------------------------------------------------------ mask
// Packed limiter decisions of one domain (1 = flux kept), see stencil.h.
struct MaskLayout {
  int64_t words;  // 64-bit words per row: ceil(ni / 64)
  int64_t x_off, y_off, ex_off, ey_off, total;

  __host__ __device__ static int64_t round256(int64_t b) { return (b + 255) & ~int64_t(255); }

  __host__ __device__ static MaskLayout make(int64_t ni, int64_t nj, int64_t nk) {
    MaskLayout m;
    if (ni <= 0 || nj <= 0 || nk <= 0) {  // an empty domain has no fluxes
      m.words = m.x_off = m.y_off = m.ex_off = m.ey_off = m.total = 0;
      return m;
    }
    m.words = (ni + 63) / 64;
    const int64_t plane = round256(8 * m.words * nj * nk);
    m.x_off = 0;
    m.y_off = plane;
    m.ex_off = 2 * plane;
    m.ey_off = m.ex_off + round256(nj * nk);
    m.total = m.ey_off + round256(ni * nk);
    return m;
  }
};

// ------------------------------------------------------------ XCD mapping
// The dispatcher hands workgroup b to XCD (b % 8).  Give each XCD one
// contiguous run of tiles so that tiles sharing halo rows share an L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  const int q = nblocks / kNumXcd, r = nblocks % kNumXcd;
  const int x = b % kNumXcd, local = b / kNumXcd;
  return x * q + (x < r ? x : r) + local;
}
// The tile of workgroup b in the given order (stencil_tile_order: 2 takes
// the dispatch order itself, anything else the XCD runs).
__device__ __forceinline__ int ordered_tile(int order, int b, int nblocks) {
  return order == 2 ? b : xcd_tile(b, nblocks);
}

// ------------------------------------------------------------ addressing
// Fields are read and written through buffer resources: a per-level
// descriptor (uniform, SGPRs: base of the level and the byte size of the
// window the kernel may touch) plus a per-lane 32-bit byte offset.  A level
// change is a scalar add; accesses beyond the window read 0 / are dropped
// by the hardware range check instead of reaching other memory.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
constexpr int kRsrcWord3 = 0x00020000;  // gfx9 raw buffer: 32-bit data, no swizzle

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRsrcWord3);
}
// CP: the cache-policy bits of the access (0 = default; kCpStream marks data
// touched once, which the caches may evict first).
constexpr int kCpStream = 2;  // gfx950 "nt"
template <int CP = 0>
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, CP));
}
template <int CP = 0>
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t off, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, CP));
}
template <int CP = 0>
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, off, 0, CP);
}
template <int CP = 0>
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, CP);
}

// A per-lane byte offset that lies outside every window: a buffer store to
// it is discarded and a load returns 0, which predicates a lane's access
// without a branch.
constexpr uint32_t kOffNone = 0xFFFFFFF0u;

// DPP wave shifts of GFX9: lane l reads lane l+1 (shl) or lane l-1 (shr);
// the lane past the wave's end reads 0.  Every lane must be active.
constexpr int kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138;

template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint32_t buf_ld_u32(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}
__device__ __forceinline__ uint32_t buf_ld_u8(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0);
}

__device__ __forceinline__ void buf_st_u8(__amdgpu_buffer_rsrc_t r, uint32_t off, uint8_t v) {
  __builtin_amdgcn_raw_buffer_store_b8(v, r, off, 0, 0);
}
__device__ __forceinline__ void buf_st_u16(__amdgpu_buffer_rsrc_t r, uint32_t off, uint16_t v) {
  __builtin_amdgcn_raw_buffer_store_b16(v, r, off, 0, 0);
}
__device__ __forceinline__ void buf_st_u32(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t v) {
  __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, 0);
}
__device__ __forceinline__ void buf_st_u64(__amdgpu_buffer_rsrc_t r, uint32_t off, uint64_t v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, off, 0, 0);
}

// One field as seen by a kernel: the level-0 base, the level stride (bytes)
// and the window (bytes) of one level.
struct LevelView {
  const char* base;
  int64_t level_bytes;
  uint32_t window;
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t at(int k) const {
    return make_rsrc(base + (int64_t)k * level_bytes, window);
  }
};

// Buffer view of a field whose pointer `p` is at domain point (0,0,0),
// with the window starting at (di, dj) relative to it and `rows` rows long.
template <typename T>
__device__ __forceinline__ LevelView level_view(const T* p, int64_t sj, int64_t sk, int di, int dj, int rows) {
  LevelView v;
  v.base = reinterpret_cast<const char*>(p + di + (int64_t)dj * sj);
  v.level_bytes = sk * (int64_t)sizeof(T);
  v.window = (uint32_t)(sj * rows * (int64_t)sizeof(T));
  return v;
}

// A level pointer that walks a field one level per step (either direction)
// and can be held at a level: the uniform state of a marching kernel.
struct LevelCursor {
  const char* p;
  int64_t step;
  uint32_t window;
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc() const { return make_rsrc(p, window); }
  __device__ __forceinline__ void advance(bool go) { p += go ? step : 0; }
};

// ------------------------------------------------------------ prefetch
// Pins the loads issued before it to this point of the program.  The column
// kernels unroll their level loop with a uniform exit after every step, and
// the compiler otherwise sinks each prefetched load into the step that
// consumes it (the exits make the load look wasted on the paths that leave
// early), so the prefetch degenerates into a load followed by a full wait.
// An empty asm that clobbers memory keeps the loads where they are written
// without forcing a wait for them.
__device__ __forceinline__ void pin_prefetch() { __asm__ volatile("" ::: "memory"); }

// ------------------------------------------------------------ limiter
// The flux is zeroed where flux * gradient > 0 (the workload's definition
// of the diffusion named in Sec. 3.1), the product taken literally in the working precision.
template <typename T>
__device__ __forceinline__ bool flux_kept(T f, T g) {
  return !(f * g > T(0));
}

// Reciprocal of a Thomas pivot.  The pivots are bounded (m >= 1, strict
// diagonal dominance), so the hardware reciprocal refined by Newton steps
// (two for binary64, one for binary32) is accurate to about an ulp.
__device__ __forceinline__ double recip(double m) {
  double r = __builtin_amdgcn_rcp(m);
  r = __builtin_fma(__builtin_fma(-m, r, 1.0), r, r);
  r = __builtin_fma(__builtin_fma(-m, r, 1.0), r, r);
  return r;
}
__device__ __forceinline__ float recip(float m) {
  float r = __builtin_amdgcn_rcpf(m);
  return __builtin_fmaf(__builtin_fmaf(-m, r, 1.0f), r, r);
}

// ------------------------------------------------------------ argument blocks
template <typename T>
struct StepArgs {
  const T* u;  // at domain point (0,0,0); read with a 2-point halo
  int64_t u_sj, u_sk;
  const T* data;
  int64_t d_sj, d_sk;
  const T* w;  // staggered level 0
  int64_t w_sj, w_sk;
  T* out;
  int64_t o_sj, o_sk;
  uint8_t* mask;  // nullable
  MaskLayout ml;
  int ni, nj, nk;
  int tiles_i, ntiles;
  int k0, k1;  // level range of this launch (hdiff kernels)
  T coeff, r4;  // r4 = dt_dz / 4
  // generalised diffusion (read only by the kernels built for it)
  const T* kappa;  // per-point coefficient at domain (0,0,0), or null (scalar coeff)
  int64_t c_sj, c_sk;
  int form;  // 0: lap = 4u - sum of the neighbours; 1: the damping form, lap = sum - 4u
  int order;  // tile order of the two-ended step: 2 = dispatch order, else XCD runs
  int tile_i;  // batched launches: the tile width of this item's field (64, 32 or 16)
};

// Sign that folds the damping form into the stated one: its Laplacian,
// fluxes and divergence are the exact negatives of the stated ones, so it
// equals the stated diffusion with the limiter's gradient and the
// coefficient multiplied by -1 (products with -1 are exact).
template <typename T>
__host__ __device__ inline T form_sign(int form) {
  return form ? T(-1) : T(1);
}

template <typename T>
struct AdjArgs {
  const T* xbar;  // domain
  int64_t x_sj, x_sk;
  const T* w;
  int64_t w_sj, w_sk;
  T* lam;  // domain (column adjoint output, data_bar)
  int64_t l_sj, l_sk;
  T* ubar;  // at domain (0,0,0); written over the 2-point halo too
  int64_t b_sj, b_sk;
  const uint8_t* mask;
  MaskLayout ml;
  int ni, nj, nk;
  int tiles_i, ntiles;
  T coeff, r4;
  // per-point coefficient of the generalised diffusion (null: the scalar
  // coeff); with it, coeff holds the form's sign
  const T* kappa;
  int64_t c_sj, c_sk;
};

// ni is even and lambda's rows keep 8-byte alignment (base, row and level
// strides): the binary32 gather then reads a lane's two columns, an even and
// an odd one, with one load
template <typename T>
__host__ __device__ inline bool lambda_pairs_ok(const AdjArgs<T>& A) {
  return A.ni % 2 == 0 && reinterpret_cast<uintptr_t>(A.lam) % 8 == 0 &&
         (A.l_sj * (int64_t)sizeof(T)) % 8 == 0 && (A.l_sk * (int64_t)sizeof(T)) % 8 == 0;
}

}  // namespace gt4mi
