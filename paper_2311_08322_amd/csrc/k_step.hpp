// k_step.hpp -- fused gfx950 kernels of the forward stencils.
//
//   k_step_fused  : hdiff (lap -> limited fluxes -> update) at every level of
//                   a TI x TJ column tile, feeding a per-lane Thomas forward
//                   elimination; the back substitution writes the new state.
//   k_vadv_fused  : the Thomas solve alone, one column per lane.
//   k_hdiff_fused : the horizontal diffusion alone, tile marched along k.
//
// Stage semantics (GT4Py paper, Sec. 2.2): the horizontal stages are
// PARALLEL, the elimination FORWARD and the substitution BACKWARD; fusing
// them keeps the "as if in program order" meaning because each stage reads
// only values the previous stage has completed for this tile and level.
// The temporaries (lap, fluxes, c', d') never leave the chip: the u-tile of
// a level lives in LDS, lap and the fluxes in registers, c'/d' of a column
// in the lane's VGPRs (the k loop is unrolled per register class).
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace gt4mi {

__device__ __forceinline__ float absv(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double absv(double x) { return __builtin_fabs(x); }

template <int TI>
__device__ __forceinline__ void store_row_bits(uint8_t* p, uint64_t bits) {
  if constexpr (TI == 64) {
    *reinterpret_cast<uint64_t*>(p) = bits;
  } else if constexpr (TI == 32) {
    *reinterpret_cast<uint32_t*>(p) = static_cast<uint32_t>(bits);
  } else {
    static_assert(TI == 16, "tile width must be 16, 32 or 64");
    *reinterpret_cast<uint16_t*>(p) = static_cast<uint16_t>(bits);
  }
}

// Where one lane records the limiter decisions of its tile row (level 0;
// level k adds k planes).  A wave covers 64/TI rows of TI columns: the
// row's first lane stores the row's TI bits of the X and Y planes, the
// lanes on the domain's i = 0 / j = 0 edges store the edge bytes.
struct MaskWriter {
  uint8_t* xrow;  // X-plane bytes of this row at i0 (null: lane stores no row)
  uint8_t* ex;    // X-edge byte of (j) (null unless i == 0)
  uint8_t* ey;    // Y-edge byte of (i) (null unless j == 0)
  int64_t plane, ex_plane, ey_plane, y_minus_x;
  int shift;

  template <typename T, int TI>
  __device__ __forceinline__ static MaskWriter make(const StepArgs<T>& A, int i0, int i, int j, bool active) {
    MaskWriter m;
    const int lane = threadIdx.x & 63;
    m.shift = (lane / TI) * TI;
    m.plane = (int64_t)A.nj * A.ml.words * 8;
    m.ex_plane = A.nj;
    m.ey_plane = A.ni;
    m.y_minus_x = A.ml.y_off - A.ml.x_off;
    m.xrow = ((lane % TI) == 0 && j < A.nj) ? A.mask + A.ml.x_off + (int64_t)j * A.ml.words * 8 + (i0 >> 3) : nullptr;
    m.ex = (active && i == 0) ? A.mask + A.ml.ex_off + j : nullptr;
    m.ey = (active && j == 0) ? A.mask + A.ml.ey_off + i : nullptr;
    return m;
  }

  // every lane of the wave must call this (ballots)
  template <int TI>
  __device__ __forceinline__ void record(int k, bool active, bool kxr, bool kyr, bool kxl, bool kyl) const {
    const uint64_t bx = __ballot(active && kxr);
    const uint64_t by = __ballot(active && kyr);
    if (xrow) {
      uint8_t* p = xrow + (int64_t)k * plane;
      store_row_bits<TI>(p, bx >> shift);
      store_row_bits<TI>(p + y_minus_x, by >> shift);
    }
    if (ex) ex[(int64_t)k * ex_plane] = kxl ? 1 : 0;
    if (ey) ey[(int64_t)k * ey_plane] = kyl ? 1 : 0;
  }
};

// The 13-point diamond of u around a point (radius 2 in i and j): all the
// values one output of the horizontal diffusion depends on.
template <typename T>
struct Diamond {
  T u00, um1, up1, um2, up2, vm1, vp1, vm2, vp2, mm, mp, pm, pp;
};

// Read the diamond from the u-tile in LDS; `c` points at u(i,j), HI is the
// tile's row pitch.
template <typename T, int HI>
__device__ __forceinline__ Diamond<T> load_diamond(const T* __restrict__ c) {
  Diamond<T> d;
  d.u00 = c[0];
  d.um1 = c[-1];
  d.up1 = c[1];
  d.um2 = c[-2];
  d.up2 = c[2];
  d.vm1 = c[-HI];
  d.vp1 = c[HI];
  d.vm2 = c[-2 * HI];
  d.vp2 = c[2 * HI];
  d.mm = c[-HI - 1];
  d.mp = c[-HI + 1];
  d.pm = c[HI - 1];
  d.pp = c[HI + 1];
  return d;
}

// Horizontal diffusion of one point from its diamond.  The five Laplacians
// the point needs are formed from the diamond (no shared lap stage, so one
// barrier per level suffices).  Returns out; the four flux decisions go to
// kxr/kxl/kyr/kyl (right/left, x/y).
template <typename T>
__device__ __forceinline__ T hdiff_of(const Diamond<T>& d, T coeff, bool& kxr, bool& kxl, bool& kyr,
                                      bool& kyl) {
  // lap = 4u - ((u[i-1] + u[i+1]) + (u[j-1] + u[j+1])) at (0,0), (+-1,0), (0,+-1)
  const T L00 = T(4) * d.u00 - ((d.um1 + d.up1) + (d.vm1 + d.vp1));
  const T Lp0 = T(4) * d.up1 - ((d.u00 + d.up2) + (d.mp + d.pp));
  const T Lm0 = T(4) * d.um1 - ((d.um2 + d.u00) + (d.mm + d.pm));
  const T L0p = T(4) * d.vp1 - ((d.pm + d.pp) + (d.u00 + d.vp2));
  const T L0m = T(4) * d.vm1 - ((d.mm + d.mp) + (d.vm2 + d.u00));
  const T fxr = Lp0 - L00, fxl = L00 - Lm0, fyr = L0p - L00, fyl = L00 - L0m;
  kxr = flux_kept(fxr, d.up1 - d.u00);
  kxl = flux_kept(fxl, d.u00 - d.um1);
  kyr = flux_kept(fyr, d.vp1 - d.u00);
  kyl = flux_kept(fyl, d.u00 - d.vm1);
  const T Fxr = kxr ? fxr : T(0), Fxl = kxl ? fxl : T(0);
  const T Fyr = kyr ? fyr : T(0), Fyl = kyl ? fyl : T(0);
  return d.u00 - coeff * ((Fxr - Fxl) + (Fyr - Fyl));
}

// The generalised diffusion: a per-point coefficient kap, and the form's
// sign gs (form_sign) on the limiter's gradient and on the coefficient.
// gs = -1 gives the damping form exactly: its fluxes are the negatives of
// the stated ones, kept where f * (-g) <= 0, and u - kap * (-div) =
// u - (-kap) * div.
template <typename T>
__device__ __forceinline__ T hdiff_var_of(const Diamond<T>& d, T kap, T gs, bool& kxr, bool& kxl, bool& kyr,
                                          bool& kyl) {
  const T L00 = T(4) * d.u00 - ((d.um1 + d.up1) + (d.vm1 + d.vp1));
  const T Lp0 = T(4) * d.up1 - ((d.u00 + d.up2) + (d.mp + d.pp));
  const T Lm0 = T(4) * d.um1 - ((d.um2 + d.u00) + (d.mm + d.pm));
  const T L0p = T(4) * d.vp1 - ((d.pm + d.pp) + (d.u00 + d.vp2));
  const T L0m = T(4) * d.vm1 - ((d.mm + d.mp) + (d.vm2 + d.u00));
  const T fxr = Lp0 - L00, fxl = L00 - Lm0, fyr = L0p - L00, fyl = L00 - L0m;
  kxr = flux_kept(fxr, gs * (d.up1 - d.u00));
  kxl = flux_kept(fxl, gs * (d.u00 - d.um1));
  kyr = flux_kept(fyr, gs * (d.vp1 - d.u00));
  kyl = flux_kept(fyl, gs * (d.u00 - d.vm1));
  const T Fxr = kxr ? fxr : T(0), Fxl = kxl ? fxl : T(0);
  const T Fyr = kyr ? fyr : T(0), Fyl = kyl ? fyl : T(0);
  return d.u00 - (gs * kap) * ((Fxr - Fxl) + (Fyr - Fyl));
}

template <typename T, int HI>
__device__ __forceinline__ T hdiff_diamond(const T* __restrict__ c, T coeff, bool& kxr, bool& kxl,
                                           bool& kyr, bool& kyl) {
  return hdiff_of(load_diamond<T, HI>(c), coeff, kxr, kxl, kyr, kyl);
}

// Level-invariant addressing of a TI x TJ tile: byte offsets of the
// lane's share of the (TI+4) x (TJ+4) u-tile from the level base at padded
// point (-2,-2), and of its own column in the interior fields.  Lanes
// outside a ragged domain edge are clamped onto valid points: they load
// (and compute) garbage that is never stored, with no per-level branches.
template <typename T, int TI, int TJ>
struct TileAddr {
  static constexpr int NT = TI * TJ, HI = TI + 4, HN = (TI + 4) * (TJ + 4);
  static constexpr int NLD = (HN + NT - 1) / NT;
  uint32_t hoff[NLD];
  int ti, tj, i0, j0, i, j, ic, jc;
  bool active;

  __device__ __forceinline__ void init(int tile, int tiles_i, int ni, int nj, int64_t u_sj) {
    init_lane(threadIdx.x, tile, tiles_i, ni, nj, u_sj);
  }
  // `tid`: the lane's index among the NT lanes that share the tile
  __device__ __forceinline__ void init_lane(int tid, int tile, int tiles_i, int ni, int nj, int64_t u_sj) {
    ti = tid % TI;
    tj = tid / TI;
    const int bi = tile % tiles_i, bj = tile / tiles_i;
    i0 = bi * TI;
    j0 = bj * TJ;
    i = i0 + ti;
    j = j0 + tj;
    active = (i < ni) && (j < nj);
    ic = min(i, ni - 1);
    jc = min(j, nj - 1);
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int e = min(tid + q * NT, HN - 1);
      const int hj = e / HI, hi = e - hj * HI;
      const int gi = min(i0 + hi, ni + 3), gj = min(j0 + hj, nj + 3);  // padded coordinates
      hoff[q] = ((uint32_t)gi + (uint32_t)gj * (uint32_t)u_sj) * (uint32_t)sizeof(T);
    }
  }
};

// ------------------------------------------------------------------ step
// COL = 1: c' and d' of the column in registers.
// COL = 2: c' in registers, d' staged in `out` (read back by the same lane).
template <typename T, int TI, int TJ, int NKMAX, int PD, int COL>
__global__ void __launch_bounds__(TI* TJ) k_step_fused(StepArgs<T> A) {
  using TA = TileAddr<T, TI, TJ>;
  constexpr int NT = TA::NT, HI = TA::HI, NLD = TA::NLD;
  static_assert(NT == kWG, "tile must hold 256 columns");
  __shared__ T su[2][NLD * NT];  // padded: every lane's store lands inside

  TA t;
  t.init(xcd_tile(blockIdx.x, gridDim.x), A.tiles_i, A.ni, A.nj, A.u_sj);
  const int nk = A.nk, tid = threadIdx.x;
  constexpr uint32_t S = sizeof(T);
  const LevelView vu = level_view(A.u, A.u_sj, A.u_sk, -2, -2, A.nj + 4);
  const LevelView vd = level_view(A.data, A.d_sj, A.d_sk, 0, 0, A.nj);
  const LevelView vw = level_view(A.w, A.w_sj, A.w_sk, 0, 0, A.nj);
  const LevelView vo = level_view<T>(A.out, A.o_sj, A.o_sk, 0, 0, A.nj);
  const uint32_t doff = ((uint32_t)t.ic + (uint32_t)t.jc * (uint32_t)A.d_sj) * S;
  const uint32_t woff = ((uint32_t)t.ic + (uint32_t)t.jc * (uint32_t)A.w_sj) * S;
  const uint32_t ooff = ((uint32_t)t.ic + (uint32_t)t.jc * (uint32_t)A.o_sj) * S;
  const bool active = t.active;
  MaskWriter mw;
  if (A.mask) mw = MaskWriter::make<T, TI>(A, t.i0, t.i, t.j, active);

  // prefetch ring: slot k % PD holds level k (u-tile share, data_k, w_{k+1})
  T pu[PD][NLD], pd[PD], pw[PD];
  auto issue = [&](int s, int k) {
    const auto ru = vu.at(k);
#pragma unroll
    for (int q = 0; q < NLD; ++q) pu[s][q] = buf_ld(ru, t.hoff[q], T());
    pd[s] = buf_ld(vd.at(k), doff, T());
    pw[s] = buf_ld(vw.at(k + 1), woff, T());  // w has nk+1 levels
  };
#pragma unroll
  for (int s = 0; s < PD; ++s)
    if (s < nk) issue(s, s);

  T cp[NKMAX];
  T dp[COL == 1 ? NKMAX : 1];
  T wk = T(0), cprev = T(0), dprev = T(0);
  const T coeff = A.coeff, r4 = A.r4;
  const int cu = (t.tj + 2) * HI + (t.ti + 2);

#pragma unroll
  for (int k = 0; k < NKMAX; ++k) {
    if (k < nk) {
      const int s = k % PD;
      T* U = su[k & 1];
#pragma unroll
      for (int q = 0; q < NLD; ++q) U[tid + q * NT] = pu[s][q];
      const T dk = pd[s], wk1 = pw[s];
      if (k + PD < nk) issue(s, k + PD);
      pin_prefetch();
      __syncthreads();
      bool kxr, kxl, kyr, kyl;
      const T h = hdiff_diamond<T, HI>(U + cu, coeff, kxr, kxl, kyr, kyl);
      if (A.mask) mw.record<TI>(k, active, kxr, kyr, kxl, kyl);
      // Thomas forward elimination, coefficients rebuilt from w
      const T a = (k > 0) ? -r4 * wk : T(0);
      const T c = (k < nk - 1) ? r4 * wk1 : T(0);
      const T b = T(1) + absv(a) + absv(c);
      const T inv = recip(b - a * cprev);
      cprev = c * inv;
      dprev = ((h + dk) - a * dprev) * inv;
      cp[k] = cprev;
      if constexpr (COL == 1) {
        dp[k] = dprev;
      } else {
        if (active) buf_st(vo.at(k), ooff, dprev);
      }
      wk = wk1;
    }
  }
  // Thomas back substitution (c'_{nk-1} = 0 starts it from x = d')
  T x = T(0);
#pragma unroll
  for (int k = NKMAX - 1; k >= 0; --k) {
    if (k < nk) {
      const auto ro = vo.at(k);
      if constexpr (COL == 1) {
        x = dp[k] - cp[k] * x;
      } else {
        x = buf_ld(ro, ooff, T()) - cp[k] * x;
      }
      if (active) buf_st(ro, ooff, x);
    }
  }
}

// ------------------------------------------------------------------ vadv
// One column per lane: d = u + data, elimination and substitution.
// COL = 1: c', d' in registers; COL = 2: d' staged in `out`.
template <typename T, int NKMAX, int PD, int COL>
__global__ void __launch_bounds__(kWG) k_vadv_fused(StepArgs<T> A) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int bi = tile % A.tiles_i, bj = tile / A.tiles_i;
  const int i = bi * 64 + (threadIdx.x & 63), j = bj * 4 + (threadIdx.x >> 6);
  if (i >= A.ni || j >= A.nj) return;
  const int nk = A.nk;
  constexpr uint32_t S = sizeof(T);
  const LevelView vu = level_view(A.u, A.u_sj, A.u_sk, 0, 0, A.nj);
  const LevelView vd = level_view(A.data, A.d_sj, A.d_sk, 0, 0, A.nj);
  const LevelView vw = level_view(A.w, A.w_sj, A.w_sk, 0, 0, A.nj);
  const LevelView vo = level_view<T>(A.out, A.o_sj, A.o_sk, 0, 0, A.nj);
  const uint32_t uoff = ((uint32_t)i + (uint32_t)j * (uint32_t)A.u_sj) * S;
  const uint32_t doff = ((uint32_t)i + (uint32_t)j * (uint32_t)A.d_sj) * S;
  const uint32_t woff = ((uint32_t)i + (uint32_t)j * (uint32_t)A.w_sj) * S;
  const uint32_t ooff = ((uint32_t)i + (uint32_t)j * (uint32_t)A.o_sj) * S;
  T pu[PD], pd[PD], pw[PD];
  auto issue = [&](int s, int k) {
    pu[s] = buf_ld(vu.at(k), uoff, T());
    pd[s] = buf_ld(vd.at(k), doff, T());
    pw[s] = buf_ld(vw.at(k + 1), woff, T());  // w has nk+1 levels
  };
#pragma unroll
  for (int s = 0; s < PD; ++s)
    if (s < nk) issue(s, s);
  T cp[NKMAX];
  T dp[COL == 1 ? NKMAX : 1];
  T wk = T(0), cprev = T(0), dprev = T(0);
  const T r4 = A.r4;
#pragma unroll
  for (int k = 0; k < NKMAX; ++k) {
    if (k < nk) {
      const int s = k % PD;
      const T dk = pu[s] + pd[s], wk1 = pw[s];
      if (k + PD < nk) issue(s, k + PD);
      pin_prefetch();
      const T a = (k > 0) ? -r4 * wk : T(0);
      const T c = (k < nk - 1) ? r4 * wk1 : T(0);
      const T b = T(1) + absv(a) + absv(c);
      const T inv = recip(b - a * cprev);
      cprev = c * inv;
      dprev = (dk - a * dprev) * inv;
      cp[k] = cprev;
      if constexpr (COL == 1) dp[k] = dprev;
      else buf_st(vo.at(k), ooff, dprev);
      wk = wk1;
    }
  }
  T x = T(0);
#pragma unroll
  for (int k = NKMAX - 1; k >= 0; --k) {
    if (k < nk) {
      const auto ro = vo.at(k);
      if constexpr (COL == 1) x = dp[k] - cp[k] * x;
      else x = buf_ld(ro, ooff, T()) - cp[k] * x;
      buf_st(ro, ooff, x);
    }
  }
}

// ------------------------------------------------------------------ hdiff
// Tile marched over the levels [kbeg, kend) of its workgroup, the next
// level's u-tile prefetched in registers while the current one is computed.
// VAR: the generalised diffusion (per-point coefficient kappa when given,
// else the scalar, and the form's sign).
template <typename T, int TI, int TJ, bool VAR>
__global__ void __launch_bounds__(TI* TJ) k_hdiff_fused(StepArgs<T> A) {
  using TA = TileAddr<T, TI, TJ>;
  constexpr int NT = TA::NT, HI = TA::HI, NLD = TA::NLD;
  __shared__ T su[2][NLD * NT];
  TA t;
  t.init(xcd_tile(blockIdx.x, gridDim.x), A.tiles_i, A.ni, A.nj, A.u_sj);
  const int tid = threadIdx.x;
  const int kbeg = blockIdx.y * A.k1, kend = min(kbeg + A.k1, A.nk);  // k1: levels per workgroup
  const LevelView vu = level_view(A.u, A.u_sj, A.u_sk, -2, -2, A.nj + 4);
  const LevelView vo = level_view<T>(A.out, A.o_sj, A.o_sk, 0, 0, A.nj);
  const uint32_t ooff = ((uint32_t)t.ic + (uint32_t)t.jc * (uint32_t)A.o_sj) * (uint32_t)sizeof(T);
  const bool active = t.active;
  MaskWriter mw;
  if (A.mask) mw = MaskWriter::make<T, TI>(A, t.i0, t.i, t.j, active);
  const int cu = (t.tj + 2) * HI + (t.ti + 2);
  // the coefficient field (VAR): a null field reads through an empty window
  // and the scalar is used instead
  const bool has_kappa = VAR && A.kappa != nullptr;
  const LevelView vk = level_view(has_kappa ? A.kappa : A.u, A.c_sj, A.c_sk, 0, 0, has_kappa ? A.nj : 0);
  const uint32_t koff = ((uint32_t)t.ic + (uint32_t)t.jc * (uint32_t)A.c_sj) * (uint32_t)sizeof(T);
  const T gs = form_sign<T>(A.form);
  T pu[NLD], pk = T(0);
  {
    const auto ru = vu.at(kbeg);
#pragma unroll
    for (int q = 0; q < NLD; ++q) pu[q] = buf_ld(ru, t.hoff[q], T());
    if constexpr (VAR) pk = buf_ld(vk.at(kbeg), koff, T());
  }
  for (int k = kbeg; k < kend; ++k) {
    T* U = su[k & 1];
#pragma unroll
    for (int q = 0; q < NLD; ++q) U[tid + q * NT] = pu[q];
    const T kk = pk;
    if (k + 1 < kend) {
      const auto ru = vu.at(k + 1);
#pragma unroll
      for (int q = 0; q < NLD; ++q) pu[q] = buf_ld(ru, t.hoff[q], T());
      if constexpr (VAR) pk = buf_ld(vk.at(k + 1), koff, T());
    }
    __syncthreads();
    bool kxr, kxl, kyr, kyl;
    T h;
    if constexpr (VAR)
      h = hdiff_var_of(load_diamond<T, HI>(U + cu), has_kappa ? kk : A.coeff, gs, kxr, kxl, kyr, kyl);
    else
      h = hdiff_diamond<T, HI>(U + cu, A.coeff, kxr, kxl, kyr, kyl);
    if (A.mask) mw.record<TI>(k, active, kxr, kyr, kxl, kyl);
    if (active) buf_st(vo.at(k), ooff, h);
  }
}

// ------------------------------------------------------------------ class dispatch
#ifndef GT4MI_PD
#define GT4MI_PD 2  // levels of u/data/w loaded ahead of the one being computed
#endif

// One instantiation per register class of the column length.  The list of
// classes is shared by the forward and adjoint column kernels.
#define GT4MI_NK_CLASSES(X) X(16) X(32) X(48) X(64) X(80) X(96) X(128) X(160)

template <typename T, int COL>
constexpr bool column_class_ok(int nkmax) {
  // FP64 with both c' and d' in VGPRs spills beyond 96 levels
  return !(sizeof(T) == 8 && COL == 1 && nkmax > 96);
}

template <typename T, int TI, int TJ, int COL>
hipError_t launch_step_classes(const StepArgs<T>& A, hipStream_t s) {
  const dim3 grid(A.ntiles), block(TI * TJ);
#define GT4MI_STEP_CASE(N)                                                             \
  if constexpr (column_class_ok<T, COL>(N)) {                                          \
    if (A.nk <= N) {                                                                   \
      hipLaunchKernelGGL((k_step_fused<T, TI, TJ, N, GT4MI_PD, COL>), grid, block, 0, s, A); \
      return hipGetLastError();                                                        \
    }                                                                                  \
  }
  GT4MI_NK_CLASSES(GT4MI_STEP_CASE)
#undef GT4MI_STEP_CASE
  return hipErrorInvalidValue;
}

template <typename T, int COL>
hipError_t launch_vadv_classes(const StepArgs<T>& A, hipStream_t s) {
  const dim3 grid(A.ntiles), block(kWG);
#define GT4MI_VADV_CASE(N)                                                          \
  if constexpr (column_class_ok<T, COL>(N)) {                                       \
    if (A.nk <= N) {                                                                \
      hipLaunchKernelGGL((k_vadv_fused<T, N, 2, COL>), grid, block, 0, s, A);      \
      return hipGetLastError();                                                     \
    }                                                                               \
  }
  GT4MI_NK_CLASSES(GT4MI_VADV_CASE)
#undef GT4MI_VADV_CASE
  return hipErrorInvalidValue;
}

}  // namespace gt4mi
