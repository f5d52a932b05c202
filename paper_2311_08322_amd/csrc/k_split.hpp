// k_split.hpp -- fused time step with each column eliminated from both ends.
//
// The tridiagonal system of a column is solved by a two-sided ("twisted")
// factorization: lanes of the upper half of the workgroup eliminate levels
// 0, 1, ..., m-1 downwards exactly as the Thomas FORWARD sweep does, lanes
// of the lower half eliminate levels nk-1, nk-2, ..., m upwards (the same
// sweep on the reversed system).  The two meet in a 2 x 2 system for
// (x_{m-1}, x_m); each half then substitutes back towards its own end.
// Every half holds the factors of only half the column, so a 256-column
// tile runs as 8 waves (two per SIMD) where the one-sided sweep fits one.
//
// Top half, level k (near = a_k, far = c_k):
//   p = b_k - a_k e_{k-1};  e_k = c_k / p;  f_k = (d_k - a_k f_{k-1}) / p
//   x_k = f_k - e_k x_{k+1}
// Bottom half, level k (near = c_k, far = a_k):
//   p = b_k - c_k e_{k+1};  e_k = a_k / p;  f_k = (d_k - c_k f_{k+1}) / p
//   x_k = f_k - e_k x_{k-1}
// Interface: x_m = (f_m - e_m f_{m-1}) / (1 - e_m e_{m-1}),
//            x_{m-1} = f_{m-1} - e_{m-1} x_m.
// Diagonal dominance (|a|, |c| <= 1/8 for |w| <= 1, dt/dz = 1/2 keeps
// |e| <= 1/8) makes every pivot, the interface one included, >= 1 - 1/64.
#pragma once

#include "k_step.hpp"

namespace gt4mi {

// Branch-free recorder of one lane's limiter decisions (buffer stores; a
// lane that stores nothing at a level uses an offset outside the window).
struct MaskRec {
  const char* base;
  int64_t plane_xy, plane_ex, plane_ey, x_off, y_off, ex_off, ey_off;
  uint32_t win_xy, win_ex, win_ey;
  uint32_t off_row, off_ex, off_ey;
  int shift;

  template <typename T, int TI>
  __device__ __forceinline__ void init(const StepArgs<T>& A, int lane_in_tile, int i0, int i, int j,
                                       bool active) {
    const int lane = lane_in_tile & 63;
    base = reinterpret_cast<const char*>(A.mask);
    plane_xy = (int64_t)A.nj * A.ml.words * 8;
    plane_ex = A.nj;
    plane_ey = A.ni;
    x_off = A.ml.x_off;
    y_off = A.ml.y_off;
    ex_off = A.ml.ex_off;
    ey_off = A.ml.ey_off;
    // a field without a mask (batched launches mix them) gets empty windows:
    // every store falls outside and is dropped
    const bool has = A.mask != nullptr;
    win_xy = has ? (uint32_t)plane_xy : 0u;
    win_ex = has ? (uint32_t)A.nj : 0u;
    win_ey = has ? (uint32_t)A.ni : 0u;
    shift = (lane / TI) * TI;
    off_row = ((lane % TI) == 0 && j < A.nj) ? (uint32_t)(j * A.ml.words * 8 + (i0 >> 3)) : kOffNone;
    off_ex = (active && i == 0) ? (uint32_t)j : kOffNone;
    off_ey = (active && j == 0) ? (uint32_t)i : kOffNone;
  }

  template <int TI>
  __device__ __forceinline__ static void bits(__amdgpu_buffer_rsrc_t r, uint32_t off, uint64_t b) {
    if constexpr (TI == 64) buf_st_u64(r, off, b);
    else if constexpr (TI == 32) buf_st_u32(r, off, (uint32_t)b);
    else buf_st_u16(r, off, (uint16_t)b);
  }

  // every lane of the wave calls this (ballots); `act` is wave-uniform
  template <int TI>
  __device__ __forceinline__ void record(int k, bool act, bool active, bool kxr, bool kyr, bool kxl,
                                         bool kyl) const {
    const uint64_t bx = __ballot(active && kxr);
    const uint64_t by = __ballot(active && kyr);
    const uint32_t orow = act ? off_row : kOffNone;
    bits<TI>(make_rsrc(base + x_off + (int64_t)k * plane_xy, win_xy), orow, bx >> shift);
    bits<TI>(make_rsrc(base + y_off + (int64_t)k * plane_xy, win_xy), orow, by >> shift);
    buf_st_u8(make_rsrc(base + ex_off + (int64_t)k * plane_ex, win_ex), act ? off_ex : kOffNone, kxl ? 1 : 0);
    buf_st_u8(make_rsrc(base + ey_off + (int64_t)k * plane_ey, win_ey), act ? off_ey : kOffNone, kyl ? 1 : 0);
  }
};

// The loop runs the steps of the column with no per-step branch besides the
// barrier and the exit after the last step: a step past the half's last
// level (odd nk) reloads a clamped level and leaves the factors unchanged
// (selects), so the prefetch stays a fixed distance ahead and the load
// counters are exact.
//
// COL = 1: both halves keep e and f of every level in VGPRs.
// COL = 2: e in VGPRs, f staged in `out` (longer columns in the same VGPRs).
// Cache policy of the streamed accesses: data, w and out are touched once
// (GT4MI_CP_ONCE), u's halo rows are shared with the neighbouring tiles
// through L2 (GT4MI_CP_HALO).
#ifndef GT4MI_CP_ONCE
#define GT4MI_CP_ONCE 0
#endif
#ifndef GT4MI_CP_HALO
#define GT4MI_CP_HALO 0
#endif

template <typename T, int TI, int TJ>
struct SplitSmem {
  static constexpr int NT = TI * TJ;          // columns of the tile (lanes per half)
  T su[2][2][TileAddr<T, TI, TJ>::NLD * NT];  // [half][step parity]
  T xch[2][2][NT];                            // innermost (e, f) of each half and column
};

// VAR: the generalised diffusion (per-point coefficient when A.kappa is
// set, the scalar otherwise; the form's sign on the limiter and coefficient).
template <typename T, int TI, int TJ, int NKH, int PD, bool MASK, int COL, bool VAR = false>
__device__ __forceinline__ void step_split_tile(const StepArgs<T>& A, int tile, SplitSmem<T, TI, TJ>& sm) {
  using TA = TileAddr<T, TI, TJ>;
  constexpr int NT = TA::NT, HI = TA::HI, NLD = TA::NLD;
  static_assert(NT == 256 || NT == 128, "a tile holds 256 or 128 columns");

  const int half = __builtin_amdgcn_readfirstlane((int)threadIdx.x / NT);  // 0: top, 1: bottom
  const int ltid = threadIdx.x - half * NT;
  TA t;
  t.init_lane(ltid, tile, A.tiles_i, A.ni, A.nj, A.u_sj);
  const int nk = A.nk, m = nk / 2;
  const int nlev = half ? nk - m : m;  // levels this half eliminates
  const int nsteps = nk - m;           // steps of the workgroup (the larger half)
  const int k0 = half ? nk - 1 : 0, dir = half ? -1 : 1;
  constexpr uint32_t S = sizeof(T);
  const LevelView vu = level_view(A.u, A.u_sj, A.u_sk, -2, -2, A.nj + 4);
  const LevelView vd = level_view(A.data, A.d_sj, A.d_sk, 0, 0, A.nj);
  const LevelView vw = level_view(A.w, A.w_sj, A.w_sk, 0, 0, A.nj);
  const LevelView vo = level_view<T>(A.out, A.o_sj, A.o_sk, 0, 0, A.nj);
  const uint32_t doff = ((uint32_t)t.ic + (uint32_t)t.jc * (uint32_t)A.d_sj) * S;
  const uint32_t woff = ((uint32_t)t.ic + (uint32_t)t.jc * (uint32_t)A.w_sj) * S;
  const uint32_t ooff = t.active ? ((uint32_t)t.ic + (uint32_t)t.jc * (uint32_t)A.o_sj) * S : kOffNone;
  const bool active = t.active;
  MaskRec mr;
  if constexpr (MASK) mr.init<T, TI>(A, ltid, t.i0, t.i, t.j, active);

  // Load cursors walk this half's levels in step order and hold at its last
  // level, so steps past it (odd nk, class padding) reload a valid level.
  LevelCursor cur_u{vu.base + (int64_t)k0 * vu.level_bytes, dir * vu.level_bytes, vu.window};
  LevelCursor cur_d{vd.base + (int64_t)k0 * vd.level_bytes, dir * vd.level_bytes, vd.window};
  LevelCursor cur_w{vw.base + (int64_t)(half ? k0 : 1) * vw.level_bytes, dir * vw.level_bytes, vw.window};
  // the coefficient field (VAR): a null field reads through an empty window
  const bool has_kappa = VAR && A.kappa != nullptr;
  const LevelView vk = level_view(has_kappa ? A.kappa : A.data, A.c_sj, A.c_sk, 0, 0, has_kappa ? A.nj : 0);
  const uint32_t koff = ((uint32_t)t.ic + (uint32_t)t.jc * (uint32_t)A.c_sj) * S;
  LevelCursor cur_k{vk.base + (int64_t)k0 * vk.level_bytes, dir * vk.level_bytes, vk.window};
  T pu[PD][NLD], pd[PD], pw[PD], pk[VAR ? PD : 1];
  auto issue = [&](int slot, int s) {
    const auto ru = cur_u.rsrc();
#pragma unroll
    for (int q = 0; q < NLD; ++q) pu[slot][q] = buf_ld<GT4MI_CP_HALO>(ru, t.hoff[q], T());
    pd[slot] = buf_ld<GT4MI_CP_ONCE>(cur_d.rsrc(), doff, T());
    pw[slot] = buf_ld<GT4MI_CP_ONCE>(cur_w.rsrc(), woff, T());  // the w level new at this step
    if constexpr (VAR) pk[slot] = buf_ld<GT4MI_CP_ONCE>(cur_k.rsrc(), koff, T());
    const bool go = s + 1 < nlev;
    cur_u.advance(go);
    cur_d.advance(go);
    cur_w.advance(go);
    if constexpr (VAR) cur_k.advance(go);
  };
#pragma unroll
  for (int s = 0; s < PD; ++s) issue(s, s);

  T ev[NKH];
  T fv[COL == 1 ? NKH : 1];
  T wp = T(0), e = T(0), f = T(0);
  const T coeff = A.coeff;
  [[maybe_unused]] const T gs = form_sign<T>(A.form);
  const T sn = half ? A.r4 : -A.r4;  // near coefficient per unit w: top a = -r/4 w, bottom c = +r/4 w
  const int cu = (t.tj + 2) * HI + (t.ti + 2);
  T hq = T(0), dq = T(0), wq = T(0);  // the previous step's diffused value, data and new w

  // Software pipeline: after the barrier of step s the diamond reads of s
  // are issued first and the column elimination of step s-1 runs while
  // they are in flight; then the diffusion of step s completes.  The only
  // branch in the unrolled steps is the exit after the column's last step
  // (so every step's load counters stay exact); the elimination of that
  // last step follows the loop.
  auto eliminate = [&](int sp) {
    const bool act = sp < nlev;
    const int k = k0 + dir * sp;
    const T nr = (sp > 0) ? sn * wp : T(0);                 // a_k (top, k >= 1) / c_k (bottom, k <= nk-2)
    const T fr = (half == 0 || k > 0) ? -sn * wq : T(0);   // c_k (top) / a_k (bottom, k >= 1)
    const T b = T(1) + absv(nr) + absv(fr);
    const T inv = recip(b - nr * e);
    const T en = fr * inv;
    const T fn = ((hq + dq) - nr * f) * inv;
    e = act ? en : e;
    f = act ? fn : f;
    wp = act ? wq : wp;
    return act;
  };
#pragma unroll
  for (int s = 0; s < NKH; ++s) {
    if (s >= nsteps) break;  // uniform
    __builtin_amdgcn_sched_barrier(0);
    const int slot = s % PD;
    T* U = sm.su[half][s & 1];
#pragma unroll
    for (int q = 0; q < NLD; ++q) U[ltid + q * NT] = pu[slot][q];
    const T dk = pd[slot], wn = pw[slot];
    [[maybe_unused]] T kk = coeff;
    if constexpr (VAR) kk = has_kappa ? pk[slot] : coeff;
    if (s + PD < NKH) issue(slot, s + PD);
    __syncthreads();
    const Diamond<T> dm = load_diamond<T, HI>(U + cu);
    if (s > 0) {
      const bool act = eliminate(s - 1);
      ev[s - 1] = e;
      if constexpr (COL == 1) fv[s - 1] = f;
      else buf_st(vo.at(min(max(k0 + dir * (s - 1), 0), nk - 1)), act ? ooff : kOffNone, f);
    }
    bool kxr, kxl, kyr, kyl;
    if constexpr (VAR)
      hq = hdiff_var_of(dm, kk, gs, kxr, kxl, kyr, kyl);
    else
      hq = hdiff_of(dm, coeff, kxr, kxl, kyr, kyl);
    dq = dk;
    wq = wn;
    if constexpr (MASK) mr.record<TI>(min(max(k0 + dir * s, 0), nk - 1), s < nlev, active, kxr, kyr, kxl, kyl);
  }
  {  // the elimination of the last step
    const int sl = nsteps - 1;
    const bool act = eliminate(sl);
#pragma unroll
    for (int s = 0; s < NKH; ++s)
      if (s == sl) {
        ev[s] = e;
        if constexpr (COL == 1) fv[s] = f;
      }
    if constexpr (COL == 2) buf_st(vo.at(min(max(k0 + dir * sl, 0), nk - 1)), act ? ooff : kOffNone, f);
  }
  // interface: the two innermost levels m-1 (top) and m (bottom)
  sm.xch[half][0][ltid] = e;
  sm.xch[half][1][ltid] = f;
  __syncthreads();
  const T eo = sm.xch[1 - half][0][ltid], fo = sm.xch[1 - half][1][ltid];
  const T et = half ? eo : e, ft = half ? fo : f;  // top's e_{m-1}, f_{m-1} (0 if nk = 1)
  const T eb = half ? e : eo, fb = half ? f : fo;  // bottom's e_m, f_m
  const T xm = (fb - eb * ft) * recip(T(1) - eb * et);
  const T xm1 = ft - et * xm;
  T x = half ? xm1 : xm;  // the value beyond this half's innermost level
#pragma unroll
  for (int s = NKH - 1; s >= 0; --s) {
    if (s < nlev) {  // uniform
      const auto ro = vo.at(k0 + dir * s);
      if constexpr (COL == 1) x = fv[s] - ev[s] * x;
      else x = buf_ld(ro, ooff, T()) - ev[s] * x;
      buf_st<GT4MI_CP_ONCE>(ro, ooff, x);
    }
  }
}


template <typename T, int TI, int TJ, int NKH, int PD, bool MASK, int COL, bool VAR>
__global__ void __launch_bounds__(2 * TI * TJ) k_step_split(StepArgs<T> A) {
  __shared__ SplitSmem<T, TI, TJ> sm;
  step_split_tile<T, TI, TJ, NKH, PD, MASK, COL, VAR>(A, ordered_tile(A.order, blockIdx.x, gridDim.x), sm);
}

// One instantiation per half-column register class.  With the early exit a
// class costs only its registers, so the classes are coarse.  FP64 keeps e
// and f of both halves in VGPRs up to 96 levels (class 48: 244-250 VGPRs, two
// waves per SIMD).  Longer FP64 columns (up to 144) run in 128-column tiles
// with e and f in VGPRs at one wave per SIMD (launch_split_long); where that
// form is not instantiated (the generalised diffusion) they keep e and
// stage f in the output, as the batched kernel does beyond 80 levels.
#define GT4MI_NKH_CLASSES(X) X(16) X(24) X(40) X(48) X(56) X(80)
constexpr int kSplitStagedNkhF64 = 72;
// Levels loaded ahead in the long FP64 form.  It runs one wave per SIMD, so
// each wave has to keep more loads in flight than in the two-wave classes.
#ifndef GT4MI_PD_LONG
#define GT4MI_PD_LONG 4
#endif

template <typename T>
constexpr int split_max_nk() {
  return sizeof(T) == 8 ? 2 * kSplitStagedNkhF64 : 160;
}

template <typename T, int TI, int TJ, bool VAR>
hipError_t launch_split_classes(const StepArgs<T>& A, hipStream_t s) {
  const dim3 grid(A.ntiles), block(2 * TI * TJ);
  const int nkh = A.nk - A.nk / 2;
#define GT4MI_SPLIT_LAUNCH(N, C)                                                                     \
  {                                                                                                  \
    if (A.mask)                                                                                      \
      hipLaunchKernelGGL((k_step_split<T, TI, TJ, N, GT4MI_PD, true, C, VAR>), grid, block, 0, s, A); \
    else                                                                                             \
      hipLaunchKernelGGL((k_step_split<T, TI, TJ, N, GT4MI_PD, false, C, VAR>), grid, block, 0, s, A); \
    return hipGetLastError();                                                                        \
  }
#define GT4MI_SPLIT_CASE(N)                                                                  \
  if constexpr (2 * N <= (sizeof(T) == 8 ? kSplitRegNkF64 : 160) && (sizeof(T) == 8 || N != 48)) { \
    if (nkh <= N) GT4MI_SPLIT_LAUNCH(N, 1)                                                   \
  }
  GT4MI_NKH_CLASSES(GT4MI_SPLIT_CASE)
  if constexpr (sizeof(T) == 8) {
    if (nkh <= kSplitStagedNkhF64) GT4MI_SPLIT_LAUNCH(kSplitStagedNkhF64, 2)
  }
#undef GT4MI_SPLIT_CASE
#undef GT4MI_SPLIT_LAUNCH
  return hipErrorInvalidValue;
}

// FP64 columns of 97..144 levels: TI x (kSplitLongNT / TI) tiles of 256 lanes,
// e and f of both halves in VGPRs (about 360; no spills).  A.tiles_i and
// A.ntiles count tiles of that shape.
template <typename T, int TI>
hipError_t launch_split_long(const StepArgs<T>& A, hipStream_t s) {
  static_assert(sizeof(T) == 8, "binary32 columns fit the 256-column classes");
  constexpr int TJ = kSplitLongNT / TI;
  const dim3 grid(A.ntiles), block(2 * TI * TJ);
  if (A.nk - A.nk / 2 > kSplitStagedNkhF64) return hipErrorInvalidValue;
  if (A.mask)
    hipLaunchKernelGGL((k_step_split<T, TI, TJ, kSplitStagedNkhF64, GT4MI_PD_LONG, true, 1, false>), grid, block, 0, s, A);
  else
    hipLaunchKernelGGL((k_step_split<T, TI, TJ, kSplitStagedNkhF64, GT4MI_PD_LONG, false, 1, false>), grid, block, 0, s, A);
  return hipGetLastError();
}

}  // namespace gt4mi
