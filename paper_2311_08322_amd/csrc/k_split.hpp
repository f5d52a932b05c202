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
    win_xy = (uint32_t)plane_xy;
    win_ex = (uint32_t)A.nj;
    win_ey = (uint32_t)A.ni;
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

// The loop runs every step of the register class with no per-step branch
// besides the barrier: a step past the half's last level reloads a clamped
// level and leaves the factors unchanged (selects), so the prefetch stays
// a fixed distance ahead and the load counters are exact.
template <typename T, int TI, int TJ, int NKH, int PD, bool MASK>
__global__ void __launch_bounds__(2 * TI * TJ) k_step_split(StepArgs<T> A) {
  using TA = TileAddr<T, TI, TJ>;
  constexpr int NT = TA::NT, HI = TA::HI, NLD = TA::NLD;
  static_assert(NT == kWG, "tile must hold 256 columns");
  __shared__ T su[2][2][NLD * NT];  // [half][step parity]
  __shared__ T xch[2][2][NT];       // innermost (e, f) of each half and column

  const int half = __builtin_amdgcn_readfirstlane((int)threadIdx.x / NT);  // 0: top, 1: bottom
  const int ltid = threadIdx.x - half * NT;
  TA t;
  t.init_lane(ltid, xcd_tile(blockIdx.x, gridDim.x), A.tiles_i, A.ni, A.nj, A.u_sj);
  const int nk = A.nk, m = nk / 2;
  const int nlev = half ? nk - m : m;  // levels this half eliminates
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
  T pu[PD][NLD], pd[PD], pw[PD];
  auto issue = [&](int slot, int s) {
    const auto ru = cur_u.rsrc();
#pragma unroll
    for (int q = 0; q < NLD; ++q) pu[slot][q] = buf_ld(ru, t.hoff[q], T());
    pd[slot] = buf_ld(cur_d.rsrc(), doff, T());
    pw[slot] = buf_ld(cur_w.rsrc(), woff, T());  // the w level new at this step
    const bool go = s + 1 < nlev;
    cur_u.advance(go);
    cur_d.advance(go);
    cur_w.advance(go);
  };
#pragma unroll
  for (int s = 0; s < PD; ++s) issue(s, s);

  T ev[NKH], fv[NKH];
  T wp = T(0), e = T(0), f = T(0);
  const T coeff = A.coeff;
  const T sn = half ? A.r4 : -A.r4;  // near coefficient per unit w: top a = -r/4 w, bottom c = +r/4 w
  const int cu = (t.tj + 2) * HI + (t.ti + 2);
  T hq = T(0), dq = T(0), wq = T(0);  // the previous step's diffused value, data and new w

  // Software pipeline: after the barrier of step s the diamond reads of s
  // are issued first and the column elimination of step s-1 runs while
  // they are in flight; then the diffusion of step s completes.
#pragma unroll
  for (int s = 0; s <= NKH; ++s) {
    __builtin_amdgcn_sched_barrier(0);
    Diamond<T> dm;
    T dk = T(0), wn = T(0);
    if (s < NKH) {
      const int slot = s % PD;
      T* U = su[half][s & 1];
#pragma unroll
      for (int q = 0; q < NLD; ++q) U[ltid + q * NT] = pu[slot][q];
      dk = pd[slot];
      wn = pw[slot];
      if (s + PD < NKH) issue(slot, s + PD);
      __syncthreads();
      dm = load_diamond<T, HI>(U + cu);
    }
    if (s > 0) {
      const int sp = s - 1;
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
      ev[sp] = e;
      fv[sp] = f;
    }
    if (s < NKH) {
      bool kxr, kxl, kyr, kyl;
      hq = hdiff_of(dm, coeff, kxr, kxl, kyr, kyl);
      dq = dk;
      wq = wn;
      if constexpr (MASK) mr.record<TI>(min(max(k0 + dir * s, 0), nk - 1), s < nlev, active, kxr, kyr, kxl, kyl);
    }
  }
  // interface: the two innermost levels m-1 (top) and m (bottom)
  xch[half][0][ltid] = e;
  xch[half][1][ltid] = f;
  __syncthreads();
  const T eo = xch[1 - half][0][ltid], fo = xch[1 - half][1][ltid];
  const T et = half ? eo : e, ft = half ? fo : f;  // top's e_{m-1}, f_{m-1} (0 if nk = 1)
  const T eb = half ? e : eo, fb = half ? f : fo;  // bottom's e_m, f_m
  const T xm = (fb - eb * ft) * recip(T(1) - eb * et);
  const T xm1 = ft - et * xm;
  T x = half ? xm1 : xm;  // the value beyond this half's innermost level
#pragma unroll
  for (int s = NKH - 1; s >= 0; --s) {
    if (s < nlev) {  // uniform; no loads follow, so the branch costs no waits
      x = fv[s] - ev[s] * x;
      buf_st(vo.at(k0 + dir * s), ooff, x);
    }
  }
}

// one instantiation per half-column register class
#define GT4MI_NKH_CLASSES(X) X(8) X(16) X(24) X(32) X(40) X(48) X(64) X(80)

template <typename T>
constexpr int split_max_nk() {
  return sizeof(T) == 8 ? 80 : 160;  // both halves' factors in <= 256 VGPRs
}

template <typename T, int TI, int TJ>
hipError_t launch_split_classes(const StepArgs<T>& A, hipStream_t s) {
  const dim3 grid(A.ntiles), block(2 * TI * TJ);
  const int nkh = A.nk - A.nk / 2;
#define GT4MI_SPLIT_CASE(N)                                                                       \
  if constexpr (2 * N <= split_max_nk<T>()) {                                                     \
    if (nkh <= N) {                                                                               \
      if (A.mask)                                                                                 \
        hipLaunchKernelGGL((k_step_split<T, TI, TJ, N, GT4MI_PD, true>), grid, block, 0, s, A);  \
      else                                                                                        \
        hipLaunchKernelGGL((k_step_split<T, TI, TJ, N, GT4MI_PD, false>), grid, block, 0, s, A); \
      return hipGetLastError();                                                                   \
    }                                                                                             \
  }
  GT4MI_NKH_CLASSES(GT4MI_SPLIT_CASE)
#undef GT4MI_SPLIT_CASE
  return hipErrorInvalidValue;
}

}  // namespace gt4mi
