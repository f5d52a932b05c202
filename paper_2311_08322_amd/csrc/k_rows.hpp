// k_rows.hpp -- fused time step with the horizontal neighbours exchanged
// between the lanes of a wave instead of through LDS.
//
// Tile of 64 x 4 columns, 8 waves.  Wave w owns the row segment
// (i0 .. i0+63, j0 + w % 4) and eliminates its columns from the top
// (w < 4) or from the bottom (w >= 4) of the column, exactly as the
// two-ended solve of k_split.hpp.  Per level a lane loads u at its own
// column for rows j-2 .. j+2; u(i +- 1) of rows j-1, j, j+1 and the
// Laplacian at (i +- 1, j) come from the adjacent lanes by whole-wave DPP
// shifts, and the two end lanes of the segment receive what lies beyond it
// (columns i0-1, i0-2 and i0+64, i0+65) from four edge loads.  Nothing goes
// through LDS and no barrier separates the levels: the waves of a tile run
// independently and meet once, at the interface of the two-ended solve.
#pragma once

#include "k_split.hpp"

namespace gt4mi {

// Whole-wave DPP shifts (gfx9 wave_shr:1 / wave_shl:1).  A lane whose
// source lies outside the wave keeps `old`.
constexpr int kDppWaveShl1 = 0x130;  // lane l reads lane l + 1
constexpr int kDppWaveShr1 = 0x138;  // lane l reads lane l - 1

template <int CTRL>
__device__ __forceinline__ float dpp_move(float old, float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                               __builtin_bit_cast(int, v), CTRL, 0xf, 0xf,
                                                               false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double old, double v) {
  const u32x2_t o = __builtin_bit_cast(u32x2_t, old), x = __builtin_bit_cast(u32x2_t, v);
  u32x2_t r;
  r.x = (unsigned)__builtin_amdgcn_update_dpp((int)o.x, (int)x.x, CTRL, 0xf, 0xf, false);
  r.y = (unsigned)__builtin_amdgcn_update_dpp((int)o.y, (int)x.y, CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, r);
}
// value of the lane to the left (i - 1); lane 0 takes `edge`
template <typename T>
__device__ __forceinline__ T from_left(T v, T edge) {
  return dpp_move<kDppWaveShr1>(edge, v);
}
// value of the lane to the right (i + 1); lane 63 takes `edge`
template <typename T>
__device__ __forceinline__ T from_right(T v, T edge) {
  return dpp_move<kDppWaveShl1>(edge, v);
}

template <typename T, int NKH, int PD, bool MASK, int COL>
__device__ __forceinline__ void step_rows_tile(const StepArgs<T>& A, int tile, T (&xch)[2][2][kWG]) {
  constexpr int TI = 64;
  constexpr int NT = kWG;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int half = wave >> 2;  // 0: top, 1: bottom
  const int lane = threadIdx.x & 63;
  const int ltid = threadIdx.x - half * NT;
  const int bi = tile % A.tiles_i, bj = tile / A.tiles_i;
  const int i0 = bi * TI, j0 = bj * 4;
  const int i = i0 + lane, j = j0 + (wave & 3);
  const int ni = A.ni, nj = A.nj;
  const bool active = (i < ni) && (j < nj);
  // u is read at columns up to ni + 1 (the halo): the lanes just past a
  // ragged edge supply the neighbours of the last interior lane
  const int iu = min(i, ni + 1), ic = min(i, ni - 1), jc = min(j, nj - 1);
  const int nk = A.nk, m = nk / 2;
  const int nlev = half ? nk - m : m;
  const int nsteps = nk - m;
  const int k0 = half ? nk - 1 : 0, dir = half ? -1 : 1;
  constexpr uint32_t S = sizeof(T);
  const LevelView vu = level_view(A.u, A.u_sj, A.u_sk, -2, -2, nj + 4);
  const LevelView vd = level_view(A.data, A.d_sj, A.d_sk, 0, 0, nj);
  const LevelView vw = level_view(A.w, A.w_sj, A.w_sk, 0, 0, nj);
  const LevelView vo = level_view<T>(A.out, A.o_sj, A.o_sk, 0, 0, nj);
  const uint32_t usj = (uint32_t)A.u_sj;
  auto uoff = [&](int ii, int jj) { return ((uint32_t)(ii + 2) + (uint32_t)(jj + 2) * usj) * S; };
  uint32_t roff[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) roff[d] = uoff(iu, jc + d - 2);
  // edge loads: lane 0 reads left of the segment, lane 63 right of it
  const bool le = lane == 0, re = lane == TI - 1;
  const int ec1 = le ? i0 - 1 : min(i0 + TI, ni + 1);
  const int ec2 = le ? i0 - 2 : min(i0 + TI + 1, ni + 1);
  uint32_t eoff[4];
  eoff[0] = (le || re) ? uoff(ec1, jc - 1) : kOffNone;
  eoff[1] = (le || re) ? uoff(ec1, jc) : kOffNone;
  eoff[2] = (le || re) ? uoff(ec1, jc + 1) : kOffNone;
  eoff[3] = (le || re) ? uoff(ec2, jc) : kOffNone;
  const uint32_t doff = ((uint32_t)ic + (uint32_t)jc * (uint32_t)A.d_sj) * S;
  const uint32_t woff = ((uint32_t)ic + (uint32_t)jc * (uint32_t)A.w_sj) * S;
  const uint32_t ooff = active ? ((uint32_t)ic + (uint32_t)jc * (uint32_t)A.o_sj) * S : kOffNone;
  MaskRec mr;
  if constexpr (MASK) mr.init<T, TI>(A, lane, i0, i, j, active);

  LevelCursor cur_u{vu.base + (int64_t)k0 * vu.level_bytes, dir * vu.level_bytes, vu.window};
  LevelCursor cur_d{vd.base + (int64_t)k0 * vd.level_bytes, dir * vd.level_bytes, vd.window};
  LevelCursor cur_w{vw.base + (int64_t)(half ? k0 : 1) * vw.level_bytes, dir * vw.level_bytes, vw.window};
  T pr[PD][5], pe[PD][4], pd[PD], pw[PD];
  auto issue = [&](int slot, int s) {
    const auto ru = cur_u.rsrc();
#pragma unroll
    for (int d = 0; d < 5; ++d) pr[slot][d] = buf_ld<GT4MI_CP_HALO>(ru, roff[d], T());
#pragma unroll
    for (int q = 0; q < 4; ++q) pe[slot][q] = buf_ld<GT4MI_CP_HALO>(ru, eoff[q], T());
    pd[slot] = buf_ld<GT4MI_CP_ONCE>(cur_d.rsrc(), doff, T());
    pw[slot] = buf_ld<GT4MI_CP_ONCE>(cur_w.rsrc(), woff, T());
    const bool go = s + 1 < nlev;
    cur_u.advance(go);
    cur_d.advance(go);
    cur_w.advance(go);
  };
#pragma unroll
  for (int s = 0; s < PD; ++s) issue(s, s);

  T ev[NKH];
  T fv[COL == 1 ? NKH : 1];
  T wp = T(0), e = T(0), f = T(0);
  const T coeff = A.coeff;
  const T sn = half ? A.r4 : -A.r4;
  T hq = T(0), dq = T(0), wq = T(0);

  auto eliminate = [&](int sp) {
    const bool act = sp < nlev;
    const int k = k0 + dir * sp;
    const T nr = (sp > 0) ? sn * wp : T(0);
    const T fr = (half == 0 || k > 0) ? -sn * wq : T(0);
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
    const T r0 = pr[slot][0], r1 = pr[slot][1], r2 = pr[slot][2], r3 = pr[slot][3], r4 = pr[slot][4];
    const T e1 = pe[slot][0], e2 = pe[slot][1], e3 = pe[slot][2], e4 = pe[slot][3];
    const T dk = pd[slot], wn = pw[slot];
    if (s + PD < NKH) issue(slot, s + PD);
    // i-neighbours of rows j-1, j, j+1
    const T uw = from_left(r2, e2), ue = from_right(r2, e2);
    const T nw = from_left(r1, e1), ne = from_right(r1, e1);
    const T sw = from_left(r3, e3), se = from_right(r3, e3);
    // lap = 4u - ((u[i-1] + u[i+1]) + (u[j-1] + u[j+1]))
    const T L00 = T(4) * r2 - ((uw + ue) + (r1 + r3));
    const T L0m = T(4) * r1 - ((nw + ne) + (r0 + r2));
    const T L0p = T(4) * r3 - ((sw + se) + (r2 + r4));
    // at the end lanes: the Laplacian just beyond the segment, (i0-1, j) or (i0+64, j)
    const T LE = T(4) * e2 - ((e4 + r2) + (e1 + e3));
    const T Lm0 = from_left(L00, LE), Lp0 = from_right(L00, LE);
    if (s > 0) {
      const bool act = eliminate(s - 1);
      ev[s - 1] = e;
      if constexpr (COL == 1) fv[s - 1] = f;
      else buf_st(vo.at(min(max(k0 + dir * (s - 1), 0), nk - 1)), act ? ooff : kOffNone, f);
    }
    const T fxr = Lp0 - L00, fxl = L00 - Lm0, fyr = L0p - L00, fyl = L00 - L0m;
    const bool kxr = flux_kept(fxr, ue - r2);
    const bool kxl = flux_kept(fxl, r2 - uw);
    const bool kyr = flux_kept(fyr, r3 - r2);
    const bool kyl = flux_kept(fyl, r2 - r1);
    const T Fxr = kxr ? fxr : T(0), Fxl = kxl ? fxl : T(0);
    const T Fyr = kyr ? fyr : T(0), Fyl = kyl ? fyl : T(0);
    hq = r2 - coeff * ((Fxr - Fxl) + (Fyr - Fyl));
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
  xch[half][0][ltid] = e;
  xch[half][1][ltid] = f;
  __syncthreads();
  const T eo = xch[1 - half][0][ltid], fo = xch[1 - half][1][ltid];
  const T et = half ? eo : e, ft = half ? fo : f;
  const T eb = half ? e : eo, fb = half ? f : fo;
  const T xm = (fb - eb * ft) * recip(T(1) - eb * et);
  const T xm1 = ft - et * xm;
  T x = half ? xm1 : xm;
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

template <typename T, int NKH, int PD, bool MASK, int COL>
__global__ void __launch_bounds__(2 * kWG) k_step_rows(StepArgs<T> A) {
  __shared__ T xch[2][2][kWG];
  step_rows_tile<T, NKH, PD, MASK, COL>(A, xcd_tile(blockIdx.x, gridDim.x), xch);
}

// The same register classes as the LDS form (k_split.hpp); tile 64 x 4.
template <typename T>
hipError_t launch_rows_classes(const StepArgs<T>& A, hipStream_t s) {
  const dim3 grid(A.ntiles), block(2 * kWG);
  const int nkh = A.nk - A.nk / 2;
#define GT4MI_ROWS_LAUNCH(N, C)                                                                  \
  {                                                                                              \
    if (A.mask)                                                                                  \
      hipLaunchKernelGGL((k_step_rows<T, N, GT4MI_PD, true, C>), grid, block, 0, s, A);         \
    else                                                                                         \
      hipLaunchKernelGGL((k_step_rows<T, N, GT4MI_PD, false, C>), grid, block, 0, s, A);        \
    return hipGetLastError();                                                                    \
  }
#define GT4MI_ROWS_CASE(N)                                                      \
  if constexpr (2 * N <= (sizeof(T) == 8 ? kSplitRegNkF64 : 160)) {             \
    if (nkh <= N) GT4MI_ROWS_LAUNCH(N, 1)                                       \
  }
  GT4MI_NKH_CLASSES(GT4MI_ROWS_CASE)
  if constexpr (sizeof(T) == 8) {
    if (nkh <= kSplitStagedNkhF64) GT4MI_ROWS_LAUNCH(kSplitStagedNkhF64, 2)
  }
#undef GT4MI_ROWS_CASE
#undef GT4MI_ROWS_LAUNCH
  return hipErrorInvalidValue;
}

}  // namespace gt4mi
