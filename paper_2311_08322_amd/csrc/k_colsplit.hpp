// k_colsplit.hpp -- the column solves alone (vertical advection and its
// adjoint), each column eliminated from both ends by two lanes.
//
// Forward:  T x = u + data.  Adjoint:  T^T lambda = x_bar.
// T^T is tridiagonal with sub-diagonal c_{k-1}, diagonal b_k and
// super-diagonal a_{k+1}; in terms of w the near/far coefficients of the two
// sweeps (see k_split.hpp) are those of T with the sign flipped:
//   top, level k:    near = c_{k-1} = +r/4 w_k,      far = a_{k+1} = -r/4 w_{k+1}
//   bottom, level k: near = a_{k+1} = -r/4 w_{k+1},  far = c_{k-1} = +r/4 w_k
// while the diagonal b_k = 1 + |a_k| + |c_k| = 1 + |near| + |far| is the same.
// So both solves are one kernel: a sign and the right-hand side differ.
#pragma once

#include "k_step.hpp"

// Levels loaded ahead by the column-only kernels (two loads per level, so
// they can run further ahead than the fused step at the same registers).
#ifndef GT4MI_COL_PD
#define GT4MI_COL_PD 2
#endif

namespace gt4mi {

// COL = 1: e and f of every level in VGPRs; COL = 2: f staged in `out`.
template <typename T, int NKH, int PD, bool ADJ, int COL>
__device__ __forceinline__ void column_split_tile(const StepArgs<T>& A, int tile, T (&xch)[2][2][kWG]) {
  constexpr int NT = kWG;
  const int half = __builtin_amdgcn_readfirstlane((int)threadIdx.x / NT);  // 0: top, 1: bottom
  const int ltid = threadIdx.x - half * NT;
  const int bi = tile % A.tiles_i, bj = tile / A.tiles_i;
  const int i = bi * 64 + (ltid & 63), j = bj * 4 + (ltid >> 6);
  const bool active = (i < A.ni) && (j < A.nj);
  const int ic = min(i, A.ni - 1), jc = min(j, A.nj - 1);
  const int nk = A.nk, m = nk / 2;
  const int nlev = half ? nk - m : m;
  const int nsteps = nk - m;
  const int k0 = half ? nk - 1 : 0, dir = half ? -1 : 1;
  constexpr uint32_t S = sizeof(T);
  // forward: u (rhs part 1), data (part 2); adjoint: u holds x_bar, data unused
  const LevelView vu = level_view(A.u, A.u_sj, A.u_sk, 0, 0, A.nj);
  const LevelView vd = level_view(A.data, A.d_sj, A.d_sk, 0, 0, A.nj);
  const LevelView vw = level_view(A.w, A.w_sj, A.w_sk, 0, 0, A.nj);
  const LevelView vo = level_view<T>(A.out, A.o_sj, A.o_sk, 0, 0, A.nj);
  const uint32_t uoff = ((uint32_t)ic + (uint32_t)jc * (uint32_t)A.u_sj) * S;
  const uint32_t doff = ((uint32_t)ic + (uint32_t)jc * (uint32_t)A.d_sj) * S;
  const uint32_t woff = ((uint32_t)ic + (uint32_t)jc * (uint32_t)A.w_sj) * S;
  const uint32_t ooff = active ? ((uint32_t)ic + (uint32_t)jc * (uint32_t)A.o_sj) * S : kOffNone;

  LevelCursor cur_u{vu.base + (int64_t)k0 * vu.level_bytes, dir * vu.level_bytes, vu.window};
  LevelCursor cur_d{vd.base + (int64_t)k0 * vd.level_bytes, dir * vd.level_bytes, vd.window};
  LevelCursor cur_w{vw.base + (int64_t)(half ? k0 : 1) * vw.level_bytes, dir * vw.level_bytes, vw.window};
  T pr[PD], pw[PD];
  auto issue = [&](int slot, int s) {
    T r = buf_ld(cur_u.rsrc(), uoff, T());
    if constexpr (!ADJ) r += buf_ld(cur_d.rsrc(), doff, T());
    pr[slot] = r;
    pw[slot] = buf_ld(cur_w.rsrc(), woff, T());
    const bool go = s + 1 < nlev;
    cur_u.advance(go);
    if constexpr (!ADJ) cur_d.advance(go);
    cur_w.advance(go);
  };
#pragma unroll
  for (int s = 0; s < PD; ++s) issue(s, s);

  T ev[NKH];
  T fv[COL == 1 ? NKH : 1];
  T wp = T(0), e = T(0), f = T(0);
  const T sn = (half ? A.r4 : -A.r4) * (ADJ ? T(-1) : T(1));
#pragma unroll
  for (int s = 0; s < NKH; ++s) {
    if (s >= nsteps) break;  // uniform; the only branch, so load counters stay exact
    __builtin_amdgcn_sched_barrier(0);
    const int slot = s % PD;
    const T rhs = pr[slot], wn = pw[slot];
    if (s + PD < NKH) issue(slot, s + PD);
    pin_prefetch();
    const bool act = s < nlev;
    const int k = k0 + dir * s;
    const T nr = (s > 0) ? sn * wp : T(0);
    const T fr = (half == 0 || k > 0) ? -sn * wn : T(0);
    const T b = T(1) + absv(nr) + absv(fr);
    const T inv = recip(b - nr * e);
    const T en = fr * inv;
    const T fn = (rhs - nr * f) * inv;
    e = act ? en : e;
    f = act ? fn : f;
    wp = act ? wn : wp;
    ev[s] = e;
    if constexpr (COL == 1) fv[s] = f;
    else buf_st(vo.at(min(max(k, 0), nk - 1)), act ? ooff : kOffNone, f);
  }
  xch[half][0][ltid] = e;
  xch[half][1][ltid] = f;
  __syncthreads();
  const T eo = xch[1 - half][0][ltid], fo = xch[1 - half][1][ltid];
  const T et = half ? eo : e, ft = half ? fo : f;
  const T eb = half ? e : eo, fb = half ? f : fo;
  const T xm = (fb - eb * ft) * recip(T(1) - eb * et);
  const T xm1 = ft - et * xm;
  T x = half ? xm1 : xm;
  if constexpr (COL == 1) {
#pragma unroll
    for (int s = NKH - 1; s >= 0; --s) {
      if (s < nlev) {
        const auto ro = vo.at(k0 + dir * s);
        x = fv[s] - ev[s] * x;
        buf_st(ro, ooff, x);
      }
    }
  } else {
    // The staged f comes back PDB levels ahead of its use.  The walk is
    // branch-free so that the load counters stay exact: levels this half
    // does not own read 0 and store nothing (offset outside the window), and
    // leave x unchanged.  Level s's value is consumed before slot s % PDB is
    // refilled with level s - PDB.
    constexpr int PDB = 4;
    T pf[PDB];
    auto level = [&](int s) { return vo.at(min(max(k0 + dir * s, 0), nk - 1)); };
#pragma unroll
    for (int s = NKH - 1 + PDB; s >= 0; --s) {
      if (s < NKH) {
        const bool act = s < nlev;
        const T xn = pf[s % PDB] - ev[s] * x;
        x = act ? xn : x;
        buf_st(level(s), act ? ooff : kOffNone, x);
      }
      const int sl = s - PDB;
      if (sl >= 0) pf[sl % PDB] = buf_ld(level(sl), sl < nlev ? ooff : kOffNone, T());
    }
  }
}

template <typename T, int NKH, int PD, bool ADJ, int COL>
__global__ void __launch_bounds__(2 * kWG) k_column_split(StepArgs<T> A) {
  __shared__ T xch[2][2][kWG];
  column_split_tile<T, NKH, PD, ADJ, COL>(A, xcd_tile(blockIdx.x, gridDim.x), xch);
}

// FP64 keeps e and f of both halves in VGPRs up to 96 levels, then stages f
// in the output up to 144; FP32 keeps both up to 160.
#ifndef GT4MI_COLSPLIT_REG_NK_F64
#define GT4MI_COLSPLIT_REG_NK_F64 96
#endif
#ifndef GT4MI_COLSPLIT_STAGED_CLASSES
#define GT4MI_COLSPLIT_STAGED_CLASSES(X) X(72)
#endif
constexpr int kColsplitRegNkF64 = GT4MI_COLSPLIT_REG_NK_F64;
constexpr int kColsplitStagedNkhF64 = 72;

template <typename T>
constexpr int column_split_max_nk() {
  return sizeof(T) == 8 ? 2 * kColsplitStagedNkhF64 : 160;
}

template <typename T, bool ADJ>
hipError_t launch_column_split_classes(StepArgs<T> A, hipStream_t s) {
  A.tiles_i = (A.ni + 63) / 64;
  A.ntiles = A.tiles_i * ((A.nj + 3) / 4);
  const dim3 grid(A.ntiles), block(2 * kWG);
  const int nkh = A.nk - A.nk / 2;
#define GT4MI_COLSPLIT_CASE(N)                                                                 \
  if constexpr (2 * N <= (sizeof(T) == 8 ? kColsplitRegNkF64 : 160)) {                         \
    if (nkh <= N) {                                                                            \
      hipLaunchKernelGGL((k_column_split<T, N, GT4MI_COL_PD, ADJ, 1>), grid, block, 0, s, A);     \
      return hipGetLastError();                                                                \
    }                                                                                          \
  }
  GT4MI_COLSPLIT_CASE(16) GT4MI_COLSPLIT_CASE(24) GT4MI_COLSPLIT_CASE(48) GT4MI_COLSPLIT_CASE(80)
#undef GT4MI_COLSPLIT_CASE
  if constexpr (sizeof(T) == 8) {
#define GT4MI_COLSPLIT_STAGED(N)                                                                 \
    if (nkh <= N) {                                                                              \
      hipLaunchKernelGGL((k_column_split<T, N, GT4MI_COL_PD, ADJ, 2>), grid, block, 0, s, A);    \
      return hipGetLastError();                                                                  \
    }
    GT4MI_COLSPLIT_STAGED_CLASSES(GT4MI_COLSPLIT_STAGED)
#undef GT4MI_COLSPLIT_STAGED
  }
  return hipErrorInvalidValue;
}

}  // namespace gt4mi
