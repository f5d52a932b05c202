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

template <typename T, int TI, int TJ, int NKH, int PD>
__global__ void __launch_bounds__(2 * TI * TJ) k_step_split(StepArgs<T> A) {
  using TA = TileAddr<T, TI, TJ>;
  constexpr int NT = TA::NT, HI = TA::HI, NLD = TA::NLD;
  static_assert(NT == kWG, "tile must hold 256 columns");
  __shared__ T su[2][2][NLD * NT];  // [half][level parity]
  __shared__ T xch[2][2][NT];       // innermost (e, f) of each half and column

  const int half = __builtin_amdgcn_readfirstlane((int)threadIdx.x / NT);  // 0: top, 1: bottom
  const int ltid = threadIdx.x - half * NT;
  TA t;
  t.init_lane(ltid, xcd_tile(blockIdx.x, gridDim.x), A.tiles_i, A.ni, A.nj, A.u_sj);
  const int nk = A.nk, m = nk / 2;
  const int nlev = half ? nk - m : m;  // levels this half eliminates
  const int nsteps = nk - m;           // the larger of the two
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

  // step s works on level s (top) or nk-1-s (bottom); the w level that is
  // new at step s is k+1 (top: c_k) or k (bottom: a_k)
  T pu[PD][NLD], pd[PD], pw[PD];
  auto issue = [&](int slot, int s) {
    const int k = half ? nk - 1 - s : s;
    const auto ru = vu.at(k);
#pragma unroll
    for (int q = 0; q < NLD; ++q) pu[slot][q] = buf_ld(ru, t.hoff[q], T());
    pd[slot] = buf_ld(vd.at(k), doff, T());
    pw[slot] = buf_ld(vw.at(half ? k : k + 1), woff, T());
  };
#pragma unroll
  for (int s = 0; s < PD; ++s)
    if (s < nlev) issue(s, s);

  T ev[NKH], fv[NKH];
  T wp = T(0), e = T(0), f = T(0);
  const T coeff = A.coeff;
  const T sn = half ? A.r4 : -A.r4;  // near coefficient per unit w: top a = -r/4 w, bottom c = +r/4 w
  const int cu = (t.tj + 2) * HI + (t.ti + 2);

#pragma unroll
  for (int s = 0; s < NKH; ++s) {
    if (s < nsteps) {
      const bool act = s < nlev;
      const int slot = s % PD;
      T* U = su[half][s & 1];
      T dk = T(0), wn = T(0);
      if (act) {
#pragma unroll
        for (int q = 0; q < NLD; ++q) U[ltid + q * NT] = pu[slot][q];
        dk = pd[slot];
        wn = pw[slot];
        if (s + PD < nlev) issue(slot, s + PD);
      }
      __syncthreads();
      if (act) {
        const int k = half ? nk - 1 - s : s;
        bool kxr, kxl, kyr, kyl;
        const T h = hdiff_diamond<T, HI>(U + cu, coeff, kxr, kxl, kyr, kyl);
        if (A.mask) mw.record<TI>(k, active, kxr, kyr, kxl, kyl);
        const T nr = (s > 0) ? sn * wp : T(0);                  // a_k (top, k >= 1) / c_k (bottom, k <= nk-2)
        const T fr = (half == 0 || k > 0) ? -sn * wn : T(0);   // c_k (top) / a_k (bottom, k >= 1)
        const T b = T(1) + absv(nr) + absv(fr);
        const T inv = recip(b - nr * e);
        e = fr * inv;
        f = ((h + dk) - nr * f) * inv;
        ev[s] = e;
        fv[s] = f;
        wp = wn;
      }
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
    if (s < nlev) {
      const int k = half ? nk - 1 - s : s;
      x = fv[s] - ev[s] * x;
      if (active) buf_st(vo.at(k), ooff, x);
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
#define GT4MI_SPLIT_CASE(N)                                                                 \
  if constexpr (2 * N <= split_max_nk<T>()) {                                               \
    if (nkh <= N) {                                                                         \
      hipLaunchKernelGGL((k_step_split<T, TI, TJ, N, GT4MI_PD>), grid, block, 0, s, A);    \
      return hipGetLastError();                                                             \
    }                                                                                       \
  }
  GT4MI_NKH_CLASSES(GT4MI_SPLIT_CASE)
#undef GT4MI_SPLIT_CASE
  return hipErrorInvalidValue;
}

}  // namespace gt4mi
