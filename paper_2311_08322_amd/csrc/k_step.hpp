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
// The temporaries (lap, fluxes, c', d') never leave the chip: lap and the
// u-tile live in LDS, c'/d' of a column in the lane's VGPRs (unrolled k).
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace gt4mi {

__device__ __forceinline__ float absv(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double absv(double x) { return __builtin_fabs(x); }

template <int TI>
__device__ __forceinline__ void store_row_bits(uint8_t* row, int i0, uint64_t bits) {
  uint8_t* p = row + (i0 >> 3);
  if constexpr (TI == 64) {
    *reinterpret_cast<uint64_t*>(p) = bits;
  } else if constexpr (TI == 32) {
    *reinterpret_cast<uint32_t*>(p) = static_cast<uint32_t>(bits);
  } else {
    static_assert(TI == 16, "tile width must be 16, 32 or 64");
    *reinterpret_cast<uint16_t*>(p) = static_cast<uint16_t>(bits);
  }
}

// Record the limiter decisions of one level.  Every lane of the wave must
// call this (ballots).  A wave covers 64/TI rows of TI columns.
template <typename T, int TI>
__device__ __forceinline__ void record_mask(const StepArgs<T>& A, int k, int i0, int i, int j,
                                            bool active, bool kxr, bool kyr, bool kxl, bool kyl) {
  const uint64_t bx = __ballot(active && kxr);
  const uint64_t by = __ballot(active && kyr);
  const int lane = threadIdx.x & 63;
  if ((lane % TI) == 0 && j < A.nj) {
    const int sh = (lane / TI) * TI;
    const int64_t row = ((int64_t)k * A.nj + j) * A.ml.words * 8;
    store_row_bits<TI>(A.mask + A.ml.x_off + row, i0, bx >> sh);
    store_row_bits<TI>(A.mask + A.ml.y_off + row, i0, by >> sh);
  }
  if (active && i == 0) A.mask[A.ml.ex_off + (int64_t)k * A.nj + j] = kxl ? 1 : 0;
  if (active && j == 0) A.mask[A.ml.ey_off + (int64_t)k * A.ni + i] = kyl ? 1 : 0;
}

// Horizontal diffusion of the lane's own point at one level, from the
// u-tile (with halo) and the lap tile in LDS.  Returns out; the four flux
// decisions go to kxr/kxl/kyr/kyl (right/left, x/y).
template <typename T, int TI, int TJ>
__device__ __forceinline__ T hdiff_point(const T* __restrict__ U, const T* __restrict__ Lp, int ti,
                                         int tj, T coeff, bool& kxr, bool& kxl, bool& kyr,
                                         bool& kyl) {
  constexpr int HI = TI + 4, LI = TI + 2;
  const int cu = (tj + 2) * HI + (ti + 2);
  const int cl = (tj + 1) * LI + (ti + 1);
  const T uc = U[cu], lc = Lp[cl];
  const T fxr = Lp[cl + 1] - lc, gxr = U[cu + 1] - uc;
  const T fxl = lc - Lp[cl - 1], gxl = uc - U[cu - 1];
  const T fyr = Lp[cl + LI] - lc, gyr = U[cu + HI] - uc;
  const T fyl = lc - Lp[cl - LI], gyl = uc - U[cu - HI];
  kxr = flux_kept(fxr, gxr);
  kxl = flux_kept(fxl, gxl);
  kyr = flux_kept(fyr, gyr);
  kyl = flux_kept(fyl, gyl);
  const T Fxr = kxr ? fxr : T(0), Fxl = kxl ? fxl : T(0);
  const T Fyr = kyr ? fyr : T(0), Fyl = kyl ? fyl : T(0);
  return uc - coeff * ((Fxr - Fxl) + (Fyr - Fyl));
}

// lap = 4u - ((u[i-1] + u[i+1]) + (u[j-1] + u[j+1])) on the (TI+2) x (TJ+2)
// box around the tile.
template <typename T, int TI, int TJ>
__device__ __forceinline__ void lap_tile(const T* __restrict__ U, T* __restrict__ Lp, int tid) {
  constexpr int NT = TI * TJ, HI = TI + 4, LI = TI + 2, LN = (TI + 2) * (TJ + 2);
#pragma unroll
  for (int q = 0; q < (LN + NT - 1) / NT; ++q) {
    const int e = tid + q * NT;
    if (e < LN) {
      const int lj = e / LI, li = e - lj * LI;
      const int c = (lj + 1) * HI + (li + 1);
      const T s = (U[c - 1] + U[c + 1]) + (U[c - HI] + U[c + HI]);
      Lp[e] = T(4) * U[c] - s;
    }
  }
}

// ------------------------------------------------------------------ step
// COL = 1: c' and d' of the column in registers.
// COL = 2: c' in registers, d' staged in `out` (read back by the same lane).
template <typename T, int TI, int TJ, int NKMAX, int PD, int COL>
__global__ void __launch_bounds__(TI* TJ) k_step_fused(StepArgs<T> A) {
  constexpr int NT = TI * TJ;
  constexpr int HI = TI + 4, HN = (TI + 4) * (TJ + 4);
  constexpr int LN = (TI + 2) * (TJ + 2);
  constexpr int NLD = (HN + NT - 1) / NT;
  static_assert(NT == kWG, "tile must hold 256 columns");
  __shared__ T su[2][HN];
  __shared__ T sl[LN];

  const int tid = threadIdx.x, ti = tid % TI, tj = tid / TI;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int bi = tile % A.tiles_i, bj = tile / A.tiles_i;
  const int i0 = bi * TI, j0 = bj * TJ, i = i0 + ti, j = j0 + tj;
  const bool active = (i < A.ni) && (j < A.nj);
  const int nk = A.nk;

  // halo-tile load plan
  int64_t hoff[NLD];
  bool hok[NLD];
#pragma unroll
  for (int q = 0; q < NLD; ++q) {
    const int e = tid + q * NT;
    const int hj = e / HI, hi = e - hj * HI;
    const int gi = i0 - 2 + hi, gj = j0 - 2 + hj;
    hok[q] = (e < HN) && (gi < A.ni + 2) && (gj < A.nj + 2);
    hoff[q] = hok[q] ? (int64_t)gi + (int64_t)gj * A.u_sj : 0;
  }
  const int64_t doff = active ? (int64_t)i + (int64_t)j * A.d_sj : 0;
  const int64_t woff = active ? (int64_t)i + (int64_t)j * A.w_sj : 0;
  const int64_t ooff = (int64_t)i + (int64_t)j * A.o_sj;

  // prefetch ring: slot k % PD holds level k
  T pu[PD][NLD], pd[PD], pw[PD];
  auto issue = [&](int s, int k) {
#pragma unroll
    for (int q = 0; q < NLD; ++q) pu[s][q] = hok[q] ? A.u[hoff[q] + (int64_t)k * A.u_sk] : T(0);
    pd[s] = active ? A.data[doff + (int64_t)k * A.d_sk] : T(0);
    pw[s] = (active && k + 1 < nk) ? A.w[woff + (int64_t)(k + 1) * A.w_sk] : T(0);
  };
#pragma unroll
  for (int s = 0; s < PD; ++s)
    if (s < nk) issue(s, s);

  T cp[NKMAX];
  T dp[COL == 1 ? NKMAX : 1];
  T wk = T(0), cprev = T(0), dprev = T(0);
  const T coeff = A.coeff, r4 = A.r4;

#pragma unroll
  for (int k = 0; k < NKMAX; ++k) {
    if (k < nk) {
      const int s = k % PD;
      T* U = su[k & 1];
#pragma unroll
      for (int q = 0; q < NLD; ++q)
        if (tid + q * NT < HN) U[tid + q * NT] = pu[s][q];
      const T dk = pd[s], wk1 = pw[s];
      if (k + PD < nk) issue(s, k + PD);
      __syncthreads();
      lap_tile<T, TI, TJ>(U, sl, tid);
      __syncthreads();
      bool kxr, kxl, kyr, kyl;
      const T h = hdiff_point<T, TI, TJ>(U, sl, ti, tj, coeff, kxr, kxl, kyr, kyl);
      if (A.mask) record_mask<T, TI>(A, k, i0, i, j, active, kxr, kyr, kxl, kyl);
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
        if (active) A.out[ooff + (int64_t)k * A.o_sk] = dprev;
      }
      wk = wk1;
    }
  }
  // Thomas back substitution (c'_{nk-1} = 0 starts it from x = d')
  T x = T(0);
#pragma unroll
  for (int k = NKMAX - 1; k >= 0; --k) {
    if (k < nk) {
      T* o = A.out + ooff + (int64_t)k * A.o_sk;
      if constexpr (COL == 1) {
        x = dp[k] - cp[k] * x;
        if (active) *o = x;
      } else {
        if (active) {
          x = *o - cp[k] * x;
          *o = x;
        }
      }
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
  const int64_t uoff = (int64_t)i + (int64_t)j * A.u_sj;
  const int64_t doff = (int64_t)i + (int64_t)j * A.d_sj;
  const int64_t woff = (int64_t)i + (int64_t)j * A.w_sj;
  const int64_t ooff = (int64_t)i + (int64_t)j * A.o_sj;
  T pu[PD], pd[PD], pw[PD];
  auto issue = [&](int s, int k) {
    pu[s] = A.u[uoff + (int64_t)k * A.u_sk];
    pd[s] = A.data[doff + (int64_t)k * A.d_sk];
    pw[s] = (k + 1 < nk) ? A.w[woff + (int64_t)(k + 1) * A.w_sk] : T(0);
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
      const T a = (k > 0) ? -r4 * wk : T(0);
      const T c = (k < nk - 1) ? r4 * wk1 : T(0);
      const T b = T(1) + absv(a) + absv(c);
      const T inv = recip(b - a * cprev);
      cprev = c * inv;
      dprev = (dk - a * dprev) * inv;
      cp[k] = cprev;
      if constexpr (COL == 1) dp[k] = dprev;
      else A.out[ooff + (int64_t)k * A.o_sk] = dprev;
      wk = wk1;
    }
  }
  T x = T(0);
#pragma unroll
  for (int k = NKMAX - 1; k >= 0; --k) {
    if (k < nk) {
      T* o = A.out + ooff + (int64_t)k * A.o_sk;
      if constexpr (COL == 1) x = dp[k] - cp[k] * x;
      else x = *o - cp[k] * x;
      *o = x;
    }
  }
}

// ------------------------------------------------------------------ hdiff
// Tile marched over the levels [k0, k1) of the launch, next level's u-tile
// prefetched in registers while the current one is computed.
template <typename T, int TI, int TJ>
__global__ void __launch_bounds__(TI* TJ) k_hdiff_fused(StepArgs<T> A) {
  constexpr int NT = TI * TJ;
  constexpr int HI = TI + 4, HN = (TI + 4) * (TJ + 4);
  constexpr int LN = (TI + 2) * (TJ + 2);
  constexpr int NLD = (HN + NT - 1) / NT;
  __shared__ T su[2][HN];
  __shared__ T sl[LN];
  const int tid = threadIdx.x, ti = tid % TI, tj = tid / TI;
  const int tile = xcd_tile(blockIdx.x, A.ntiles) ;
  const int bi = tile % A.tiles_i, bj = tile / A.tiles_i;
  const int i0 = bi * TI, j0 = bj * TJ, i = i0 + ti, j = j0 + tj;
  const bool active = (i < A.ni) && (j < A.nj);
  const int kb = blockIdx.y;
  const int kbeg = A.k0 + kb * A.k1, kend = min(kbeg + A.k1, A.nk);  // k1 = levels per block
  int64_t hoff[NLD];
  bool hok[NLD];
#pragma unroll
  for (int q = 0; q < NLD; ++q) {
    const int e = tid + q * NT;
    const int hj = e / HI, hi = e - hj * HI;
    const int gi = i0 - 2 + hi, gj = j0 - 2 + hj;
    hok[q] = (e < HN) && (gi < A.ni + 2) && (gj < A.nj + 2);
    hoff[q] = hok[q] ? (int64_t)gi + (int64_t)gj * A.u_sj : 0;
  }
  const int64_t ooff = (int64_t)i + (int64_t)j * A.o_sj;
  T pu[NLD];
#pragma unroll
  for (int q = 0; q < NLD; ++q) pu[q] = (hok[q] && kbeg < kend) ? A.u[hoff[q] + (int64_t)kbeg * A.u_sk] : T(0);
  for (int k = kbeg; k < kend; ++k) {
    T* U = su[k & 1];
#pragma unroll
    for (int q = 0; q < NLD; ++q)
      if (tid + q * NT < HN) U[tid + q * NT] = pu[q];
    if (k + 1 < kend) {
#pragma unroll
      for (int q = 0; q < NLD; ++q) pu[q] = hok[q] ? A.u[hoff[q] + (int64_t)(k + 1) * A.u_sk] : T(0);
    }
    __syncthreads();
    lap_tile<T, TI, TJ>(U, sl, tid);
    __syncthreads();
    bool kxr, kxl, kyr, kyl;
    const T h = hdiff_point<T, TI, TJ>(U, sl, ti, tj, A.coeff, kxr, kxl, kyr, kyl);
    if (A.mask) record_mask<T, TI>(A, k, i0, i, j, active, kxr, kyr, kxl, kyl);
    if (active) A.out[ooff + (int64_t)k * A.o_sk] = h;
  }
}

// ------------------------------------------------------------------ class dispatch
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
      hipLaunchKernelGGL((k_step_fused<T, TI, TJ, N, 2, COL>), grid, block, 0, s, A); \
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
