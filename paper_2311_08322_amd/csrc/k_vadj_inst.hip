// k_vadj_inst.hip -- the register-resident column adjoint lambda = T^{-T} x_bar
// (derivation at the top of k_adjoint.hip), instantiated per register class
// of the column length for one (dtype, column store) per compilation:
//   -DGT4MI_T=double|float -DGT4MI_COL=1|2
#include "common.hpp"
#include "launch.hpp"

namespace gt4mi {

__device__ __forceinline__ float absa(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double absa(double x) { return __builtin_fabs(x); }

// COL = 1: c' and y in registers; COL = 2: y staged in the lambda field.
template <typename T, int NKMAX, int PD, int COL>
__global__ void __launch_bounds__(kWG) k_vadv_adjoint_fused(AdjArgs<T> A) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int bi = tile % A.tiles_i, bj = tile / A.tiles_i;
  const int i = bi * 64 + (threadIdx.x & 63), j = bj * 4 + (threadIdx.x >> 6);
  if (i >= A.ni || j >= A.nj) return;
  const int nk = A.nk;
  const int64_t xoff = (int64_t)i + (int64_t)j * A.x_sj;
  const int64_t woff = (int64_t)i + (int64_t)j * A.w_sj;
  const int64_t loff = (int64_t)i + (int64_t)j * A.l_sj;
  T px[PD], pw[PD];
  auto issue = [&](int s, int k) {
    px[s] = A.xbar[xoff + (int64_t)k * A.x_sk];
    pw[s] = (k + 1 < nk) ? A.w[woff + (int64_t)(k + 1) * A.w_sk] : T(0);
  };
#pragma unroll
  for (int s = 0; s < PD; ++s)
    if (s < nk) issue(s, s);
  T cp[NKMAX];
  T yv[COL == 1 ? NKMAX : 1];
  T wk = T(0), cprev = T(0), ccoef_prev = T(0), yprev = T(0);
  const T r4 = A.r4;
#pragma unroll
  for (int k = 0; k < NKMAX; ++k) {
    if (k < nk) {
      const int s = k % PD;
      const T xb = px[s], wk1 = pw[s];
      if (k + PD < nk) issue(s, k + PD);
      pin_prefetch();
      const T a = (k > 0) ? -r4 * wk : T(0);
      const T c = (k < nk - 1) ? r4 * wk1 : T(0);
      const T b = T(1) + absa(a) + absa(c);
      const T inv = recip(b - a * cprev);
      yprev = (xb - ccoef_prev * yprev) * inv;
      cprev = c * inv;
      ccoef_prev = c;
      cp[k] = cprev;
      if constexpr (COL == 1) yv[k] = yprev;
      else A.lam[loff + (int64_t)k * A.l_sk] = yprev;
      wk = wk1;
    }
  }
  T lam = T(0);
#pragma unroll
  for (int k = NKMAX - 1; k >= 0; --k) {
    if (k < nk) {
      T* l = A.lam + loff + (int64_t)k * A.l_sk;
      if constexpr (COL == 1) lam = yv[k] + cp[k] * lam;
      else lam = *l + cp[k] * lam;
      *l = lam;
    }
  }
}


template <typename T, int COL>
hipError_t launch_vadj_classes(const AdjArgs<T>& A, hipStream_t s) {
  const dim3 grid(A.ntiles), block(kWG);
#define GT4MI_VADJ_CASE(N)                                                                \
  if constexpr (!(sizeof(T) == 8 && COL == 1 && N > 96)) {                                \
    if (A.nk <= N) {                                                                      \
      hipLaunchKernelGGL((k_vadv_adjoint_fused<T, N, 2, COL>), grid, block, 0, s, A);    \
      return hipGetLastError();                                                           \
    }                                                                                     \
  }
  GT4MI_VADJ_CASE(16) GT4MI_VADJ_CASE(32) GT4MI_VADJ_CASE(48) GT4MI_VADJ_CASE(64)
  GT4MI_VADJ_CASE(80) GT4MI_VADJ_CASE(96) GT4MI_VADJ_CASE(128) GT4MI_VADJ_CASE(160)
#undef GT4MI_VADJ_CASE
  return hipErrorInvalidValue;
}

template hipError_t launch_vadj_classes<GT4MI_T, GT4MI_COL>(const AdjArgs<GT4MI_T>&, hipStream_t);

}  // namespace gt4mi
