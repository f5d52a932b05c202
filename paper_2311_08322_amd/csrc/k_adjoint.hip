// k_adjoint.hip -- adjoint (reverse-mode) kernels of the two stencils.
//
// Column adjoint: lambda = T^{-T} x_bar.  With T = L U (Thomas: U has the
// pivots m_k on its diagonal and c_k above it, L is unit lower with
// a_k / m_{k-1} below), T^T = U^T L^T, so
//   y_k      = (x_bar_k - c_{k-1} y_{k-1}) / m_k            (FORWARD)
//   lambda_k = y_k - (a_{k+1} / m_k) lambda_{k+1}            (BACKWARD)
// and since a_{k+1} = -c_k exactly (both are +-dt_dz/4 * w_{k+1}),
//   lambda_k = y_k + c'_k lambda_{k+1},   c'_k = c_k / m_k,
// the same two sweeps as the forward solve, with the pivots rebuilt from w.
//
// Horizontal adjoint: the transpose of the diffusion's Jacobian with the
// forward limiter decisions held fixed:
//   gx(q)    = Mx(q) * (-coeff) * (lambda(q) - lambda(q + e_i))
//   gy(q)    = My(q) * (-coeff) * (lambda(q) - lambda(q + e_j))
//   lbar(q)  = gx(q - e_i) - gx(q) + gy(q - e_j) - gy(q)
//   ubar(p)  = [p in I] lambda(p) + 4 lbar(p) - lbar(p +- e_i) - lbar(p +- e_j)
// with lambda = 0 outside the interior and fluxes outside their definition
// sets ([-1,ni) x [0,nj) and [0,ni) x [-1,nj)) equal to zero.
#include <string.h>

#include "common.hpp"
#include "k_hadj_strip.hpp"
#include "launch.hpp"

namespace gt4mi {

__device__ __forceinline__ float absa(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double absa(double x) { return __builtin_fabs(x); }

// ---------------------------------------------------------------- columns
// (the register-resident column kernel is in k_vadj_inst.hip)
template <typename T>
__global__ void __launch_bounds__(kWG) k_vadv_adjoint_fwd_plain(AdjArgs<T> A, T* __restrict__ yw,
                                                                T* __restrict__ cw) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y;
  if (i >= A.ni || j >= A.nj) return;
  const int64_t plane = (int64_t)A.ni * A.nj, col = (int64_t)i + (int64_t)j * A.ni;
  const T* xb = A.xbar + (int64_t)i + (int64_t)j * A.x_sj;
  const T* w = A.w + (int64_t)i + (int64_t)j * A.w_sj;
  T wk = T(0), cprev = T(0), cc = T(0), y = T(0);
  for (int k = 0; k < A.nk; ++k) {
    const T wk1 = (k + 1 < A.nk) ? w[(int64_t)(k + 1) * A.w_sk] : T(0);
    const T a = (k > 0) ? -A.r4 * wk : T(0);
    const T c = (k < A.nk - 1) ? A.r4 * wk1 : T(0);
    const T b = T(1) + absa(a) + absa(c);
    const T inv = recip(b - a * cprev);
    y = (xb[(int64_t)k * A.x_sk] - cc * y) * inv;
    cprev = c * inv;
    cc = c;
    yw[col + k * plane] = y;
    cw[col + k * plane] = cprev;
    wk = wk1;
  }
}

template <typename T>
__global__ void __launch_bounds__(kWG) k_vadv_adjoint_bwd_plain(AdjArgs<T> A, const T* __restrict__ yw,
                                                                const T* __restrict__ cw) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y;
  if (i >= A.ni || j >= A.nj) return;
  const int64_t plane = (int64_t)A.ni * A.nj, col = (int64_t)i + (int64_t)j * A.ni;
  T* l = A.lam + (int64_t)i + (int64_t)j * A.l_sj;
  T lam = T(0);
  for (int k = A.nk - 1; k >= 0; --k) {
    lam = yw[col + k * plane] + cw[col + k * plane] * lam;
    l[(int64_t)k * A.l_sk] = lam;
  }
}

// ---------------------------------------------------------------- horizontal
// (the gather kernel is in k_hadj_strip.hpp)

// ---------------------------------------------------------------- launchers
template <typename T>
hipError_t launch_vadv_adjoint(AdjArgs<T> A, int impl_plain, T* ws_y, T* ws_c, hipStream_t s) {
  if (impl_plain) {
    const dim3 blk(64, 4), grd((A.ni + 63) / 64, (A.nj + 3) / 4);
    hipLaunchKernelGGL(k_vadv_adjoint_fwd_plain<T>, grd, blk, 0, s, A, ws_y, ws_c);
    hipLaunchKernelGGL(k_vadv_adjoint_bwd_plain<T>, grd, blk, 0, s, A, ws_y, ws_c);
    return hipGetLastError();
  }
  if (A.nk <= column_split_limit(sizeof(T))) {
    // the two-ended column kernel with T^T: right-hand side x_bar, output lambda
    StepArgs<T> C;
    memset(&C, 0, sizeof C);
    C.u = A.xbar;
    C.u_sj = A.x_sj;
    C.u_sk = A.x_sk;
    C.data = A.xbar;  // unused by the adjoint
    C.d_sj = A.x_sj;
    C.d_sk = A.x_sk;
    C.w = A.w;
    C.w_sj = A.w_sj;
    C.w_sk = A.w_sk;
    C.out = A.lam;
    C.o_sj = A.l_sj;
    C.o_sk = A.l_sk;
    C.ni = A.ni;
    C.nj = A.nj;
    C.nk = A.nk;
    C.r4 = A.r4;
    return launch_column_split_classes<T, true>(C, s);
  }
  A.tiles_i = (A.ni + 63) / 64;
  A.ntiles = A.tiles_i * ((A.nj + 3) / 4);
  if constexpr (sizeof(T) == 4) {
    return launch_vadj_classes<T, 1>(A, s);
  } else {
    // FP64 beyond 96 levels stages y in the output (lambda) field
    if (A.nk > 96) return launch_vadj_classes<T, 2>(A, s);
    return launch_vadj_classes<T, 1>(A, s);
  }
}

// strips of 60 x strip_rows outputs over the padded domain, four per
// workgroup, one level per grid row
template <typename T>
hipError_t launch_hdiff_adjoint(AdjArgs<T> A, hipStream_t s) {
  const bool var = A.kappa != nullptr && A.lam != nullptr;  // per-point coefficient
  if constexpr (sizeof(T) == 4) {
    // binary32: two columns per lane, strips of 124 x strip_rows outputs
    A.tiles_i = (A.ni + 4 + kStripOut2 - 1) / kStripOut2;
    A.ntiles = A.tiles_i * ((A.nj + 4 + strip_rows<T>() - 1) / strip_rows<T>());
    const dim3 grid((A.ntiles + kStripsPerWG - 1) / kStripsPerWG, A.nk), block(kWG);
    const bool pair = lambda_pairs_ok(A);
    if (var && pair)
      hipLaunchKernelGGL((k_hdiff_adjoint_strip2<true, true>), grid, block, 0, s, A);
    else if (var)
      hipLaunchKernelGGL((k_hdiff_adjoint_strip2<true, false>), grid, block, 0, s, A);
    else if (pair)
      hipLaunchKernelGGL((k_hdiff_adjoint_strip2<false, true>), grid, block, 0, s, A);
    else
      hipLaunchKernelGGL((k_hdiff_adjoint_strip2<false, false>), grid, block, 0, s, A);
    return hipGetLastError();
  }
  A.tiles_i = (A.ni + 4 + kStripOut - 1) / kStripOut;
  A.ntiles = A.tiles_i * ((A.nj + 4 + strip_rows<T>() - 1) / strip_rows<T>());
  const dim3 grid((A.ntiles + kStripsPerWG - 1) / kStripsPerWG, A.nk), block(kWG);
  if (var)
    hipLaunchKernelGGL((k_hdiff_adjoint_strip<T, true>), grid, block, 0, s, A);
  else
    hipLaunchKernelGGL((k_hdiff_adjoint_strip<T, false>), grid, block, 0, s, A);
  return hipGetLastError();
}

template hipError_t launch_vadv_adjoint<float>(AdjArgs<float>, int, float*, float*, hipStream_t);
template hipError_t launch_vadv_adjoint<double>(AdjArgs<double>, int, double*, double*, hipStream_t);
template hipError_t launch_hdiff_adjoint<float>(AdjArgs<float>, hipStream_t);
template hipError_t launch_hdiff_adjoint<double>(AdjArgs<double>, hipStream_t);

}  // namespace gt4mi
