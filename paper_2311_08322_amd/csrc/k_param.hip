// k_param.hip -- gradients of one step with respect to its parameters
// (coeff and the vertical velocity w), for parameter tuning.
//
// With the limiter decisions held fixed the diffusion is h = u - coeff D(u),
// D the divergence of the limited fluxes (independent of coeff), and the
// column solve is T(w) x = h + data.  Given lam = T^{-T} x_bar (the step
// adjoint's data_bar) and the step's output x:
//   coeff_bar = -sum_p lam(p) D(u)(p)
//   w_bar_j   = r/4 [lam_j x_{j-1} - lam_{j-1} x_j - s_j (lam_j x_j + lam_{j-1} x_{j-1})]
// for the staggered levels j = 1 .. nk-1 (s_j = sign w_j, 0 at 0), the
// chain rule of dL/dT(k,l) = -lam_k x_l through a_j = -r/4 w_j,
// c_{j-1} = r/4 w_j and the |a|, |c| terms of the diagonal; w_0 and w_nk do
// not enter T and get 0.
#include "k_step.hpp"
#include "launch.hpp"

namespace gt4mi {

// D(u) at the diamond's centre: the flux stage of the diffusion (the same
// limiter and association as the forward kernels), without the update.
// gs is the form's sign (form_sign): the damping form's divergence is gs
// times the stated one taken with the limiter's gradient times gs.
template <typename T>
__device__ __forceinline__ T divergence_of(const Diamond<T>& d, T gs) {
  const T L00 = T(4) * d.u00 - ((d.um1 + d.up1) + (d.vm1 + d.vp1));
  const T Lp0 = T(4) * d.up1 - ((d.u00 + d.up2) + (d.mp + d.pp));
  const T Lm0 = T(4) * d.um1 - ((d.um2 + d.u00) + (d.mm + d.pm));
  const T L0p = T(4) * d.vp1 - ((d.pm + d.pp) + (d.u00 + d.vp2));
  const T L0m = T(4) * d.vm1 - ((d.mm + d.mp) + (d.vm2 + d.u00));
  const T fxr = Lp0 - L00, fxl = L00 - Lm0, fyr = L0p - L00, fyl = L00 - L0m;
  const T Fxr = flux_kept(fxr, gs * (d.up1 - d.u00)) ? fxr : T(0);
  const T Fxl = flux_kept(fxl, gs * (d.u00 - d.um1)) ? fxl : T(0);
  const T Fyr = flux_kept(fyr, gs * (d.vp1 - d.u00)) ? fyr : T(0);
  const T Fyl = flux_kept(fyl, gs * (d.u00 - d.vm1)) ? fyl : T(0);
  return gs * ((Fxr - Fxl) + (Fyr - Fyl));
}

// One workgroup per TI x TJ tile of the interior marches the levels with
// the u-tile (+2 halo) staged in LDS (one barrier per level, the next
// level's loads in flight) and accumulates lam * D(u) in FP64; the tile's
// sum goes to partial[tile] (fixed order: the result does not depend on
// scheduling).  A.data holds lam.
// FIELD: the gradient of a per-point coefficient instead, -lam(p) D(u)(p)
// stored point by point into A.out (partial unused).
template <typename T, int TI, int TJ, bool FIELD>
__global__ void __launch_bounds__(TI* TJ) k_coeff_partial(StepArgs<T> A, double* partial) {
  using TA = TileAddr<T, TI, TJ>;
  constexpr int NT = TA::NT, HI = TA::HI, NLD = TA::NLD;
  __shared__ T su[2][NLD * NT];
  __shared__ double red[NT];
  const int tile = blockIdx.x;
  TA t;
  t.init(tile, A.tiles_i, A.ni, A.nj, A.u_sj);
  const int tid = threadIdx.x;
  constexpr uint32_t S = sizeof(T);
  const LevelView vu = level_view(A.u, A.u_sj, A.u_sk, -2, -2, A.nj + 4);
  const LevelView vl = level_view(A.data, A.d_sj, A.d_sk, 0, 0, A.nj);
  const uint32_t loff = ((uint32_t)t.ic + (uint32_t)t.jc * (uint32_t)A.d_sj) * S;
  [[maybe_unused]] const LevelView vo = level_view<T>(A.out, A.o_sj, A.o_sk, 0, 0, A.nj);
  [[maybe_unused]] const uint32_t ooff =
      t.active ? ((uint32_t)t.ic + (uint32_t)t.jc * (uint32_t)A.o_sj) * S : kOffNone;
  const T gs = form_sign<T>(A.form);
  LevelCursor cu_{vu.base, vu.level_bytes, vu.window};
  LevelCursor cl{vl.base, vl.level_bytes, vl.window};
  const int nk = A.nk;
  T nu[NLD], nl;
  auto issue = [&](int k) {
    const auto r = cu_.rsrc();
#pragma unroll
    for (int q = 0; q < NLD; ++q) nu[q] = buf_ld(r, t.hoff[q], T());
    nl = buf_ld(cl.rsrc(), loff, T());
    const bool go = k + 1 < nk;  // hold at the last level: no branch around the loads
    cu_.advance(go);
    cl.advance(go);
  };
  issue(0);
  const int cu = (t.tj + 2) * HI + (t.ti + 2);
  double acc = 0.0;
  for (int k = 0; k < nk; ++k) {
    T* U = su[k & 1];
#pragma unroll
    for (int q = 0; q < NLD; ++q) U[tid + q * NT] = nu[q];
    const T lam = nl;
    issue(k + 1);
    __syncthreads();
    const T div = divergence_of(load_diamond<T, HI>(U + cu), gs);
    if constexpr (FIELD)
      buf_st(vo.at(k), ooff, -(lam * div));
    else
      acc += t.active ? (double)lam * (double)div : 0.0;
  }
  if constexpr (FIELD) return;
  red[tid] = acc;
  __syncthreads();
#pragma unroll
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) partial[tile] = red[0];
}

// coeff_bar = -(sum of the partials), summed in a fixed order by one workgroup.
__global__ void __launch_bounds__(kWG) k_coeff_final(const double* partial, int n, double* coeff_bar) {
  __shared__ double red[kWG];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int p = tid; p < n; p += kWG) s += partial[p];
  red[tid] = s;
  __syncthreads();
#pragma unroll
  for (int h = kWG / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) coeff_bar[0] = n > 0 ? -red[0] : 0.0;
}

// w_bar per column, one lane per column of a 64 x 4 tile, marching the
// staggered levels 0..nk with the level below in registers.
template <typename T>
__global__ void __launch_bounds__(kWG) k_w_grad(WGradArgs<T> A) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int bi = tile % A.tiles_i, bj = tile / A.tiles_i;
  const int i = bi * 64 + (threadIdx.x & 63), j = bj * 4 + (threadIdx.x >> 6);
  const bool active = i < A.ni && j < A.nj;
  const int ic = min(i, A.ni - 1), jc = min(j, A.nj - 1);
  constexpr uint32_t S = sizeof(T);
  const LevelView vw = level_view(A.w, A.w_sj, A.w_sk, 0, 0, A.nj);
  const LevelView vx = level_view(A.x, A.x_sj, A.x_sk, 0, 0, A.nj);
  const LevelView vl = level_view(A.lam, A.l_sj, A.l_sk, 0, 0, A.nj);
  const LevelView vb = level_view<T>(A.wbar, A.b_sj, A.b_sk, 0, 0, A.nj);
  const uint32_t woff = ((uint32_t)ic + (uint32_t)jc * (uint32_t)A.w_sj) * S;
  const uint32_t xoff = ((uint32_t)ic + (uint32_t)jc * (uint32_t)A.x_sj) * S;
  const uint32_t loff = ((uint32_t)ic + (uint32_t)jc * (uint32_t)A.l_sj) * S;
  const uint32_t boff = active ? ((uint32_t)ic + (uint32_t)jc * (uint32_t)A.b_sj) * S : kOffNone;
  const int nk = A.nk;
  // w_0 does not enter T
  buf_st(vb.at(0), boff, T(0));
  if (nk < 1) return;
  T lp = buf_ld(vl.at(0), loff, T()), xp = buf_ld(vx.at(0), xoff, T());
  // the loads of level j run one level ahead (clamped at the last level)
  T ln = buf_ld(vl.at(min(1, nk - 1)), loff, T()), xn = buf_ld(vx.at(min(1, nk - 1)), xoff, T());
  T wn = buf_ld(vw.at(1), woff, T());
  for (int jl = 1; jl < nk; ++jl) {
    const T lj = ln, xj = xn, wj = wn;
    const int nx = min(jl + 1, nk - 1);
    ln = buf_ld(vl.at(nx), loff, T());
    xn = buf_ld(vx.at(nx), xoff, T());
    wn = buf_ld(vw.at(min(jl + 1, nk)), woff, T());
    const T s = wj > T(0) ? T(1) : (wj < T(0) ? T(-1) : T(0));
    const T g = A.q * ((lj * xp - lp * xj) - s * (lj * xj + lp * xp));
    buf_st(vb.at(jl), boff, g);
    lp = lj;
    xp = xj;
  }
  // w_nk does not enter T
  buf_st(vb.at(nk), boff, T(0));
}

// ------------------------------------------------------------------ launchers
template <typename T>
hipError_t launch_param_grads(const StepArgs<T>& Ain, const WGradArgs<T>* W, double* partial,
                              double* coeff_bar, hipStream_t s) {
  StepArgs<T> A = Ain;
  A.tiles_i = (A.ni + 63) / 64;
  A.ntiles = A.tiles_i * ((A.nj + 3) / 4);
  const bool some = A.ni > 0 && A.nj > 0;
  if (coeff_bar) {
    if (some && A.nk > 0)
      hipLaunchKernelGGL((k_coeff_partial<T, 64, 4, false>), dim3(A.ntiles), dim3(kWG), 0, s, A, partial);
    const int n = (some && A.nk > 0) ? A.ntiles : 0;
    hipLaunchKernelGGL(k_coeff_final, dim3(1), dim3(kWG), 0, s, partial, n, coeff_bar);
  }
  if (W && some) {
    WGradArgs<T> B = *W;
    B.tiles_i = (B.ni + 63) / 64;
    const int nt = B.tiles_i * ((B.nj + 3) / 4);
    hipLaunchKernelGGL(k_w_grad<T>, dim3(nt), dim3(kWG), 0, s, B);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coeff_field_grad(const StepArgs<T>& Ain, hipStream_t s) {
  StepArgs<T> A = Ain;
  A.tiles_i = (A.ni + 63) / 64;
  A.ntiles = A.tiles_i * ((A.nj + 3) / 4);
  if (A.ni > 0 && A.nj > 0 && A.nk > 0)
    hipLaunchKernelGGL((k_coeff_partial<T, 64, 4, true>), dim3(A.ntiles), dim3(kWG), 0, s, A, nullptr);
  return hipGetLastError();
}

template hipError_t launch_coeff_field_grad<float>(const StepArgs<float>&, hipStream_t);
template hipError_t launch_coeff_field_grad<double>(const StepArgs<double>&, hipStream_t);
template hipError_t launch_param_grads<float>(const StepArgs<float>&, const WGradArgs<float>*, double*, double*,
                                              hipStream_t);
template hipError_t launch_param_grads<double>(const StepArgs<double>&, const WGradArgs<double>*, double*, double*,
                                               hipStream_t);

}  // namespace gt4mi
