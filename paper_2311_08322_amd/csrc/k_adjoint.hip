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
__device__ __forceinline__ uint64_t buf_ld_u64(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ uint32_t buf_ld_u8(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0);
}

// Tile of output points p over the padded domain [-2, ni+2) x [-2, nj+2),
// marched over levels [kbeg, kend).  LDS: lambda on the tile + 2-ring
// (double buffered), the masked flux cotangents gx, gy and lbar on the tile
// + 1-ring.  Three barriers per level; the next level's lambda tile and
// mask words are loaded while the current one is computed.  Every LDS box
// is padded to a multiple of the workgroup so all lanes work unpredicated;
// lanes past a box compute values nobody reads.  Points outside the
// interior read lambda = 0 and flux points outside their definition sets
// read mask 0, both through out-of-window buffer offsets.
template <typename T, int TI, int TJ>
__global__ void __launch_bounds__(TI* TJ) k_hdiff_adjoint(AdjArgs<T> A, int kper) {
  constexpr int NT = TI * TJ;
  constexpr int HI = TI + 4, HN = HI * (TJ + 4), NLD = (HN + NT - 1) / NT;  // lambda box
  constexpr int GI = TI + 3, GN = GI * (TJ + 2), NGX = (GN + NT - 1) / NT;  // gx: i in [p0-2, p0+T], j in [p0-1, p0+T]
  constexpr int YI = TI + 2, YN = YI * (TJ + 3), NGY = (YN + NT - 1) / NT;  // gy: i in [p0-1, p0+T], j in [p0-2, p0+T]
  constexpr int LI = TI + 2, LN = LI * (TJ + 2), NLB = (LN + NT - 1) / NT;  // lbar: [p0-1, p0+T]^2
  constexpr uint32_t S = sizeof(T);
  __shared__ T slam[2][NLD * NT];
  __shared__ T sgx[NGX * NT];
  __shared__ T sgy[NGY * NT];
  __shared__ T slb[NLB * NT];
  const int tid = threadIdx.x, ti = tid % TI, tj = tid / TI;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int bi = tile % A.tiles_i, bj = tile / A.tiles_i;
  const int pi0 = -2 + bi * TI, pj0 = -2 + bj * TJ;  // first output point of the tile
  const int pi = pi0 + ti, pj = pj0 + tj;
  const int ni = A.ni, nj = A.nj;
  const int kbeg = blockIdx.y * kper, kend = min(kbeg + kper, A.nk);
  const T ncoeff = -A.coeff;
  const bool edge_x = (bi == 0), edge_y = (bj == 0);  // tile-uniform: the gx/gy boxes reach i/j = -1
  auto in_I = [&](int a, int b) { return a >= 0 && a < ni && b >= 0 && b < nj; };

  // level-invariant lane offsets
  uint32_t loff[NLD];
#pragma unroll
  for (int q = 0; q < NLD; ++q) {
    const int e = min(tid + q * NT, HN - 1);
    const int hj = e / HI, hi = e - hj * HI;
    const int gi = pi0 - 2 + hi, gj = pj0 - 2 + hj;
    loff[q] = in_I(gi, gj) ? ((uint32_t)gi + (uint32_t)gj * (uint32_t)A.l_sj) * S : kOffNone;
  }
  const int64_t W = A.ml.words;
  uint32_t xw_off[NGX], xe_off[NGX], yw_off[NGY], ye_off[NGY];
  int xbit[NGX], ybit[NGY];
#pragma unroll
  for (int q = 0; q < NGX; ++q) {
    const int e = min(tid + q * NT, GN - 1);
    const int gj = e / GI, gi = e - gj * GI;
    const int qi = pi0 - 2 + gi, qj = pj0 - 1 + gj;
    const bool row = A.mask && qj >= 0 && qj < nj;
    xw_off[q] = (row && qi >= 0 && qi < ni) ? (uint32_t)((qj * W + (qi >> 6)) * 8) : kOffNone;
    xe_off[q] = (row && qi == -1) ? (uint32_t)qj : kOffNone;
    xbit[q] = qi & 63;
  }
#pragma unroll
  for (int q = 0; q < NGY; ++q) {
    const int e = min(tid + q * NT, YN - 1);
    const int gj = e / YI, gi = e - gj * YI;
    const int qi = pi0 - 1 + gi, qj = pj0 - 2 + gj;
    const bool col = A.mask && qi >= 0 && qi < ni;
    yw_off[q] = (col && qj >= 0 && qj < nj) ? (uint32_t)((qj * W + (qi >> 6)) * 8) : kOffNone;
    ye_off[q] = (col && qj == -1) ? (uint32_t)qi : kOffNone;
    ybit[q] = qi & 63;
  }
  const bool outp = (pi < ni + 2) && (pj < nj + 2);
  const uint32_t uoff = outp ? ((uint32_t)(pi + 2) + (uint32_t)(pj + 2) * (uint32_t)A.b_sj) * S : kOffNone;

  const LevelView vl = level_view<T>(A.lam, A.l_sj, A.l_sk, 0, 0, nj);
  const LevelView vb = level_view<T>(A.ubar, A.b_sj, A.b_sk, -2, -2, nj + 4);
  const char* mbase = reinterpret_cast<const char*>(A.mask);
  const int64_t plane_xy = (int64_t)nj * W * 8;
  const uint32_t win_xy = (uint32_t)plane_xy;
  auto mrsrc = [&](int64_t off, int k, int64_t plane, uint32_t win) {
    return make_rsrc(mbase + off + (int64_t)k * plane, win);
  };

  T pl[NLD];
  uint64_t pxw[NGX], pyw[NGY];
  uint32_t pxe[NGX], pye[NGY];
  auto issue = [&](int k) {
    const auto rl = vl.at(k);
#pragma unroll
    for (int q = 0; q < NLD; ++q) pl[q] = buf_ld(rl, loff[q], T());
    const auto rx = mrsrc(A.ml.x_off, k, plane_xy, win_xy);
    const auto ry = mrsrc(A.ml.y_off, k, plane_xy, win_xy);
#pragma unroll
    for (int q = 0; q < NGX; ++q) pxw[q] = buf_ld_u64(rx, xw_off[q]);
#pragma unroll
    for (int q = 0; q < NGY; ++q) pyw[q] = buf_ld_u64(ry, yw_off[q]);
    if (edge_x) {
      const auto re = mrsrc(A.ml.ex_off, k, nj, (uint32_t)nj);
#pragma unroll
      for (int q = 0; q < NGX; ++q) pxe[q] = buf_ld_u8(re, xe_off[q]);
    }
    if (edge_y) {
      const auto re = mrsrc(A.ml.ey_off, k, ni, (uint32_t)ni);
#pragma unroll
      for (int q = 0; q < NGY; ++q) pye[q] = buf_ld_u8(re, ye_off[q]);
    }
  };
#pragma unroll
  for (int q = 0; q < NGX; ++q) pxe[q] = 0;
#pragma unroll
  for (int q = 0; q < NGY; ++q) pye[q] = 0;
  if (kbeg < kend) issue(kbeg);

  for (int k = kbeg; k < kend; ++k) {
    T* sl = slam[k & 1];
#pragma unroll
    for (int q = 0; q < NLD; ++q) sl[tid + q * NT] = pl[q];
    bool kx[NGX], ky[NGY];
#pragma unroll
    for (int q = 0; q < NGX; ++q) kx[q] = ((pxw[q] >> xbit[q]) & 1) | pxe[q];
#pragma unroll
    for (int q = 0; q < NGY; ++q) ky[q] = ((pyw[q] >> ybit[q]) & 1) | pye[q];
    if (k + 1 < kend) issue(k + 1);
    __syncthreads();
    // masked flux cotangents
#pragma unroll
    for (int q = 0; q < NGX; ++q) {
      const int e = min(tid + q * NT, GN - 1);
      const int gj = e / GI, gi = e - gj * GI;
      const int c = (gj + 1) * HI + gi;  // lambda(q) in the lambda box
      sgx[tid + q * NT] = kx[q] ? ncoeff * (sl[c] - sl[c + 1]) : T(0);
    }
#pragma unroll
    for (int q = 0; q < NGY; ++q) {
      const int e = min(tid + q * NT, YN - 1);
      const int gj = e / YI, gi = e - gj * YI;
      const int c = gj * HI + gi + 1;
      sgy[tid + q * NT] = ky[q] ? ncoeff * (sl[c] - sl[c + HI]) : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NLB; ++q) {
      const int e = min(tid + q * NT, LN - 1);
      const int lj = e / LI, li = e - lj * LI;
      // q = (pi0 - 1 + li, pj0 - 1 + lj): gx(q - e_i) at gx-box (li, lj), gx(q) at (li + 1, lj);
      // gy(q - e_j) at gy-box (li, lj), gy(q) at (li, lj + 1)
      const int cx = lj * GI + li;
      const int cy = lj * YI + li;
      slb[tid + q * NT] = (sgx[cx] - sgx[cx + 1]) + (sgy[cy] - sgy[cy + YI]);
    }
    __syncthreads();
    {
      const int c = (tj + 1) * LI + (ti + 1);
      const T lp = sl[(tj + 2) * HI + (ti + 2)];  // 0 outside the interior
      const T v = lp + T(4) * slb[c] - slb[c + 1] - slb[c - 1] - slb[c + LI] - slb[c - LI];
      buf_st(vb.at(k), uoff, v);
    }
  }
}

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

template <typename T>
hipError_t launch_hdiff_adjoint(AdjArgs<T> A, int tile_i, hipStream_t s) {
  const int tile_j = kWG / tile_i;
  A.tiles_i = (A.ni + 4 + tile_i - 1) / tile_i;
  A.ntiles = A.tiles_i * ((A.nj + 4 + tile_j - 1) / tile_j);
  int kper = A.nk;
  while (kper > 4 && (int64_t)A.ntiles * ((A.nk + kper - 1) / kper) < 4096) kper = (kper + 1) / 2;
  dim3 grid(A.ntiles, (A.nk + kper - 1) / kper), block(kWG);
  if (tile_i == 64)
    hipLaunchKernelGGL((k_hdiff_adjoint<T, 64, 4>), grid, block, 0, s, A, kper);
  else if (tile_i == 32)
    hipLaunchKernelGGL((k_hdiff_adjoint<T, 32, 8>), grid, block, 0, s, A, kper);
  else
    hipLaunchKernelGGL((k_hdiff_adjoint<T, 16, 16>), grid, block, 0, s, A, kper);
  return hipGetLastError();
}

template hipError_t launch_vadv_adjoint<float>(AdjArgs<float>, int, float*, float*, hipStream_t);
template hipError_t launch_vadv_adjoint<double>(AdjArgs<double>, int, double*, double*, hipStream_t);
template hipError_t launch_hdiff_adjoint<float>(AdjArgs<float>, int, hipStream_t);
template hipError_t launch_hdiff_adjoint<double>(AdjArgs<double>, int, hipStream_t);

}  // namespace gt4mi
