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
// Mask lookups; out of the definition sets (or without a mask) -> 0.
template <typename T>
__device__ __forceinline__ bool mask_x(const AdjArgs<T>& A, int k, int qi, int qj) {
  if (!A.mask || qj < 0 || qj >= A.nj || qi < -1 || qi >= A.ni) return false;
  if (qi < 0) return A.mask[A.ml.ex_off + (int64_t)k * A.nj + qj] != 0;
  const uint64_t* w = reinterpret_cast<const uint64_t*>(A.mask + A.ml.x_off);
  return (w[((int64_t)k * A.nj + qj) * A.ml.words + (qi >> 6)] >> (qi & 63)) & 1;
}
template <typename T>
__device__ __forceinline__ bool mask_y(const AdjArgs<T>& A, int k, int qi, int qj) {
  if (!A.mask || qi < 0 || qi >= A.ni || qj < -1 || qj >= A.nj) return false;
  if (qj < 0) return A.mask[A.ml.ey_off + (int64_t)k * A.ni + qi] != 0;
  const uint64_t* w = reinterpret_cast<const uint64_t*>(A.mask + A.ml.y_off);
  return (w[((int64_t)k * A.nj + qj) * A.ml.words + (qi >> 6)] >> (qi & 63)) & 1;
}

// Tile of output points p over the padded domain [-2, ni+2) x [-2, nj+2),
// marched over levels [kbeg, kend).  LDS: lambda on the tile + 2-ring,
// gx, gy, lbar on the tile + 1-ring.
template <typename T, int TI, int TJ>
__global__ void __launch_bounds__(TI* TJ) k_hdiff_adjoint(AdjArgs<T> A, int kper) {
  constexpr int NT = TI * TJ;
  constexpr int HI = TI + 4, HJ = TJ + 4, HN = HI * HJ;      // lambda box: p0-2 .. p0+T+1
  constexpr int GI = TI + 3, GJ = TJ + 2, GN = GI * GJ;      // gx box: i in [p0-2, p0+T], j in [p0-1, p0+T]
  constexpr int YI = TI + 2, YJ = TJ + 3, YN = YI * YJ;      // gy box: i in [p0-1, p0+T], j in [p0-2, p0+T]
  constexpr int LI = TI + 2, LJ = TJ + 2, LN = LI * LJ;      // lbar box: [p0-1, p0+T]^2
  constexpr int NLD = (HN + NT - 1) / NT;
  __shared__ T slam[2][HN];  // double buffered: level k+1 is stored while k is read
  __shared__ T sgx[GN];
  __shared__ T sgy[YN];
  __shared__ T slb[LN];
  const int tid = threadIdx.x, ti = tid % TI, tj = tid / TI;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int bi = tile % A.tiles_i, bj = tile / A.tiles_i;
  const int pi0 = -2 + bi * TI, pj0 = -2 + bj * TJ;  // first output point of the tile
  const int pi = pi0 + ti, pj = pj0 + tj;
  const bool outp = (pi < A.ni + 2) && (pj < A.nj + 2);
  const int kbeg = blockIdx.y * kper, kend = min(kbeg + kper, A.nk);
  const T ncoeff = -A.coeff;

  int64_t hoff[NLD];
  bool hok[NLD];
#pragma unroll
  for (int q = 0; q < NLD; ++q) {
    const int e = tid + q * NT;
    const int hj = e / HI, hi = e - hj * HI;
    const int gi = pi0 - 2 + hi, gj = pj0 - 2 + hj;
    hok[q] = (e < HN) && gi >= 0 && gi < A.ni && gj >= 0 && gj < A.nj;
    hoff[q] = hok[q] ? (int64_t)gi + (int64_t)gj * A.l_sj : 0;
  }
  T pl[NLD];
#pragma unroll
  for (int q = 0; q < NLD; ++q)
    pl[q] = (hok[q] && kbeg < kend) ? A.lam[hoff[q] + (int64_t)kbeg * A.l_sk] : T(0);

  for (int k = kbeg; k < kend; ++k) {
    T* sl = slam[k & 1];
#pragma unroll
    for (int q = 0; q < NLD; ++q)
      if (tid + q * NT < HN) sl[tid + q * NT] = pl[q];
    if (k + 1 < kend) {
#pragma unroll
      for (int q = 0; q < NLD; ++q)
        pl[q] = hok[q] ? A.lam[hoff[q] + (int64_t)(k + 1) * A.l_sk] : T(0);
    }
    __syncthreads();
    // masked flux cotangents
    for (int e = tid; e < GN; e += NT) {
      const int gj = e / GI, gi = e - gj * GI;
      const int qi = pi0 - 2 + gi, qj = pj0 - 1 + gj;
      const int c = (gj + 1) * HI + gi;  // lambda(q) in the lambda box
      sgx[e] = mask_x(A, k, qi, qj) ? ncoeff * (sl[c] - sl[c + 1]) : T(0);
    }
    for (int e = tid; e < YN; e += NT) {
      const int gj = e / YI, gi = e - gj * YI;
      const int qi = pi0 - 1 + gi, qj = pj0 - 2 + gj;
      const int c = gj * HI + gi + 1;
      sgy[e] = mask_y(A, k, qi, qj) ? ncoeff * (sl[c] - sl[c + HI]) : T(0);
    }
    __syncthreads();
    for (int e = tid; e < LN; e += NT) {
      const int lj = e / LI, li = e - lj * LI;
      // q = (pi0 - 1 + li, pj0 - 1 + lj); gx(q) at gx-box (li + 1, lj), gx(q - e_i) at (li, lj)
      const int cx = lj * GI + li;
      const int cy = lj * YI + li;  // gy(q - e_j) at gy-box (li, lj), gy(q) at (li, lj + 1)
      slb[e] = (sgx[cx] - sgx[cx + 1]) + (sgy[cy] - sgy[cy + YI]);
    }
    __syncthreads();
    if (outp) {
      const int c = (tj + 1) * LI + (ti + 1);
      const bool inI = pi >= 0 && pi < A.ni && pj >= 0 && pj < A.nj;
      const T lp = inI ? sl[(tj + 2) * HI + (ti + 2)] : T(0);
      const T v = lp + T(4) * slb[c] - slb[c + 1] - slb[c - 1] - slb[c + LI] - slb[c - LI];
      A.ubar[(int64_t)pi + (int64_t)pj * A.b_sj + (int64_t)k * A.b_sk] = v;
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
