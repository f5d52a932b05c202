// k_hadj.hpp -- the horizontal diffusion's adjoint (transposed gather).
//
// With the forward limiter decisions held fixed:
//   gx(q)    = Mx(q) * (-coeff) * (lambda(q) - lambda(q + e_i))
//   gy(q)    = My(q) * (-coeff) * (lambda(q) - lambda(q + e_j))
//   lbar(q)  = gx(q - e_i) - gx(q) + gy(q - e_j) - gy(q)
//   ubar(p)  = [p in I] lambda(p) + 4 lbar(p) - lbar(p +- e_i) - lbar(p +- e_j)
// with lambda = 0 outside the interior and fluxes outside their definition
// sets ([-1,ni) x [0,nj) and [0,ni) x [-1,nj)) equal to zero.
#pragma once

#include "common.hpp"

namespace gt4mi {

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
struct HadjShape {
  static constexpr int NT = TI * TJ;
  static constexpr int HI = TI + 4, HN = HI * (TJ + 4), NLD = (HN + NT - 1) / NT;  // lambda box
  static constexpr int GI = TI + 3, GN = GI * (TJ + 2), NGX = (GN + NT - 1) / NT;  // gx: i in [p0-2, p0+T], j in [p0-1, p0+T]
  static constexpr int YI = TI + 2, YN = YI * (TJ + 3), NGY = (YN + NT - 1) / NT;  // gy: i in [p0-1, p0+T], j in [p0-2, p0+T]
  static constexpr int LI = TI + 2, LN = LI * (TJ + 2), NLB = (LN + NT - 1) / NT;  // lbar: [p0-1, p0+T]^2
};

template <typename T, int TI, int TJ>
struct HadjSmem {
  using H = HadjShape<T, TI, TJ>;
  T slam[2][H::NLD * H::NT];
  T sgx[H::NGX * H::NT];
  T sgy[H::NGY * H::NT];
  T slb[H::NLB * H::NT];
};

// One output tile `tile` of the padded domain over levels [kbeg, kend).
// VAR: a per-point coefficient kappa (A.kappa, never null then): the box
// holds kappa * lambda, whose differences the flux cotangents take (times
// -A.coeff, the form's sign), and lambda(p) of the identity term is loaded
// on its own.
template <typename T, int TI, int TJ, bool VAR = false>
__device__ __forceinline__ void hdiff_adjoint_tile(const AdjArgs<T>& A, int tile, int kbeg, int kend,
                                                   HadjSmem<T, TI, TJ>& sm) {
  using H = HadjShape<T, TI, TJ>;
  constexpr int NT = H::NT, HI = H::HI, HN = H::HN, NLD = H::NLD, GI = H::GI, GN = H::GN, NGX = H::NGX;
  constexpr int YI = H::YI, YN = H::YN, NGY = H::NGY, LI = H::LI, LN = H::LN, NLB = H::NLB;
  constexpr uint32_t S = sizeof(T);
  auto& slam = sm.slam;
  auto& sgx = sm.sgx;
  auto& sgy = sm.sgy;
  auto& slb = sm.slb;
  const int tid = threadIdx.x, ti = tid % TI, tj = tid / TI;
  const int bi = tile % A.tiles_i, bj = tile / A.tiles_i;
  const int pi0 = -2 + bi * TI, pj0 = -2 + bj * TJ;  // first output point of the tile
  const int pi = pi0 + ti, pj = pj0 + tj;
  const int ni = A.ni, nj = A.nj;
  const T ncoeff = -A.coeff;
  const bool edge_x = (bi == 0), edge_y = (bj == 0);  // tile-uniform: the gx/gy boxes reach i/j = -1
  auto in_I = [&](int a, int b) { return a >= 0 && a < ni && b >= 0 && b < nj; };

  // level-invariant lane offsets
  uint32_t loff[NLD];
  [[maybe_unused]] uint32_t koff[VAR ? NLD : 1];
#pragma unroll
  for (int q = 0; q < NLD; ++q) {
    const int e = min(tid + q * NT, HN - 1);
    const int hj = e / HI, hi = e - hj * HI;
    const int gi = pi0 - 2 + hi, gj = pj0 - 2 + hj;
    loff[q] = in_I(gi, gj) ? ((uint32_t)gi + (uint32_t)gj * (uint32_t)A.l_sj) * S : kOffNone;
    if constexpr (VAR) koff[q] = in_I(gi, gj) ? ((uint32_t)gi + (uint32_t)gj * (uint32_t)A.c_sj) * S : kOffNone;
  }
  // lambda at the lane's own output point (VAR)
  [[maybe_unused]] const uint32_t coff =
      in_I(pi, pj) ? ((uint32_t)pi + (uint32_t)pj * (uint32_t)A.l_sj) * S : kOffNone;
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
  [[maybe_unused]] const LevelView vk = level_view<T>(VAR ? A.kappa : A.lam, A.c_sj, A.c_sk, 0, 0, nj);
  const LevelView vb = level_view<T>(A.ubar, A.b_sj, A.b_sk, -2, -2, nj + 4);
  const char* mbase = reinterpret_cast<const char*>(A.mask);
  const int64_t plane_xy = (int64_t)nj * W * 8;
  const uint32_t win_xy = (uint32_t)plane_xy;
  auto mrsrc = [&](int64_t off, int k, int64_t plane, uint32_t win) {
    return make_rsrc(mbase + off + (int64_t)k * plane, win);
  };

  T pl[NLD];
  [[maybe_unused]] T pk[VAR ? NLD : 1], plc = T(0);
  uint64_t pxw[NGX], pyw[NGY];
  uint32_t pxe[NGX], pye[NGY];
  auto issue = [&](int k) {
    const auto rl = vl.at(k);
#pragma unroll
    for (int q = 0; q < NLD; ++q) pl[q] = buf_ld(rl, loff[q], T());
    if constexpr (VAR) {
      const auto rk = vk.at(k);
#pragma unroll
      for (int q = 0; q < NLD; ++q) pk[q] = buf_ld(rk, koff[q], T());
      plc = buf_ld(rl, coff, T());
    }
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
    [[maybe_unused]] T lc = T(0);
    if constexpr (VAR) {
#pragma unroll
      for (int q = 0; q < NLD; ++q) sl[tid + q * NT] = pk[q] * pl[q];
      lc = plc;
    } else {
#pragma unroll
      for (int q = 0; q < NLD; ++q) sl[tid + q * NT] = pl[q];
    }
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
      const T lp = VAR ? lc : sl[(tj + 2) * HI + (ti + 2)];  // 0 outside the interior
      const T v = lp + T(4) * slb[c] - slb[c + 1] - slb[c - 1] - slb[c + LI] - slb[c - LI];
      buf_st(vb.at(k), uoff, v);
    }
  }
}

template <typename T, int TI, int TJ, bool VAR>
__global__ void __launch_bounds__(TI* TJ) k_hdiff_adjoint(AdjArgs<T> A, int kper) {
  __shared__ HadjSmem<T, TI, TJ> sm;
  const int kbeg = blockIdx.y * kper;
  hdiff_adjoint_tile<T, TI, TJ, VAR>(A, xcd_tile(blockIdx.x, gridDim.x), kbeg, min(kbeg + kper, A.nk), sm);
}


}  // namespace gt4mi
