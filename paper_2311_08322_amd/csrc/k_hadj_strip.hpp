// k_hadj_strip.hpp -- the horizontal diffusion's adjoint (transposed gather).
//
// With the forward limiter decisions held fixed:
//   gx(q)    = Mx(q) * (-coeff) * (mu(q) - mu(q + e_i))
//   gy(q)    = My(q) * (-coeff) * (mu(q) - mu(q + e_j))
//   lbar(q)  = gx(q - e_i) - gx(q) + gy(q - e_j) - gy(q)
//   ubar(p)  = [p in I] lambda(p) + 4 lbar(p) - lbar(p +- e_i) - lbar(p +- e_j)
// with mu = lambda (or kappa * lambda for a per-point coefficient), zero
// outside the interior, and fluxes outside their definition sets zero.
//
// One wavefront owns a strip of 64 consecutive i (lane = i) and walks TJ
// output rows in j at one level.  Neighbours in i come from the lanes next
// door through DPP wave shifts (one register move per 32 bits); neighbours
// in j are the rows before, held in registers as the walk advances.  No
// LDS and no barriers: every wave runs on its own.  Each shift costs the
// strip one lane at its edges, so of the 64 lanes the 60 in the middle
// (lanes 2..61) write ubar; strips overlap by 4 columns.  A row of fluxes
// needs the row after it, so the walk reads rows j0-2 .. j0+TJ+1 for the
// outputs j0 .. j0+TJ-1, PD rows ahead of their use.  Strips cover the
// padded domain [-2, ni+2) x [-2, nj+2); points outside the interior read
// lambda = 0 and flux points outside their definition sets read mask 0.
#pragma once

#include "common.hpp"

namespace gt4mi {

// The strip `t` (of A.tiles_i strips in i times the row blocks in j) at level k.
template <typename T, int TJ, int PD, bool VAR>
__device__ __forceinline__ void hdiff_adjoint_strip(const AdjArgs<T>& A, int t, int k) {
  static_assert((TJ + 4) % PD == 0, "the row walk is unrolled by the prefetch depth");
  constexpr uint32_t S = sizeof(T);
  const int lane = threadIdx.x & 63;
  const int si = t % A.tiles_i, sj = t / A.tiles_i;
  const int ni = A.ni, nj = A.nj;
  const int i = -4 + kStripOut * si + lane;  // lane 2 is the strip's first output column
  const int j0 = -2 + TJ * sj;              // first output row
  const bool iI = i >= 0 && i < ni;
  const bool has_mask = A.mask != nullptr;
  const bool outc = lane >= 2 && lane < 2 + kStripOut && i < ni + 2;
  const T ncoeff = -A.coeff;

  // Every access goes through a descriptor of one row (uniform: its base
  // and a window of the row's width, 0 for a row outside the field) and a
  // lane offset fixed for the whole walk; the window's range check drops
  // the lanes past the row's end.
  const char* lbase = reinterpret_cast<const char*>(A.lam) + (int64_t)k * A.l_sk * S;
  [[maybe_unused]] const char* kbase = reinterpret_cast<const char*>(VAR ? A.kappa : A.lam) + (int64_t)k * A.c_sk * S;
  const char* bbase = reinterpret_cast<const char*>(A.ubar) + ((int64_t)k * A.b_sk - 2 - 2 * A.b_sj) * S;
  const char* mbase = reinterpret_cast<const char*>(A.mask);
  const int64_t W = A.ml.words, plane_xy = (int64_t)nj * W * 8;
  const char* xbase = mbase + A.ml.x_off + (int64_t)k * plane_xy;
  const char* ybase = mbase + A.ml.y_off + (int64_t)k * plane_xy;
  const auto row_rsrc = [&](const char* base, int64_t row_bytes, int r, int rows, uint32_t width) {
    const bool in = r >= 0 && r < rows;
    return make_rsrc(base + (in ? (int64_t)r * row_bytes : 0), in ? width : 0u);
  };
  const uint32_t l_off = i >= 0 ? (uint32_t)i * S : kOffNone;  // lambda, kappa (window: ni)
  // the 32-bit half of the row's mask word that holds bit i
  const uint32_t m_off = (iI && has_mask) ? (uint32_t)((i >> 6) * 8 + ((i >> 5) & 1) * 4) : kOffNone;
  const int mbit = i & 31;
  const uint32_t b_off = outc ? (uint32_t)(i + 2) * S : kOffNone;  // ubar (window: ni + 4)
  const bool edge_i = si == 0;  // the strip holds i = -1, the x fluxes' extra column
  const auto rex = make_rsrc(mbase + A.ml.ex_off + (int64_t)k * nj, has_mask ? (uint32_t)nj : 0u);
  const auto rey = make_rsrc(mbase + A.ml.ey_off + (int64_t)k * ni, has_mask ? (uint32_t)ni : 0u);

  // the edge fluxes' masks, read once per strip: Mx(-1, r) for the rows of
  // the walk (lane l holds row r0 + l + 64 e; read back with readlane), and
  // My(i, -1) for the strip's columns
  const int r0 = j0 - 2;
  constexpr int NR = TJ + 4, NEX = (NR + 63) / 64;
  uint32_t exv[NEX];
#pragma unroll
  for (int e = 0; e < NEX; ++e) {
    const int r = r0 + lane + 64 * e;
    exv[e] = edge_i ? buf_ld_u8(rex, (r >= 0 && r < nj) ? (uint32_t)r : kOffNone) : 0u;
  }
  const bool edge_j = r0 <= -1;
  const uint32_t eyv = edge_j ? buf_ld_u8(rey, iI ? (uint32_t)i : kOffNone) : 0u;

  // the ring of rows in flight: raw loads, consumed PD rows later
  T pl[PD];
  [[maybe_unused]] T pk[VAR ? PD : 1];
  uint32_t pmx[PD], pmy[PD];
  auto issue = [&](int r, int s) {
    pl[s] = buf_ld(row_rsrc(lbase, A.l_sj * S, r, nj, (uint32_t)ni * S), l_off, T());
    if constexpr (VAR) pk[s] = buf_ld(row_rsrc(kbase, A.c_sj * S, r, nj, (uint32_t)ni * S), l_off, T());
    pmx[s] = buf_ld_u32(row_rsrc(xbase, W * 8, r, nj, (uint32_t)(W * 8)), m_off);
    pmy[s] = buf_ld_u32(row_rsrc(ybase, W * 8, r, nj, (uint32_t)(W * 8)), m_off);
  };

  // the walk's state: row r-1 (mu, lambda, gx, the My bit), r-2 (lambda,
  // gy, lbar) and r-3 (lbar)
  T mu1 = T(0), lam1 = T(0), lam2 = T(0), gx1 = T(0), gy2 = T(0), lb2 = T(0), lb3 = T(0);
  bool my1 = false;
  // row n of the walk (r = r0 + n) from ring slot s; refill the slot with row n + PD
  auto step = [&](int n, int s, bool refill) {
    const int r = r0 + n;
    T lam = pl[s];
    // a copy of its own: the slot's register is free for the refill while
    // lambda lives on in the walk's state
    asm volatile("" : "+v"(lam));
    T mu = lam;
    if constexpr (VAR) mu = pk[s] * lam;
    const uint32_t ex = (uint32_t)__builtin_amdgcn_readlane((int)exv[NEX == 1 ? 0 : n / 64], n % 64);
    const bool mx = ((pmx[s] >> mbit) & 1) | (i == -1 && ex != 0u);  // Mx(r)
    const bool my = ((pmy[s] >> mbit) & 1) | (r == -1 && eyv != 0u);  // My(r)
    if (refill) issue(r + PD, s);
    // the shifts run with every lane active (a disabled lane would read as 0)
    const T mu_e = lane_shift<kDppWaveShl1>(mu), gx1_w = lane_shift<kDppWaveShr1>(gx1);
    const T lb2_e = lane_shift<kDppWaveShl1>(lb2), lb2_w = lane_shift<kDppWaveShr1>(lb2);
    const T gx = mx ? ncoeff * (mu - mu_e) : T(0);   // gx(r)
    const T gy1 = my1 ? ncoeff * (mu1 - mu) : T(0);  // gy(r-1)
    const T lb1 = (gx1_w - gx1) + (gy2 - gy1);       // lbar(r-1)
    const int q = r - 2;                             // ubar(r-2)
    const T v = lam2 + T(4) * lb2 - lb2_e - lb2_w - lb1 - lb3;
    if (q >= j0) buf_st(row_rsrc(bbase, A.b_sj * S, q + 2, nj + 4, (uint32_t)(ni + 4) * S), b_off, v);
    lb3 = lb2;
    lb2 = lb1;
    gy2 = gy1;
    gx1 = gx;
    mu1 = mu;
    my1 = my;
    lam2 = lam1;
    lam1 = lam;
  };

#pragma unroll
  for (int s = 0; s < PD; ++s) issue(r0 + s, s);
  int n = 0;
  for (; n < NR - PD; n += PD) {
#pragma unroll
    for (int s = 0; s < PD; ++s) step(n + s, s, true);
  }
#pragma unroll
  for (int s = 0; s < PD; ++s) step(n + s, s, false);
}

// FP32: two adjacent columns per lane (a = i0 + 2l, b = a + 1; i0 even), 128
// columns per wave of which lanes 1..62 write the middle 124.  The east
// neighbour of a and the west neighbour of b are in the lane itself, so a
// row needs half the shifts, and both columns' limiter bits sit in one 32-bit
// word of each mask plane.  Same values as hdiff_adjoint_strip, in the same
// order of operations.  PAIR: ni is even and lambda's rows keep 8-byte
// alignment (the caller checks: lambda_pairs_ok), so a lane reads its two
// columns with one 8-byte load, one request per cache line instead of two.
template <int TJ, int PD, bool VAR, bool PAIR = false>
__device__ __forceinline__ void hdiff_adjoint_strip2(const AdjArgs<float>& A, int t, int k) {
  static_assert((TJ + 4) % PD == 0, "the row walk is unrolled by the prefetch depth");
  using T = float;
  constexpr uint32_t S = 4;
  const int lane = threadIdx.x & 63;
  const int si = t % A.tiles_i, sj = t / A.tiles_i;
  const int ni = A.ni, nj = A.nj;
  const int ia = -4 + kStripOut2 * si + 2 * lane, ib = ia + 1;
  const int j0 = -2 + TJ * sj;
  const bool aI = ia >= 0 && ia < ni, bI = ib >= 0 && ib < ni;
  const bool has_mask = A.mask != nullptr;
  const bool outl = lane >= 1 && lane <= 62;
  const T ncoeff = -A.coeff;

  const auto row_rsrc = [&](const char* base, int64_t row_bytes, int r, int rows, uint32_t width) {
    const bool in = r >= 0 && r < rows;
    return make_rsrc(base + (in ? (int64_t)r * row_bytes : 0), in ? width : 0u);
  };
  const char* lbase = reinterpret_cast<const char*>(A.lam) + (int64_t)k * A.l_sk * S;
  [[maybe_unused]] const char* kbase = reinterpret_cast<const char*>(VAR ? A.kappa : A.lam) + (int64_t)k * A.c_sk * S;
  const char* bbase = reinterpret_cast<const char*>(A.ubar) + ((int64_t)k * A.b_sk - 2 - 2 * A.b_sj) * S;
  const char* mbase = reinterpret_cast<const char*>(A.mask);
  const int64_t W = A.ml.words, plane_xy = (int64_t)nj * W * 8;
  const char* xbase = mbase + A.ml.x_off + (int64_t)k * plane_xy;
  const char* ybase = mbase + A.ml.y_off + (int64_t)k * plane_xy;
  const uint32_t la_off = ia >= 0 ? (uint32_t)ia * S : kOffNone;  // window: ni
  const uint32_t lb_off = ib >= 0 ? (uint32_t)ib * S : kOffNone;
  // PAIR: both columns in one load (ia even and ni even: a inside the row
  // means b inside too; ia < 0 means both outside)
  [[maybe_unused]] const uint32_t lp_off = (ia >= 0 && ia < ni) ? (uint32_t)ia * S : kOffNone;
  // the 32-bit word of a mask row that holds bits a and b (a even)
  const uint32_t m_off = (aI && has_mask) ? (uint32_t)((ia >> 6) * 8 + ((ia >> 5) & 1) * 4) : kOffNone;
  const int mbit = ia & 31;
  const uint32_t ba_off = (outl && ia < ni + 2) ? (uint32_t)(ia + 2) * S : kOffNone;  // window: ni + 4
  const uint32_t bb_off = (outl && ib < ni + 2) ? (uint32_t)(ib + 2) * S : kOffNone;
  const bool edge_i = si == 0;  // lane 1's b column is i = -1, the x fluxes' extra column
  const auto rex = make_rsrc(mbase + A.ml.ex_off + (int64_t)k * nj, has_mask ? (uint32_t)nj : 0u);
  const auto rey = make_rsrc(mbase + A.ml.ey_off + (int64_t)k * ni, has_mask ? (uint32_t)ni : 0u);

  const int r0 = j0 - 2;
  constexpr int NR = TJ + 4, NEX = (NR + 63) / 64;
  uint32_t exv[NEX];
#pragma unroll
  for (int e = 0; e < NEX; ++e) {
    const int r = r0 + lane + 64 * e;
    exv[e] = edge_i ? buf_ld_u8(rex, (r >= 0 && r < nj) ? (uint32_t)r : kOffNone) : 0u;
  }
  const bool edge_j = r0 <= -1;
  const uint32_t eya = edge_j ? buf_ld_u8(rey, aI ? (uint32_t)ia : kOffNone) : 0u;
  const uint32_t eyb = edge_j ? buf_ld_u8(rey, bI ? (uint32_t)ib : kOffNone) : 0u;

  T pla[PD], plb[PD];
  [[maybe_unused]] T pka[VAR ? PD : 1], pkb[VAR ? PD : 1];
  uint32_t pmx[PD], pmy[PD];
  auto issue = [&](int r, int s) {
    const auto rl = row_rsrc(lbase, A.l_sj * S, r, nj, (uint32_t)ni * S);
    if constexpr (PAIR) {
      // the 8 bytes are taken apart as a float vector: element access on the
      // builtin's integer vector narrowed the load to its first word here
      typedef float f32x2_t __attribute__((ext_vector_type(2)));
      const f32x2_t v = __builtin_bit_cast(f32x2_t, __builtin_amdgcn_raw_buffer_load_b64(rl, lp_off, 0, 0));
      pla[s] = v[0];
      plb[s] = v[1];
    } else {
      pla[s] = buf_ld(rl, la_off, T());
      plb[s] = buf_ld(rl, lb_off, T());
    }
    if constexpr (VAR) {
      const auto rk = row_rsrc(kbase, A.c_sj * S, r, nj, (uint32_t)ni * S);
      pka[s] = buf_ld(rk, la_off, T());
      pkb[s] = buf_ld(rk, lb_off, T());
    }
    pmx[s] = buf_ld_u32(row_rsrc(xbase, W * 8, r, nj, (uint32_t)(W * 8)), m_off);
    pmy[s] = buf_ld_u32(row_rsrc(ybase, W * 8, r, nj, (uint32_t)(W * 8)), m_off);
  };

  T mu1a = 0, mu1b = 0, lam1a = 0, lam1b = 0, lam2a = 0, lam2b = 0, gx1a = 0, gx1b = 0;
  T gy2a = 0, gy2b = 0, lb2a = 0, lb2b = 0, lb3a = 0, lb3b = 0;
  bool my1a = false, my1b = false;
  auto step = [&](int n, int s, bool refill) {
    const int r = r0 + n;
    T lama = pla[s], lamb = plb[s];
    asm volatile("" : "+v"(lama), "+v"(lamb));  // copies of their own: the slots are free for the refill
    T mua = lama, mub = lamb;
    if constexpr (VAR) {
      mua = pka[s] * lama;
      mub = pkb[s] * lamb;
    }
    const uint32_t ex = (uint32_t)__builtin_amdgcn_readlane((int)exv[NEX == 1 ? 0 : n / 64], n % 64);
    const uint32_t wx = pmx[s] >> mbit, wy = pmy[s] >> mbit;
    // bit b of a column past ni reads as 0: the word is read only where a < ni
    const bool mxa = (wx & 1) != 0, mxb = (bI && ((wx >> 1) & 1)) || (ib == -1 && ex != 0u);
    const bool mya = ((wy & 1) != 0) || (r == -1 && eya != 0u);
    const bool myb = (bI && ((wy >> 1) & 1)) || (r == -1 && eyb != 0u);
    if (refill) issue(r + PD, s);
    // the shifts run with every lane active (a disabled lane would read as 0)
    const T mua_e = lane_shift<kDppWaveShl1>(mua);    // east of b
    const T gx1b_w = lane_shift<kDppWaveShr1>(gx1b);  // west of a
    const T lb2a_e = lane_shift<kDppWaveShl1>(lb2a);  // east of b
    const T lb2b_w = lane_shift<kDppWaveShr1>(lb2b);  // west of a
    const T gxa = mxa ? ncoeff * (mua - mub) : T(0);  // gx(r)
    const T gxb = mxb ? ncoeff * (mub - mua_e) : T(0);
    const T gy1a = my1a ? ncoeff * (mu1a - mua) : T(0);  // gy(r-1)
    const T gy1b = my1b ? ncoeff * (mu1b - mub) : T(0);
    const T lb1a = (gx1b_w - gx1a) + (gy2a - gy1a);  // lbar(r-1)
    const T lb1b = (gx1a - gx1b) + (gy2b - gy1b);
    const int q = r - 2;  // ubar(r-2)
    const T va = lam2a + T(4) * lb2a - lb2b - lb2b_w - lb1a - lb3a;
    const T vb = lam2b + T(4) * lb2b - lb2a_e - lb2a - lb1b - lb3b;
    if (q >= j0) {
      const auto rb = row_rsrc(bbase, A.b_sj * S, q + 2, nj + 4, (uint32_t)(ni + 4) * S);
      buf_st(rb, ba_off, va);
      buf_st(rb, bb_off, vb);
    }
    lb3a = lb2a; lb3b = lb2b;
    lb2a = lb1a; lb2b = lb1b;
    gy2a = gy1a; gy2b = gy1b;
    gx1a = gxa; gx1b = gxb;
    mu1a = mua; mu1b = mub;
    my1a = mya; my1b = myb;
    lam2a = lam1a; lam2b = lam1b;
    lam1a = lama; lam1b = lamb;
  };

#pragma unroll
  for (int s = 0; s < PD; ++s) issue(r0 + s, s);
  int n = 0;
  for (; n < NR - PD; n += PD) {
#pragma unroll
    for (int s = 0; s < PD; ++s) step(n + s, s, true);
  }
#pragma unroll
  for (int s = 0; s < PD; ++s) step(n + s, s, false);
}

template <bool VAR, bool PAIR>
__global__ void __launch_bounds__(kWG) k_hdiff_adjoint_strip2(AdjArgs<float> A) {
  const int t = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * kStripsPerWG +
                                               (int)(threadIdx.x >> 6));
  if (t >= A.ntiles) return;  // whole waves only: no barrier follows
  hdiff_adjoint_strip2<strip_rows<float>(), strip_pd<float>(), VAR, PAIR>(A, t, blockIdx.y);
}

// One strip per wave, at one level per grid row.
template <typename T, bool VAR>
__global__ void __launch_bounds__(kWG) k_hdiff_adjoint_strip(AdjArgs<T> A) {
  // the wave's strip (uniform: the conditions on it stay scalar branches)
  const int t = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * kStripsPerWG +
                                               (int)(threadIdx.x >> 6));
  if (t >= A.ntiles) return;  // whole waves only: no barrier follows
  hdiff_adjoint_strip<T, strip_rows<T>(), strip_pd<T>(), VAR>(A, t, blockIdx.y);
}

}  // namespace gt4mi
