// k_hdiff_strip.hpp -- the horizontal diffusion alone (stated form, scalar
// coefficient) as a row walk.
//
// Per level, on the interior:
//   lap(p)  = 4 u(p) - ((u(p - e_i) + u(p + e_i)) + (u(p - e_j) + u(p + e_j)))
//   fx(q)   = lap(q + e_i) - lap(q), kept unless fx * (u(q + e_i) - u(q)) > 0
//   fy(q)   = lap(q + e_j) - lap(q), kept likewise with u(q + e_j) - u(q)
//   out(p)  = u(p) - coeff ((Fx(p) - Fx(p - e_i)) + (Fy(p) - Fy(p - e_j)))
// with the same association as the tile kernel, so values and limiter bits
// are the same bit for bit.
//
// One wavefront owns 64 consecutive i (lane = i) of one level and walks
// 16 + 4 rows in j, one u row loaded per step PD rows ahead; neighbours in i
// come from DPP wave shifts, neighbours in j from the rows already walked.
// Per step it forms lap of the row before the newest, its x fluxes, the y
// fluxes below it, and out of the row two back: every value once.  Lanes
// 4..59 own the strip's 56 output columns, which start on a byte of the
// mask rows, so a strip writes its limiter bits as whole bytes (a wave
// ballot) and strips never share a byte.  No LDS, no barriers.
#pragma once

#include "common.hpp"

namespace gt4mi {

constexpr int kHStripOut = 56;   // output columns per strip: 7 bytes of a mask row
constexpr int kHStripRows = 16;  // output rows per strip
constexpr int kHStripPD = 4;     // u rows in flight ahead of their use

// The strip `t` (A.tiles_i strips in i times the row blocks in j) at level k.
template <typename T, int TJ, int PD>
__device__ __forceinline__ void hdiff_strip(const StepArgs<T>& A, int t, int k) {
  static_assert((TJ + 4) % PD == 0, "the row walk is unrolled by the prefetch depth");
  constexpr uint32_t S = sizeof(T);
  const int lane = threadIdx.x & 63;
  const int si = t % A.tiles_i, sj = t / A.tiles_i;
  const int ni = A.ni, nj = A.nj;
  const int i = kHStripOut * si - 4 + lane;  // lane 4 is the strip's first output column
  const int j0 = TJ * sj;                    // first output row
  const bool own = lane >= 4 && lane < 4 + kHStripOut && i < ni;
  const bool has_mask = A.mask != nullptr;
  const T coeff = A.coeff;

  // One descriptor per row (uniform base, a window of the row's width, empty
  // for a row outside the field) and a lane offset fixed for the walk.
  const auto row_rsrc = [&](const char* base, int64_t row_bytes, int r, int rows, uint32_t width) {
    const bool in = r >= 0 && r < rows;
    return make_rsrc(base + (in ? (int64_t)r * row_bytes : 0), in ? width : 0u);
  };
  const char* ubase = reinterpret_cast<const char*>(A.u) + ((int64_t)k * A.u_sk - 2 - 2 * A.u_sj) * S;
  const char* obase = reinterpret_cast<const char*>(A.out) + (int64_t)k * A.o_sk * S;
  const uint32_t u_off = (i >= -2 && i < ni + 2) ? (uint32_t)(i + 2) * S : kOffNone;  // window: ni + 4
  const uint32_t o_off = own ? (uint32_t)i * S : kOffNone;                            // window: ni
  // The limiter bits: one descriptor over the whole mask (the host sends
  // masks below 4 GiB here), so one byte store writes a row's x bytes
  // (lanes 0..6) and y bytes (lanes 8..14) together.
  const auto rm = make_rsrc(A.mask, has_mask ? (uint32_t)A.ml.total : 0u);
  const int64_t W = A.ml.words, plane_xy = (int64_t)nj * W * 8;
  const int64_t x_lev = A.ml.x_off + (int64_t)k * plane_xy, y_lev = A.ml.y_off + (int64_t)k * plane_xy;
  const int mb = lane & 7;                                  // the lane's byte of the strip's 7
  const bool xlane = lane < 7, ylane = lane >= 8 && lane < 15;
  const uint32_t mcol = (uint32_t)(kHStripOut / 8 * si + mb);  // byte within a mask row
  const bool mcol_in = mcol < (uint32_t)(W * 8);
  const int byte_shift = 4 + 8 * mb;
  const uint32_t ex_base = (uint32_t)(A.ml.ex_off + (int64_t)k * nj), ey_base = (uint32_t)(A.ml.ey_off + (int64_t)k * ni);

  T pu[PD];
  const int r0 = j0 - 2;
  constexpr int NR = TJ + 4;
  auto issue = [&](int r, int s) { pu[s] = buf_ld(row_rsrc(ubase, A.u_sj * S, r + 2, nj + 4, (uint32_t)(ni + 4) * S), u_off, T()); };

  // the walk's state: u of rows R-1 and R-2, lap of row R-2, the kept x
  // fluxes of row R-2 and the kept y fluxes between rows R-3 and R-2
  T u1 = T(0), u2 = T(0), lap2 = T(0), Fx2 = T(0), Fy3 = T(0);
  auto step = [&](int n, int s, bool refill) {
    const int R = r0 + n;
    T uR = pu[s];
    asm volatile("" : "+v"(uR));  // a copy of its own: the slot is free for the refill
    if (refill) issue(R + PD, s);
    // the shifts run with every lane active (a disabled lane would read as 0)
    const T ue1 = lane_shift<kDppWaveShl1>(u1), uw1 = lane_shift<kDppWaveShr1>(u1);
    const T lap1 = T(4) * u1 - ((uw1 + ue1) + (u2 + uR));  // lap(R-1)
    const T lape1 = lane_shift<kDppWaveShl1>(lap1);
    const T Fxw2 = lane_shift<kDppWaveShr1>(Fx2);
    const T fx = lape1 - lap1;  // x flux of row R-1
    const bool kx = flux_kept(fx, ue1 - u1);
    const T Fx1 = kx ? fx : T(0);
    const T fy = lap1 - lap2;  // y flux between rows R-2 and R-1
    const bool ky = flux_kept(fy, u1 - u2);
    const T Fy2 = ky ? fy : T(0);
    const int q = R - 2;  // out(R-2)
    const T v = u2 - coeff * ((Fx2 - Fxw2) + (Fy2 - Fy3));
    const bool qrow = q >= j0 && q < j0 + TJ;  // uniform
    if (qrow) buf_st(row_rsrc(obase, A.o_sj * S, q, nj, (uint32_t)ni * S), o_off, v);
    if (has_mask) {
      // x bits of row R-1 and y bits between rows R-2 and R-1, one store
      const int rx = R - 1;
      const uint64_t bx = __ballot(own && kx), by = __ballot(own && ky);
      const bool xrow = rx >= j0 && rx < j0 + TJ && rx < nj, yrow = qrow && q < nj;  // uniform
      uint32_t off = kOffNone;
      if (xlane && xrow && mcol_in) off = (uint32_t)(x_lev + (int64_t)rx * W * 8) + mcol;
      if (ylane && yrow && mcol_in) off = (uint32_t)(y_lev + (int64_t)q * W * 8) + mcol;
      buf_st_u8(rm, off, (uint8_t)((ylane ? by : bx) >> byte_shift));
      // the x flux at i = -1 and the y flux below row 0 have byte planes of their own
      if (si == 0 && xrow && rx >= 0) buf_st_u8(rm, i == -1 ? ex_base + (uint32_t)rx : kOffNone, kx ? 1 : 0);
      if (q == -1) buf_st_u8(rm, own ? ey_base + (uint32_t)i : kOffNone, ky ? 1 : 0);
    }
    Fy3 = Fy2;
    Fx2 = Fx1;
    lap2 = lap1;
    u2 = u1;
    u1 = uR;
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

// FP32: two adjacent columns per lane (a = 120 s - 4 + 2 l, b = a + 1), 128
// columns per wave of which lanes 2..61 own the strip's 120 output columns
// (15 bytes of a mask row).  The east neighbour of a and the west neighbour
// of b are in the lane itself, so a row needs half the shifts; the two
// columns' limiter bits come from two ballots, interleaved into the row's
// bytes.  Same values and bits as hdiff_strip.
constexpr int kHStripOut2 = 120;

// bits 0..3 of v to bits 0, 2, 4, 6
__device__ __forceinline__ uint32_t spread4(uint32_t v) {
  return (v & 1u) | ((v & 2u) << 1) | ((v & 4u) << 2) | ((v & 8u) << 3);
}

// PAIR: ni is even and the rows of u (from its padded corner) and out keep
// 8-byte alignment, so a lane reads and writes its two columns with one
// 8-byte access each (one request per cache line instead of two).
template <int TJ, int PD, bool PAIR = false>
__device__ __forceinline__ void hdiff_strip2(const StepArgs<float>& A, int t, int k) {
  static_assert((TJ + 4) % PD == 0, "the row walk is unrolled by the prefetch depth");
  using T = float;
  constexpr uint32_t S = 4;
  const int lane = threadIdx.x & 63;
  const int si = t % A.tiles_i, sj = t / A.tiles_i;
  const int ni = A.ni, nj = A.nj;
  const int ia = kHStripOut2 * si - 4 + 2 * lane, ib = ia + 1;  // lane 2's a is the first output column
  const int j0 = TJ * sj;
  const bool owna = lane >= 2 && lane < 2 + kHStripOut2 / 2 && ia < ni;
  const bool ownb = lane >= 2 && lane < 2 + kHStripOut2 / 2 && ib < ni;
  const bool has_mask = A.mask != nullptr;
  const T coeff = A.coeff;

  const auto row_rsrc = [&](const char* base, int64_t row_bytes, int r, int rows, uint32_t width) {
    const bool in = r >= 0 && r < rows;
    return make_rsrc(base + (in ? (int64_t)r * row_bytes : 0), in ? width : 0u);
  };
  const char* ubase = reinterpret_cast<const char*>(A.u) + ((int64_t)k * A.u_sk - 2 - 2 * A.u_sj) * S;
  const char* obase = reinterpret_cast<const char*>(A.out) + (int64_t)k * A.o_sk * S;
  const uint32_t ua_off = (ia >= -2 && ia < ni + 2) ? (uint32_t)(ia + 2) * S : kOffNone;  // window: ni + 4
  const uint32_t ub_off = (ib >= -2 && ib < ni + 2) ? (uint32_t)(ib + 2) * S : kOffNone;
  const uint32_t oa_off = owna ? (uint32_t)ia * S : kOffNone;  // window: ni
  const uint32_t ob_off = ownb ? (uint32_t)ib * S : kOffNone;
  // PAIR (ni even, ia even): a inside its window means b inside too
  typedef float f32x2_t __attribute__((ext_vector_type(2)));
  [[maybe_unused]] const uint32_t up_off = ua_off;
  [[maybe_unused]] const uint32_t op_off = oa_off;
  // limiter bytes: one descriptor over the whole mask (below 4 GiB), lanes
  // 0..14 the x bytes of a row, lanes 16..30 its y bytes
  const auto rm = make_rsrc(A.mask, has_mask ? (uint32_t)A.ml.total : 0u);
  const int64_t W = A.ml.words, plane_xy = (int64_t)nj * W * 8;
  const int64_t x_lev = A.ml.x_off + (int64_t)k * plane_xy, y_lev = A.ml.y_off + (int64_t)k * plane_xy;
  const int mb = lane & 15;  // the lane's byte of the strip's 15
  const bool xlane = lane < 15, ylane = lane >= 16 && lane < 31;
  const uint32_t mcol = (uint32_t)(kHStripOut2 / 8 * si + mb);
  const bool mcol_in = mcol < (uint32_t)(W * 8);
  const int bshift = 2 + 4 * mb;  // byte mb holds columns 8 mb .. 8 mb + 7: lanes 2 + 4 mb .. 5 + 4 mb
  const uint32_t ex_base = (uint32_t)(A.ml.ex_off + (int64_t)k * nj), ey_base = (uint32_t)(A.ml.ey_off + (int64_t)k * ni);

  T pa[PD], pb[PD];
  const int r0 = j0 - 2;
  constexpr int NR = TJ + 4;
  auto issue = [&](int r, int s) {
    const auto ru = row_rsrc(ubase, A.u_sj * S, r + 2, nj + 4, (uint32_t)(ni + 4) * S);
    if constexpr (PAIR) {
      // taken apart as a float vector: element access on the builtin's
      // integer vector narrowed the load to its first word
      const f32x2_t v = __builtin_bit_cast(f32x2_t, __builtin_amdgcn_raw_buffer_load_b64(ru, up_off, 0, 0));
      pa[s] = v[0];
      pb[s] = v[1];
    } else {
      pa[s] = buf_ld(ru, ua_off, T());
      pb[s] = buf_ld(ru, ub_off, T());
    }
  };

  T u1a = 0, u1b = 0, u2a = 0, u2b = 0, lap2a = 0, lap2b = 0, Fx2a = 0, Fx2b = 0, Fy3a = 0, Fy3b = 0;
  auto step = [&](int n, int s, bool refill) {
    const int R = r0 + n;
    T uRa = pa[s], uRb = pb[s];
    asm volatile("" : "+v"(uRa), "+v"(uRb));  // copies of their own: the slots are free for the refill
    if (refill) issue(R + PD, s);
    // the shifts run with every lane active (a disabled lane would read as 0)
    const T u1a_e = lane_shift<kDppWaveShl1>(u1a);  // east of b
    const T u1b_w = lane_shift<kDppWaveShr1>(u1b);  // west of a
    const T lap1a = T(4) * u1a - ((u1b_w + u1b) + (u2a + uRa));  // lap(R-1)
    const T lap1b = T(4) * u1b - ((u1a + u1a_e) + (u2b + uRb));
    const T lap1a_e = lane_shift<kDppWaveShl1>(lap1a);
    const T Fx2b_w = lane_shift<kDppWaveShr1>(Fx2b);
    const T fxa = lap1b - lap1a, fxb = lap1a_e - lap1b;  // x fluxes of row R-1
    const bool kxa = flux_kept(fxa, u1b - u1a), kxb = flux_kept(fxb, u1a_e - u1b);
    const T Fx1a = kxa ? fxa : T(0), Fx1b = kxb ? fxb : T(0);
    const T fya = lap1a - lap2a, fyb = lap1b - lap2b;  // y fluxes between rows R-2 and R-1
    const bool kya = flux_kept(fya, u1a - u2a), kyb = flux_kept(fyb, u1b - u2b);
    const T Fy2a = kya ? fya : T(0), Fy2b = kyb ? fyb : T(0);
    const int q = R - 2;  // out(R-2)
    const T va = u2a - coeff * ((Fx2a - Fx2b_w) + (Fy2a - Fy3a));
    const T vb = u2b - coeff * ((Fx2b - Fx2a) + (Fy2b - Fy3b));
    const bool qrow = q >= j0 && q < j0 + TJ;  // uniform
    if (qrow) {
      const auto ro = row_rsrc(obase, A.o_sj * S, q, nj, (uint32_t)ni * S);
      if constexpr (PAIR) {
        const f32x2_t v = {va, vb};
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), ro, op_off, 0, 0);
      } else {
        buf_st(ro, oa_off, va);
        buf_st(ro, ob_off, vb);
      }
    }
    if (has_mask) {
      const int rx = R - 1;
      const uint64_t bxa = __ballot(owna && kxa), bxb = __ballot(ownb && kxb);
      const uint64_t bya = __ballot(owna && kya), byb = __ballot(ownb && kyb);
      const bool xrow = rx >= j0 && rx < j0 + TJ && rx < nj, yrow = qrow && q < nj;  // uniform
      const uint64_t ba = ylane ? bya : bxa, bb = ylane ? byb : bxb;
      const uint8_t byte = (uint8_t)(spread4((uint32_t)(ba >> bshift) & 15u) | (spread4((uint32_t)(bb >> bshift) & 15u) << 1));
      uint32_t off = kOffNone;
      if (xlane && xrow && mcol_in) off = (uint32_t)(x_lev + (int64_t)rx * W * 8) + mcol;
      if (ylane && yrow && mcol_in) off = (uint32_t)(y_lev + (int64_t)q * W * 8) + mcol;
      buf_st_u8(rm, off, byte);
      // the x flux at i = -1 (column b of lane 1 in the first strip) and the
      // y flux below row 0 have byte planes of their own
      if (si == 0 && xrow && rx >= 0) buf_st_u8(rm, ib == -1 ? ex_base + (uint32_t)rx : kOffNone, kxb ? 1 : 0);
      if (q == -1) {
        buf_st_u8(rm, owna ? ey_base + (uint32_t)ia : kOffNone, kya ? 1 : 0);
        buf_st_u8(rm, ownb ? ey_base + (uint32_t)ib : kOffNone, kyb ? 1 : 0);
      }
    }
    Fy3a = Fy2a; Fy3b = Fy2b;
    Fx2a = Fx1a; Fx2b = Fx1b;
    lap2a = lap1a; lap2b = lap1b;
    u2a = u1a; u2b = u1b;
    u1a = uRa; u1b = uRb;
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

template <bool PAIR>
__global__ void __launch_bounds__(kWG) k_hdiff_strip2(StepArgs<float> A) {
  const int t = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * kStripsPerWG +
                                               (int)(threadIdx.x >> 6));
  if (t >= A.ntiles) return;  // whole waves only: no barrier follows
  hdiff_strip2<kHStripRows, kHStripPD, PAIR>(A, t, blockIdx.y);
}

// ni is even and the rows of u (from its padded corner) and out keep 8-byte
// alignment: the binary32 row walk then reads and writes column pairs
inline bool hdiff_pairs_ok(const StepArgs<float>& A) {
  const auto al = [](const void* p, int64_t sj, int64_t sk) {
    return reinterpret_cast<uintptr_t>(p) % 8 == 0 && (sj * 4) % 8 == 0 && (sk * 4) % 8 == 0;
  };
  return A.ni % 2 == 0 && al(A.u - 2 - 2 * A.u_sj, A.u_sj, A.u_sk) && al(A.out, A.o_sj, A.o_sk);
}

// One strip per wave, at one level per grid row.
template <typename T>
__global__ void __launch_bounds__(kWG) k_hdiff_strip(StepArgs<T> A) {
  // the wave's strip (uniform: the conditions on it stay scalar branches)
  const int t = __builtin_amdgcn_readfirstlane(xcd_tile(blockIdx.x, gridDim.x) * kStripsPerWG +
                                               (int)(threadIdx.x >> 6));
  if (t >= A.ntiles) return;  // whole waves only: no barrier follows
  hdiff_strip<T, kHStripRows, kHStripPD>(A, t, blockIdx.y);
}

}  // namespace gt4mi
