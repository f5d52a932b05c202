// k_hdiff.hip -- launcher of the horizontal diffusion alone: the row walk
// (k_hdiff_strip.hpp) for the stated form with a scalar coefficient, the
// tile kernel (k_step.hpp) for the generalised diffusion.
#include "k_hdiff_strip.hpp"
#include "k_step.hpp"

namespace gt4mi {

template <typename T>
hipError_t launch_hdiff_fused(StepArgs<T> A, int tile_i, hipStream_t s) {
  const bool var = A.kappa != nullptr || A.form != 0;  // the generalised diffusion
  // the walk addresses the mask through one 32-bit window
  const bool small_mask = A.mask == nullptr || A.ml.total <= (int64_t)kOffNone - 16;
  if (!var && small_mask) {
    // the row walk: strips of 56 x kHStripRows outputs (FP32: 120, two
    // columns per lane), four per workgroup, one level per grid row (the tile
    // option does not apply)
    if constexpr (sizeof(T) == 4) {
      A.tiles_i = (A.ni + kHStripOut2 - 1) / kHStripOut2;
      A.ntiles = A.tiles_i * ((A.nj + kHStripRows - 1) / kHStripRows);
      const dim3 grid((A.ntiles + kStripsPerWG - 1) / kStripsPerWG, A.nk), block(kWG);
      if (hdiff_pairs_ok(A))
        hipLaunchKernelGGL(k_hdiff_strip2<true>, grid, block, 0, s, A);
      else
        hipLaunchKernelGGL(k_hdiff_strip2<false>, grid, block, 0, s, A);
      return hipGetLastError();
    }
    A.tiles_i = (A.ni + kHStripOut - 1) / kHStripOut;
    A.ntiles = A.tiles_i * ((A.nj + kHStripRows - 1) / kHStripRows);
    const dim3 grid((A.ntiles + kStripsPerWG - 1) / kStripsPerWG, A.nk), block(kWG);
    hipLaunchKernelGGL(k_hdiff_strip<T>, grid, block, 0, s, A);
    return hipGetLastError();
  }
  // the generalised diffusion (and masks of 4 GiB or more): a tile marched
  // over a block of levels; enough workgroups to fill the chip
  const int tj = kWG / tile_i;
  A.tiles_i = (A.ni + tile_i - 1) / tile_i;
  A.ntiles = A.tiles_i * ((A.nj + tj - 1) / tj);
  int kper = A.nk;
  while (kper > 4 && (int64_t)A.ntiles * ((A.nk + kper - 1) / kper) < 4096) kper = (kper + 1) / 2;
  A.k0 = 0;
  A.k1 = kper;
  dim3 grid(A.ntiles, (A.nk + kper - 1) / kper), block(kWG);
#define GT4MI_HDIFF_LAUNCH(TI, TJ)                                                  \
  if (var)                                                                          \
    hipLaunchKernelGGL((k_hdiff_fused<T, TI, TJ, true>), grid, block, 0, s, A);    \
  else                                                                              \
    hipLaunchKernelGGL((k_hdiff_fused<T, TI, TJ, false>), grid, block, 0, s, A);
  if (tile_i == 64) {
    GT4MI_HDIFF_LAUNCH(64, 4)
  } else if (tile_i == 32) {
    GT4MI_HDIFF_LAUNCH(32, 8)
  } else {
    GT4MI_HDIFF_LAUNCH(16, 16)
  }
#undef GT4MI_HDIFF_LAUNCH
  return hipGetLastError();
}

template hipError_t launch_hdiff_fused<float>(StepArgs<float>, int, hipStream_t);
template hipError_t launch_hdiff_fused<double>(StepArgs<double>, int, hipStream_t);

}  // namespace gt4mi
