// k_hdiff.hip -- launcher of the fused horizontal diffusion alone.
#include "k_step.hpp"

namespace gt4mi {

template <typename T>
hipError_t launch_hdiff_fused(StepArgs<T> A, int tile_i, hipStream_t s) {
  // tile marched over a block of levels; enough workgroups to fill the chip
  const int tj = kWG / tile_i;
  A.tiles_i = (A.ni + tile_i - 1) / tile_i;
  A.ntiles = A.tiles_i * ((A.nj + tj - 1) / tj);
  int kper = A.nk;
  while (kper > 4 && (int64_t)A.ntiles * ((A.nk + kper - 1) / kper) < 4096) kper = (kper + 1) / 2;
  A.k0 = 0;
  A.k1 = kper;
  dim3 grid(A.ntiles, (A.nk + kper - 1) / kper), block(kWG);
  const bool var = A.kappa != nullptr || A.form != 0;  // the generalised diffusion
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
