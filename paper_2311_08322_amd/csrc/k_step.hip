// k_step.hip -- host dispatch of the fused forward column kernels (the
// register classes themselves are instantiated in k_step_inst.hip).
#include "launch.hpp"

namespace gt4mi {

template <typename T, int COL>
static hipError_t step_by_tile(const StepArgs<T>& A, int tile_i, hipStream_t s) {
  if (tile_i == 64) return launch_step_classes<T, 64, 4, COL>(A, s);
  if (tile_i == 32) return launch_step_classes<T, 32, 8, COL>(A, s);
  return launch_step_classes<T, 16, 16, COL>(A, s);
}

template <typename T, int NT>
static hipError_t split_by_tile(const StepArgs<T>& A, int tile_i, bool var, hipStream_t s) {
  if (var) {
    if (tile_i == 64) return launch_split_classes<T, 64, NT / 64, true>(A, s);
    if (tile_i == 32) return launch_split_classes<T, 32, NT / 32, true>(A, s);
    return launch_split_classes<T, 16, NT / 16, true>(A, s);
  }
  if (tile_i == 64) return launch_split_classes<T, 64, NT / 64, false>(A, s);
  if (tile_i == 32) return launch_split_classes<T, 32, NT / 32, false>(A, s);
  return launch_split_classes<T, 16, NT / 16, false>(A, s);
}

// tile_j: with tile_i, the tile of the two-ended step (tile_i * tile_j = 256
// or 128 columns); the one-lane kernels take tile_i x (256 / tile_i)
template <typename T>
hipError_t launch_step_fused(StepArgs<T> A, int tile_i, int tile_j, int col, hipStream_t s) {
  const bool var = A.kappa != nullptr || A.form != 0;  // the generalised diffusion: two-ended step only
  if (var || (col == 3 && A.nk <= split_step_limit(sizeof(T)))) {  // STENCIL_COLUMN_SPLIT
    if (A.nk > split_step_limit(sizeof(T))) return hipErrorInvalidValue;
    if constexpr (sizeof(T) == 8) {
      if (!var && A.nk > kSplitRegNkF64) {  // 97..144 levels: 128-column tiles, all in VGPRs
        const int tj = kSplitLongNT / tile_i;
        A.tiles_i = (A.ni + tile_i - 1) / tile_i;
        A.ntiles = A.tiles_i * ((A.nj + tj - 1) / tj);
        if (tile_i == 64) return launch_split_long<T, 64>(A, s);
        if (tile_i == 32) return launch_split_long<T, 32>(A, s);
        return launch_split_long<T, 16>(A, s);
      }
    }
    const bool narrow = tile_i * tile_j == 128;
    const int tj = (narrow ? 128 : 256) / tile_i;
    A.tiles_i = (A.ni + tile_i - 1) / tile_i;
    A.ntiles = A.tiles_i * ((A.nj + tj - 1) / tj);
    return narrow ? split_by_tile<T, 128>(A, tile_i, var, s) : split_by_tile<T, 256>(A, tile_i, var, s);
  }
  const int tj = kWG / tile_i;
  A.tiles_i = (A.ni + tile_i - 1) / tile_i;
  A.ntiles = A.tiles_i * ((A.nj + tj - 1) / tj);
  if constexpr (sizeof(T) == 4) {
    // binary32 columns up to the largest class fit their registers
    (void)col;
    return step_by_tile<T, 1>(A, tile_i, s);
  } else {
    // FP64 beyond 96 levels stages d' in the output field
    if (col == 2 || A.nk > 96) return step_by_tile<T, 2>(A, tile_i, s);
    return step_by_tile<T, 1>(A, tile_i, s);
  }
}

template <typename T>
hipError_t launch_vadv_fused(StepArgs<T> A, hipStream_t s) {
  if (A.nk <= column_split_limit(sizeof(T))) return launch_column_split_classes<T, false>(A, s);
  A.tiles_i = (A.ni + 63) / 64;
  A.ntiles = A.tiles_i * ((A.nj + 3) / 4);
  if constexpr (sizeof(T) == 4) {
    return launch_vadv_classes<T, 1>(A, s);
  } else {
    if (A.nk > 96) return launch_vadv_classes<T, 2>(A, s);
    return launch_vadv_classes<T, 1>(A, s);
  }
}

template hipError_t launch_step_fused<float>(StepArgs<float>, int, int, int, hipStream_t);
template hipError_t launch_step_fused<double>(StepArgs<double>, int, int, int, hipStream_t);
template hipError_t launch_vadv_fused<float>(StepArgs<float>, hipStream_t);
template hipError_t launch_vadv_fused<double>(StepArgs<double>, hipStream_t);

}  // namespace gt4mi
