// k_step_inst.hip -- explicit instantiations of the fused column kernels,
// one (dtype, tile, column store) set per compilation of this file:
//   -DGT4MI_T=double|float -DGT4MI_TI=64|32|16 -DGT4MI_COL=1|2  (step)
//   -DGT4MI_T=... -DGT4MI_VADV -DGT4MI_COL=1|2                   (vadv)
//   -DGT4MI_T=... -DGT4MI_TI=64|32|16 -DGT4MI_SPLIT [-DGT4MI_VAR]  (two-ended step; VAR:
//                                                                  the generalised diffusion;
//                                                                  -DGT4MI_SPLIT_LONG with FP64
//                                                                  and no VAR: also the
//                                                                  128-column long form)
//   -DGT4MI_T=... -DGT4MI_COLSPLIT -DGT4MI_ADJ=false|true          (two-ended column solves)
// Splitting keeps each fully unrolled register class in a parallel job.
#include "k_colsplit.hpp"
#include "k_split.hpp"

namespace gt4mi {

#if defined(GT4MI_COLSPLIT)
template hipError_t launch_column_split_classes<GT4MI_T, GT4MI_ADJ>(StepArgs<GT4MI_T>, hipStream_t);
#elif defined(GT4MI_SPLIT)
#ifdef GT4MI_VAR
template hipError_t launch_split_classes<GT4MI_T, GT4MI_TI, GT4MI_SPLIT_NT / GT4MI_TI, true>(
    const StepArgs<GT4MI_T>&, hipStream_t);
#else
template hipError_t launch_split_classes<GT4MI_T, GT4MI_TI, GT4MI_SPLIT_NT / GT4MI_TI, false>(
    const StepArgs<GT4MI_T>&, hipStream_t);
#ifdef GT4MI_SPLIT_LONG
template hipError_t launch_split_long<double, GT4MI_TI>(const StepArgs<double>&, hipStream_t);
#endif
#endif
#elif defined(GT4MI_VADV)
template hipError_t launch_vadv_classes<GT4MI_T, GT4MI_COL>(const StepArgs<GT4MI_T>&, hipStream_t);
#else
template hipError_t launch_step_classes<GT4MI_T, GT4MI_TI, 256 / GT4MI_TI, GT4MI_COL>(
    const StepArgs<GT4MI_T>&, hipStream_t);
#endif

}  // namespace gt4mi
