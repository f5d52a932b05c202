// launch.hpp -- host-side launchers of the gfx950 kernels (library-internal).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace gt4mi {

// Longest column the fused (register-resident) column kernels accept.
constexpr int kMaxFusedNk = 160;

// fused forward (k_step.hip dispatches; k_step_inst.hip instantiates the
// register classes of each dtype / tile / column store)
template <typename T>
hipError_t launch_step_fused(StepArgs<T> A, int tile_i, int column_store, hipStream_t s);
template <typename T, int TI, int TJ, int COL>
hipError_t launch_step_classes(const StepArgs<T>& A, hipStream_t s);
template <typename T, int COL>
hipError_t launch_vadv_classes(const StepArgs<T>& A, hipStream_t s);
template <typename T, int TI, int TJ>
hipError_t launch_split_classes(const StepArgs<T>& A, hipStream_t s);
// two-ended column solve: ADJ = false, out = T^{-1}(u + data);
// ADJ = true, out = T^{-T} u (u holds x_bar); nk <= 96 (FP64) / 160 (FP32)
template <typename T, bool ADJ>
hipError_t launch_column_split_classes(StepArgs<T> A, hipStream_t s);
constexpr int column_split_limit(int elem_bytes) { return elem_bytes == 8 ? 96 : 160; }
template <typename T>
hipError_t launch_vadv_fused(StepArgs<T> A, hipStream_t s);
template <typename T>
hipError_t launch_hdiff_fused(StepArgs<T> A, int tile_i, hipStream_t s);

// plain per-stage forward (k_plain.hip); ws holds the stage temporaries
template <typename T>
struct PlainWs {
  T* lap;  // (ni+2) x (nj+2) x nk
  T* fx;   // (ni+1) x nj x nk
  T* fy;   // ni x (nj+1) x nk
  T* cp;   // ni x nj x nk
  T* dp;   // ni x nj x nk
};
template <typename T>
hipError_t launch_hdiff_plain(const StepArgs<T>& A, const PlainWs<T>& ws, hipStream_t s);
// out = T^{-1}(u + data) with u, data, out given by A; elimination factors in ws
template <typename T>
hipError_t launch_vadv_plain(const StepArgs<T>& A, const PlainWs<T>& ws, hipStream_t s);

// adjoints (k_adjoint.hip; column classes in k_vadj_inst.hip)
template <typename T>
hipError_t launch_vadv_adjoint(AdjArgs<T> A, int impl_plain, T* ws_y, T* ws_c, hipStream_t s);
template <typename T, int COL>
hipError_t launch_vadj_classes(const AdjArgs<T>& A, hipStream_t s);
template <typename T>
hipError_t launch_hdiff_adjoint(AdjArgs<T> A, int tile_i, hipStream_t s);

// fill a strided box with a deterministic pattern (autotuner scratch)
template <typename T>
hipError_t launch_fill_pattern(T* p, int64_t n, T lo, T hi, uint32_t seed, hipStream_t s);

}  // namespace gt4mi
