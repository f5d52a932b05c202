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
hipError_t launch_step_fused(StepArgs<T> A, int tile_i, int tile_j, int column_store, hipStream_t s);
template <typename T, int TI, int TJ, int COL>
hipError_t launch_step_classes(const StepArgs<T>& A, hipStream_t s);
template <typename T, int COL>
hipError_t launch_vadv_classes(const StepArgs<T>& A, hipStream_t s);
// VAR: the generalised diffusion (per-point coefficient, damping form)
template <typename T, int TI, int TJ, bool VAR>
hipError_t launch_split_classes(const StepArgs<T>& A, hipStream_t s);
// FP64 columns of 97..144 levels in 128-column tiles (k_split.hpp)
template <typename T, int TI>
hipError_t launch_split_long(const StepArgs<T>& A, hipStream_t s);
// two-ended column solve: ADJ = false, out = T^{-1}(u + data);
// ADJ = true, out = T^{-T} u (u holds x_bar); nk <= 144 (FP64) / 160 (FP32)
template <typename T, bool ADJ>
hipError_t launch_column_split_classes(StepArgs<T> A, hipStream_t s);
constexpr int column_split_limit(int elem_bytes) { return elem_bytes == 8 ? 144 : 160; }
// Columns per tile of the two-ended fused step (two lanes per column) in one
// compilation of k_step_inst.hip: 256 makes 512-lane workgroups, 128 makes
// 256-lane ones; both are built and the tile option (a tuned dimension)
// picks one.
#ifndef GT4MI_SPLIT_NT
#define GT4MI_SPLIT_NT 256
#endif
// two-ended fused step (k_split.hpp): nk <= 144 (FP64) / 160 (FP32)
constexpr int split_step_limit(int elem_bytes) { return elem_bytes == 8 ? 144 : 160; }
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
hipError_t launch_hdiff_adjoint(AdjArgs<T> A, hipStream_t s);

// batched launches (k_batched.hip).  The work list sits in device memory: a
// BatchHeader, then prefix[n + 1] (first work item of each field), then the
// fields' argument blocks.
struct BatchHeader {
  uint32_t queue;  // next work item, taken with atomicAdd (persistent launches)
  int32_t n;       // fields
  int32_t total;   // work items
  int32_t pad;
  __host__ __device__ const int32_t* prefix() const { return reinterpret_cast<const int32_t*>(this + 1); }
};
// longest column of a batched field (both halves' e in VGPRs, f staged)
constexpr int kMaxBatchedNk = 144;
// stream-ordered copy of a small host table into device memory (kernel
// arguments, so that a captured graph holds its own copy)
hipError_t launch_upload(void* dst, const void* src, size_t bytes, hipStream_t s);
// FP64 columns of up to kBatchedShortNk levels run in the 40-level
// half-column class, longer ones in launch_step_batched_long; FP32 columns
// all run in the 72-level class.  Each argument block names its field's
// tile width (StepArgs::tile_i: tiles of kWG columns, kSplitLongNT in the
// long launch).
constexpr int kBatchedShortNk = 80;
template <typename T>
hipError_t launch_step_batched(BatchHeader* h, const StepArgs<T>* ent, int total, bool mask, hipStream_t s);
template <typename T>
hipError_t launch_step_batched_long(BatchHeader* h, const StepArgs<T>* ent, int total, bool mask, hipStream_t s);
template <typename T>
hipError_t launch_vadj_batched(BatchHeader* h, const StepArgs<T>* ent, int total, hipStream_t s);
template <typename T>
hipError_t launch_hadj_batched(BatchHeader* h, const AdjArgs<T>* ent, int total, hipStream_t s);

// parameter gradients of a step (k_param.hip)
template <typename T>
struct WGradArgs {
  const T* w;  // staggered level 0 at domain (0,0)
  int64_t w_sj, w_sk;
  const T* x;  // the step's output
  int64_t x_sj, x_sk;
  const T* lam;  // T^{-T} x_bar
  int64_t l_sj, l_sk;
  T* wbar;  // staggered, nk+1 levels written
  int64_t b_sj, b_sk;
  int ni, nj, nk, tiles_i;
  T q;  // dt_dz / 4
};
// per-tile partial sums of the coeff gradient: one double per 64 x 4 tile
inline size_t coeff_partial_count(int64_t ni, int64_t nj) {
  return (size_t)((ni + 63) / 64) * (size_t)((nj + 3) / 4);
}
// A: u (halo) and lam in the data slot; W may be NULL (no w_bar);
// coeff_bar may be NULL (no reduction; partial unused)
template <typename T>
hipError_t launch_param_grads(const StepArgs<T>& A, const WGradArgs<T>* W, double* partial, double* coeff_bar,
                              hipStream_t s);

// gradient of a per-point coefficient: A.out(p) = -A.data(p) D(u)(p)
// (A.data holds lam; A.form selects the Laplacian form)
template <typename T>
hipError_t launch_coeff_field_grad(const StepArgs<T>& A, hipStream_t s);

// periodic halo fill of a padded field (p at domain (0,0,0); k_halo.hip)
template <typename T>
hipError_t launch_halo_periodic(T* p, int64_t sj, int64_t sk, int ni, int nj, int nk, hipStream_t s);

// fill a strided box with a deterministic pattern (autotuner scratch)
template <typename T>
hipError_t launch_fill_pattern(T* p, int64_t n, T lo, T hi, uint32_t seed, hipStream_t s);

}  // namespace gt4mi
