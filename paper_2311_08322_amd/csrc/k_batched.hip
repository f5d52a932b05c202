// k_batched.hip -- kernels that run a batch of fields of uneven sizes in one
// launch each.
//
// The host sorts the fields longest column first and writes a table into
// the caller's workspace (a header with the per-field prefix sums of work
// items, then one argument block per field) with small copy kernels, so the
// whole call is stream-ordered device work that a HIP graph can capture.
// The column kernels (forward step, column adjoint) are persistent: every
// workgroup pulls work items (field, column tile) from an atomic queue in
// the header until the queue is exhausted.  The horizontal adjoint's items
// (field, four strips, one level) are short, so it launches one workgroup
// per item instead, which finds its item in the prefix sums.  A work item
// runs the same body as the single-field kernel.
#include <string.h>

#include "common.hpp"
#include "k_colsplit.hpp"
#include "k_hadj_strip.hpp"
#include "k_split.hpp"
#include "launch.hpp"
#include "persist.hpp"

namespace gt4mi {

// ------------------------------------------------------------------ table upload
#ifdef GT4MI_UPLOAD
struct ByteChunk {
  uint32_t nwords;
  uint32_t words[960];
};

__global__ void __launch_bounds__(kWG) k_write_words(uint32_t* dst, ByteChunk c) {
  for (uint32_t t = threadIdx.x; t < c.nwords; t += kWG) dst[t] = c.words[t];
}

hipError_t launch_upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const uint32_t* w = static_cast<const uint32_t*>(src);
  const size_t nwords = (bytes + 3) / 4;
  for (size_t off = 0; off < nwords; off += 960) {
    ByteChunk c;
    c.nwords = (uint32_t)((nwords - off) < 960 ? (nwords - off) : 960);
    memcpy(c.words, w + off, c.nwords * 4);
    hipLaunchKernelGGL(k_write_words, dim3(1), dim3(kWG), 0, s, static_cast<uint32_t*>(dst) + off, c);
  }
  return hipGetLastError();
}
#endif

// ------------------------------------------------------------------ queue
// The work list is written by the upload kernels before the launch and is
// the same for every lane: values read from it are taken from lane 0, so
// the field, its argument block and the buffer descriptors built from it
// are known to be uniform and stay in SGPRs.
__device__ __forceinline__ int uniform_ld(const int32_t* p) { return __builtin_amdgcn_readfirstlane(*p); }

template <typename S>
__device__ __forceinline__ S uniform_ld(const S* p) {
  static_assert(sizeof(S) % 4 == 0, "argument blocks are whole words");
  struct Words {
    uint32_t w[sizeof(S) / 4];
  } v;
  const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(S) / 4); ++i) v.w[i] = __builtin_amdgcn_readfirstlane(q[i]);
  return __builtin_bit_cast(S, v);
}

// Next work item of the workgroup (uniform), or -1 when the queue is empty.
// The table upload of each call zeroes the counter, so no reset is needed.
__device__ __forceinline__ int next_work(BatchHeader* h, int* slot) {
  if (threadIdx.x == 0) *slot = (int)atomicAdd(&h->queue, 1u);
  __syncthreads();
  // every lane reads the same value; taking lane 0's makes it a scalar, so
  // the item's argument block and buffer descriptors stay in SGPRs
  const int w = __builtin_amdgcn_readfirstlane(*slot);
  __syncthreads();  // every lane has the value before the slot is reused
  return w < uniform_ld(&h->total) ? w : -1;
}

// Field of work item w: the last e with prefix[e] <= w.
__device__ __forceinline__ int find_entry(const BatchHeader* h, int w) {
  const int32_t* p = h->prefix();
  int lo = 0, hi = uniform_ld(&h->n) - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (uniform_ld(p + mid) <= w) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------------ kernels
// The fields of one launch may run different tile shapes (each field takes
// the tile that wastes the fewest lanes on its ragged edges): the work item
// runs the body of its field's tile, a uniform branch, in LDS shared by the
// three shapes.
template <typename T, int NT>
union BatchSmem {
  SplitSmem<T, 64, NT / 64> t64;
  SplitSmem<T, 32, NT / 32> t32;
  SplitSmem<T, 16, NT / 16> t16;
};

template <typename T, int NT, int NKH, int PD, bool MASK>
__device__ __forceinline__ void batched_step_item(const StepArgs<T>& A, int tile, BatchSmem<T, NT>& sm) {
  if (A.tile_i == 64)
    step_split_tile<T, 64, NT / 64, NKH, PD, MASK, 1>(A, tile, sm.t64);
  else if (A.tile_i == 32)
    step_split_tile<T, 32, NT / 32, NKH, PD, MASK, 1>(A, tile, sm.t32);
  else
    step_split_tile<T, 16, NT / 16, NKH, PD, MASK, 1>(A, tile, sm.t16);
}

// Forward step, half-column register class NKH.  FP64 columns up to
// kBatchedShortNk levels run in the 40-level class (the 48-level class
// would spill beside the persistent loop's own registers), longer ones in
// k_step_batched_long; FP32 columns all run in the 72-level class.
template <typename T, int NKH, bool MASK>
__global__ void __launch_bounds__(2 * kWG) k_step_batched(BatchHeader* h, const StepArgs<T>* ent) {
  __shared__ BatchSmem<T, kWG> sm;
  __shared__ int slot;
  for (;;) {
    const int w = next_work(h, &slot);
    if (w < 0) break;
    const int e = find_entry(h, w);
    const StepArgs<T> A = uniform_ld(ent + e);
    const int tile = w - uniform_ld(h->prefix() + e);
    batched_step_item<T, kWG, NKH, GT4MI_PD, MASK>(A, tile, sm);
    __syncthreads();  // the LDS is reused by the next item
  }
}

#ifdef GT4MI_BATCHED_LONG
// FP64 columns of kBatchedShortNk+1 .. 144 levels: tiles of kSplitLongNT
// columns (256 lanes) with e and f in VGPRs, as the single-field long form.
template <typename T, bool MASK>
__global__ void __launch_bounds__(2 * kSplitLongNT) k_step_batched_long(BatchHeader* h, const StepArgs<T>* ent) {
  __shared__ BatchSmem<T, kSplitLongNT> sm;
  __shared__ int slot;
  for (;;) {
    const int w = next_work(h, &slot);
    if (w < 0) break;
    const int e = find_entry(h, w);
    const StepArgs<T> A = uniform_ld(ent + e);
    const int tile = w - uniform_ld(h->prefix() + e);
    batched_step_item<T, kSplitLongNT, kSplitStagedNkhF64, GT4MI_PD_LONG, MASK>(A, tile, sm);
    __syncthreads();
  }
}
#endif

// Column adjoint lambda = T^{-T} x_bar (argument blocks in column form).
template <typename T>
__global__ void __launch_bounds__(2 * kWG) k_vadj_batched(BatchHeader* h, const StepArgs<T>* ent) {
  __shared__ T xch[2][2][kWG];
  __shared__ int slot;
  for (;;) {
    const int w = next_work(h, &slot);
    if (w < 0) break;
    const int e = find_entry(h, w);
    const StepArgs<T> A = uniform_ld(ent + e);
    const int tile = w - uniform_ld(h->prefix() + e);
    if constexpr (sizeof(T) == 8) {
      if (A.nk <= 96)
        column_split_tile<T, 48, GT4MI_COL_PD, true, 1>(A, tile, xch);
      else
        column_split_tile<T, 72, GT4MI_COL_PD, true, 2>(A, tile, xch);
    } else {
      column_split_tile<T, 72, GT4MI_COL_PD, true, 1>(A, tile, xch);
    }
    __syncthreads();
  }
}

// Horizontal adjoint: one workgroup per work item (field, group of
// kStripsPerWG strips, level), as the single-field gather's grid; each wave
// walks its strip of the group (FP32 strips hold two columns per lane).
template <typename T>
__global__ void __launch_bounds__(kWG) k_hadj_batched(const BatchHeader* h, const AdjArgs<T>* ent) {
  const int w = blockIdx.x;
  const int e = find_entry(h, w);
  const AdjArgs<T> A = uniform_ld(ent + e);
  const int local = w - uniform_ld(h->prefix() + e);
  const int groups = (A.ntiles + kStripsPerWG - 1) / kStripsPerWG;
  const int g = local % groups, k = local / groups;
  const int t = __builtin_amdgcn_readfirstlane(g * kStripsPerWG + (int)(threadIdx.x >> 6));
  if (t < A.ntiles) {
    if constexpr (sizeof(T) == 4)
    {  // two columns per lane, read in pairs where the item's lambda allows (uniform)
      if (lambda_pairs_ok(A))
        hdiff_adjoint_strip2<strip_rows<float>(), strip_pd<float>(), false, true>(A, t, k);
      else
        hdiff_adjoint_strip2<strip_rows<float>(), strip_pd<float>(), false, false>(A, t, k);
    }
    else
      hdiff_adjoint_strip<T, strip_rows<T>(), strip_pd<T>(), false>(A, t, k);
  }
}

// ------------------------------------------------------------------ launchers
template <typename T>
hipError_t launch_step_batched(BatchHeader* h, const StepArgs<T>* ent, int total, bool mask, hipStream_t s) {
  constexpr int NKH = sizeof(T) == 8 ? kBatchedShortNk / 2 : 72;
  auto go = [&](auto kernel) {
    const int grid = persistent_grid(kernel, 2 * kWG, total);
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(2 * kWG), 0, s, h, ent);
    return hipGetLastError();
  };
  return mask ? go(k_step_batched<T, NKH, true>) : go(k_step_batched<T, NKH, false>);
}

#ifdef GT4MI_BATCHED_LONG
template <typename T>
hipError_t launch_step_batched_long(BatchHeader* h, const StepArgs<T>* ent, int total, bool mask, hipStream_t s) {
  auto go = [&](auto kernel) {
    const int grid = persistent_grid(kernel, 2 * kSplitLongNT, total);
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(2 * kSplitLongNT), 0, s, h, ent);
    return hipGetLastError();
  };
  return mask ? go(k_step_batched_long<T, true>) : go(k_step_batched_long<T, false>);
}
#endif

template <typename T>
hipError_t launch_vadj_batched(BatchHeader* h, const StepArgs<T>* ent, int total, hipStream_t s) {
  const int grid = persistent_grid(k_vadj_batched<T>, 2 * kWG, total);
  hipLaunchKernelGGL(k_vadj_batched<T>, dim3(grid), dim3(2 * kWG), 0, s, h, ent);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_hadj_batched(BatchHeader* h, const AdjArgs<T>* ent, int total, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hadj_batched<T>, dim3(total), dim3(kWG), 0, s, h, ent);
  return hipGetLastError();
}

// one object per element type (-DGT4MI_T=float|double); the float one also
// holds the table upload (-DGT4MI_UPLOAD), the double one the long-column
// forward (-DGT4MI_BATCHED_LONG)
template hipError_t launch_step_batched<GT4MI_T>(BatchHeader*, const StepArgs<GT4MI_T>*, int, bool, hipStream_t);
template hipError_t launch_vadj_batched<GT4MI_T>(BatchHeader*, const StepArgs<GT4MI_T>*, int, hipStream_t);
template hipError_t launch_hadj_batched<GT4MI_T>(BatchHeader*, const AdjArgs<GT4MI_T>*, int, hipStream_t);
#ifdef GT4MI_BATCHED_LONG
template hipError_t launch_step_batched_long<GT4MI_T>(BatchHeader*, const StepArgs<GT4MI_T>*, int, bool, hipStream_t);
#endif

}  // namespace gt4mi
