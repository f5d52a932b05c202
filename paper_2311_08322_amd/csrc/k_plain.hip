// k_plain.hip -- the per-stage ("plain") forward kernels: one kernel per
// stage of the two benchmark stencils (Sec. 3.1), every temporary
// round-tripping through HBM.  They are the baseline the fused kernels are
// measured against and the fallback for columns longer than the fused
// kernels' register classes.
#include "common.hpp"
#include "launch.hpp"

namespace gt4mi {

// lap on the box [-1, ni] x [-1, nj]
template <typename T>
__global__ void __launch_bounds__(kWG) k_lap_plain(StepArgs<T> A, T* __restrict__ lap) {
  const int li = blockIdx.x * 64 + threadIdx.x, lj = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
  const int LI = A.ni + 2, LJ = A.nj + 2;
  if (li >= LI || lj >= LJ) return;
  const T* u = A.u + (int64_t)(li - 1) + (int64_t)(lj - 1) * A.u_sj + (int64_t)k * A.u_sk;
  const T s = (u[-1] + u[1]) + (u[-A.u_sj] + u[A.u_sj]);
  lap[(int64_t)li + (int64_t)lj * LI + (int64_t)k * LI * LJ] = T(4) * u[0] - s;
}

// x-fluxes on [-1, ni) x [0, nj); one wave per 64-wide row chunk
template <typename T>
__global__ void __launch_bounds__(kWG) k_flx_plain(StepArgs<T> A, const T* __restrict__ lap,
                                                   T* __restrict__ fx) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
  const int LI = A.ni + 2, LJ = A.nj + 2;
  const bool row = j < A.nj;
  const bool on = row && i < A.ni;
  const T* L = lap + (int64_t)(j + 1) * LI + (int64_t)k * LI * LJ;  // L[i+1] = lap(i, j)
  const T* u = A.u + (int64_t)j * A.u_sj + (int64_t)k * A.u_sk;
  T* F = fx + (int64_t)j * (A.ni + 1) + (int64_t)k * (A.ni + 1) * A.nj;  // F[i+1] = Fx(i)
  bool keep = false;
  if (on) {
    const T f = L[i + 2] - L[i + 1], g = u[i + 1] - u[i];
    keep = flux_kept(f, g);
    F[i + 1] = keep ? f : T(0);
  }
  const uint64_t bits = __ballot(on && keep);
  if (A.mask && row && threadIdx.x == 0) {
    uint64_t* w = reinterpret_cast<uint64_t*>(A.mask + A.ml.x_off) +
                  ((int64_t)k * A.nj + j) * A.ml.words + blockIdx.x;
    *w = bits;
  }
  if (row && i == 0 && A.ni > 0) {  // the edge flux between (-1, j) and (0, j)
    const T f = L[1] - L[0], g = u[0] - u[-1];
    const bool ke = flux_kept(f, g);
    F[0] = ke ? f : T(0);
    if (A.mask) A.mask[A.ml.ex_off + (int64_t)k * A.nj + j] = ke ? 1 : 0;
  }
}

// y-fluxes on [0, ni) x [-1, nj); row lj holds j = lj - 1
template <typename T>
__global__ void __launch_bounds__(kWG) k_fly_plain(StepArgs<T> A, const T* __restrict__ lap,
                                                   T* __restrict__ fy) {
  const int i = blockIdx.x * 64 + threadIdx.x, lj = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
  const int j = lj - 1;
  const int LI = A.ni + 2, LJ = A.nj + 2;
  const bool row = lj < A.nj + 1;
  const bool on = row && i < A.ni;
  bool keep = false;
  if (on) {
    const T* L = lap + (int64_t)k * LI * LJ;
    const T l0 = L[(int64_t)(i + 1) + (int64_t)(j + 1) * LI];
    const T l1 = L[(int64_t)(i + 1) + (int64_t)(j + 2) * LI];
    const T* u = A.u + (int64_t)i + (int64_t)j * A.u_sj + (int64_t)k * A.u_sk;
    const T f = l1 - l0, g = u[A.u_sj] - u[0];
    keep = flux_kept(f, g);
    fy[(int64_t)i + (int64_t)lj * A.ni + (int64_t)k * A.ni * (A.nj + 1)] = keep ? f : T(0);
  }
  const uint64_t bits = __ballot(on && keep);
  if (A.mask && row) {
    if (j >= 0) {
      if (threadIdx.x == 0) {
        uint64_t* w = reinterpret_cast<uint64_t*>(A.mask + A.ml.y_off) +
                      ((int64_t)k * A.nj + j) * A.ml.words + blockIdx.x;
        *w = bits;
      }
    } else if (on) {
      A.mask[A.ml.ey_off + (int64_t)k * A.ni + i] = keep ? 1 : 0;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kWG) k_update_plain(StepArgs<T> A, const T* __restrict__ fx,
                                                      const T* __restrict__ fy) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, k = blockIdx.z;
  if (i >= A.ni || j >= A.nj) return;
  const T* F = fx + (int64_t)j * (A.ni + 1) + (int64_t)k * (A.ni + 1) * A.nj;
  const T* G = fy + (int64_t)i + (int64_t)k * A.ni * (A.nj + 1);
  const T div = (F[i + 1] - F[i]) + (G[(int64_t)(j + 1) * A.ni] - G[(int64_t)j * A.ni]);
  const T uc = A.u[(int64_t)i + (int64_t)j * A.u_sj + (int64_t)k * A.u_sk];
  A.out[(int64_t)i + (int64_t)j * A.o_sj + (int64_t)k * A.o_sk] = uc - A.coeff * div;
}

// Thomas elimination per column, c' and d' to HBM (interior layout)
template <typename T>
__global__ void __launch_bounds__(kWG) k_vadv_fwd_plain(StepArgs<T> A, T* __restrict__ cpw,
                                                        T* __restrict__ dpw) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y;
  if (i >= A.ni || j >= A.nj) return;
  const int64_t plane = (int64_t)A.ni * A.nj, col = (int64_t)i + (int64_t)j * A.ni;
  const T* u = A.u + (int64_t)i + (int64_t)j * A.u_sj;
  const T* d = A.data + (int64_t)i + (int64_t)j * A.d_sj;
  const T* w = A.w + (int64_t)i + (int64_t)j * A.w_sj;
  T cprev = T(0), dprev = T(0), wk = T(0);
  for (int k = 0; k < A.nk; ++k) {
    const T wk1 = (k + 1 < A.nk) ? w[(int64_t)(k + 1) * A.w_sk] : T(0);
    const T a = (k > 0) ? -A.r4 * wk : T(0);
    const T c = (k < A.nk - 1) ? A.r4 * wk1 : T(0);
    const T b = T(1) + (a < T(0) ? -a : a) + (c < T(0) ? -c : c);
    const T inv = recip(b - a * cprev);
    const T rhs = u[(int64_t)k * A.u_sk] + d[(int64_t)k * A.d_sk];
    cprev = c * inv;
    dprev = (rhs - a * dprev) * inv;
    cpw[col + k * plane] = cprev;
    dpw[col + k * plane] = dprev;
    wk = wk1;
  }
}

template <typename T>
__global__ void __launch_bounds__(kWG) k_vadv_bwd_plain(StepArgs<T> A, const T* __restrict__ cpw,
                                                        const T* __restrict__ dpw) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y;
  if (i >= A.ni || j >= A.nj) return;
  const int64_t plane = (int64_t)A.ni * A.nj, col = (int64_t)i + (int64_t)j * A.ni;
  T* o = A.out + (int64_t)i + (int64_t)j * A.o_sj;
  T x = T(0);
  for (int k = A.nk - 1; k >= 0; --k) {
    x = dpw[col + k * plane] - cpw[col + k * plane] * x;
    o[(int64_t)k * A.o_sk] = x;
  }
}

template <typename T>
hipError_t launch_hdiff_plain(const StepArgs<T>& A, const PlainWs<T>& ws, hipStream_t s) {
  const dim3 blk(64, 4);
  hipLaunchKernelGGL(k_lap_plain<T>, dim3((A.ni + 2 + 63) / 64, (A.nj + 2 + 3) / 4, A.nk), blk, 0,
                     s, A, ws.lap);
  hipLaunchKernelGGL(k_flx_plain<T>, dim3((A.ni + 63) / 64, (A.nj + 3) / 4, A.nk), blk, 0, s, A,
                     ws.lap, ws.fx);
  hipLaunchKernelGGL(k_fly_plain<T>, dim3((A.ni + 63) / 64, (A.nj + 1 + 3) / 4, A.nk), blk, 0, s,
                     A, ws.lap, ws.fy);
  hipLaunchKernelGGL(k_update_plain<T>, dim3((A.ni + 63) / 64, (A.nj + 3) / 4, A.nk), blk, 0, s,
                     A, ws.fx, ws.fy);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_vadv_plain(const StepArgs<T>& A, const PlainWs<T>& ws, hipStream_t s) {
  const dim3 blk(64, 4), grd((A.ni + 63) / 64, (A.nj + 3) / 4);
  hipLaunchKernelGGL(k_vadv_fwd_plain<T>, grd, blk, 0, s, A, ws.cp, ws.dp);
  hipLaunchKernelGGL(k_vadv_bwd_plain<T>, grd, blk, 0, s, A, ws.cp, ws.dp);
  return hipGetLastError();
}

// deterministic fill (autotuner scratch fields): a hash of the index
template <typename T>
__global__ void __launch_bounds__(kWG) k_fill(T* p, int64_t n, T lo, T hi, uint32_t seed) {
  for (int64_t e = blockIdx.x * (int64_t)kWG + threadIdx.x; e < n; e += (int64_t)gridDim.x * kWG) {
    uint32_t h = (uint32_t)e * 2654435761u ^ seed;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    p[e] = lo + (hi - lo) * (T)(h >> 8) * (T)(1.0 / 16777216.0);
  }
}

template <typename T>
hipError_t launch_fill_pattern(T* p, int64_t n, T lo, T hi, uint32_t seed, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + kWG - 1) / kWG;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(kWG), 0, s, p, n, lo, hi, seed);
  return hipGetLastError();
}

template hipError_t launch_hdiff_plain<float>(const StepArgs<float>&, const PlainWs<float>&, hipStream_t);
template hipError_t launch_hdiff_plain<double>(const StepArgs<double>&, const PlainWs<double>&, hipStream_t);
template hipError_t launch_vadv_plain<float>(const StepArgs<float>&, const PlainWs<float>&, hipStream_t);
template hipError_t launch_vadv_plain<double>(const StepArgs<double>&, const PlainWs<double>&, hipStream_t);
template hipError_t launch_fill_pattern<float>(float*, int64_t, float, float, uint32_t, hipStream_t);
template hipError_t launch_fill_pattern<double>(double*, int64_t, double, double, uint32_t, hipStream_t);

}  // namespace gt4mi
