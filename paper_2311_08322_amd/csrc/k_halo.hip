// k_halo.hip -- periodic boundary condition: the 2-point halo of a padded
// field is filled from the interior at the wrapped indices (i mod ni,
// j mod nj), corners included.  The sources are interior points only, so
// one pass over the halo ring of every level is race free.
#include "launch.hpp"

namespace gt4mi {

__device__ __forceinline__ int wrap_index(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

// p: the field at domain point (0,0,0).  Ring of a level: rows -2, -1 and
// nj, nj+1 over i in [-2, ni+2), then columns -2, -1, ni, ni+1 of rows
// 0 .. nj-1.
template <typename T>
__global__ void __launch_bounds__(kWG) k_halo_periodic(T* p, int64_t sj, int64_t sk, int ni, int nj, int nk) {
  const int W = ni + 4;
  const int64_t ring = 4 * (int64_t)W + 4 * (int64_t)nj;
  const int64_t total = ring * nk;
  for (int64_t t = blockIdx.x * (int64_t)kWG + threadIdx.x; t < total; t += (int64_t)gridDim.x * kWG) {
    const int k = (int)(t / ring);
    const int r = (int)(t - (int64_t)k * ring);
    int i, j;
    if (r < 4 * W) {  // the two rows above and the two below
      const int row = r / W;
      i = r - row * W - 2;
      j = row < 2 ? row - 2 : nj + row - 2;
    } else {  // the side columns of the interior rows
      const int s = r - 4 * W;
      j = s >> 2;
      const int c = s & 3;
      i = c < 2 ? c - 2 : ni + c - 2;
    }
    const T v = p[(int64_t)k * sk + (int64_t)wrap_index(j, nj) * sj + wrap_index(i, ni)];
    p[(int64_t)k * sk + (int64_t)j * sj + i] = v;
  }
}

template <typename T>
hipError_t launch_halo_periodic(T* p, int64_t sj, int64_t sk, int ni, int nj, int nk, hipStream_t s) {
  if (ni <= 0 || nj <= 0 || nk <= 0) return hipSuccess;
  const int64_t total = (4 * (int64_t)(ni + 4) + 4 * (int64_t)nj) * nk;
  const int64_t blocks = (total + kWG - 1) / kWG;
  const int grid = (int)(blocks < 4096 ? blocks : 4096);
  hipLaunchKernelGGL(k_halo_periodic<T>, dim3(grid), dim3(kWG), 0, s, p, sj, sk, ni, nj, nk);
  return hipGetLastError();
}

template hipError_t launch_halo_periodic<float>(float*, int64_t, int64_t, int, int, int, hipStream_t);
template hipError_t launch_halo_periodic<double>(double*, int64_t, int64_t, int, int, int, hipStream_t);

}  // namespace gt4mi
