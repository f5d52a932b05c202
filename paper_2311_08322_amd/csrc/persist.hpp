// persist.hpp -- grid size of persistent kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

namespace gt4mi {

// Resident workgroups per CU times the CU count: the persistent grid.  The
// occupancy query runs once per device and kernel (and so never inside a
// stream capture after an eager call).
template <typename K>
inline int persistent_grid(K kernel, int block, int total) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  int g = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_pair(dev, reinterpret_cast<const void*>(kernel));
    auto it = cache.find(key);
    if (it == cache.end()) {
      int cus = 0, per = 0;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, block, 0) != hipSuccess || per <= 0) per = 1;
      it = cache.emplace(key, cus * per).first;
    }
    g = it->second;
  }
  return total < g ? (total > 0 ? total : 1) : g;
}

}  // namespace gt4mi
