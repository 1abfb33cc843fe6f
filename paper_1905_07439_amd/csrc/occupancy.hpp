// Resident workgroups of a leaf kernel on the current device (occupancy per CU
// times the CU count), cached per device and kernel, and the split of a tile
// count into whole rounds of full tiles plus a quarter-split last round (see
// split_tail in gemm_tiles.hpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <utility>

namespace rbc {

inline int64_t resident_blocks(const void* kernel, int block_threads) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, int64_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_pair(dev, kernel);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block_threads, 0) != hipSuccess)
    return 0;
  const int64_t r = (int64_t)cus * per_cu;
  cache[key] = r;
  return r;
}

struct TailSplit {
  int64_t n_big, n_small;  // full tiles, quarter tiles
};

// nt full-size tiles on `slots` resident workgroups: whole rounds stay full
// size and a partial last round is split in quarters; a launch of at most a
// quarter round is split entirely (four times the workgroups, all resident).
inline TailSplit tail_split(int64_t nt, int64_t slots) {
  if (slots <= 0 || nt % slots == 0 || nt > (int64_t(1) << 28)) return {nt, 0};
  if (4 * nt <= slots) return {0, 4 * nt};
  if (nt < slots) return {nt, 0};
  const int64_t big = (nt / slots) * slots;
  return {big, 4 * (nt - big)};
}

}  // namespace rbc
