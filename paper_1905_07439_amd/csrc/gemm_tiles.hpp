// Device-side leaf product tiles, shared by the leaf kernels (gemm*.hip) and by
// the batch engine's kernels (batch*.hip).  Each tile function computes one
// output tile given its logical tile index and a pointer to the workgroup's LDS
// block; one header per leaf format (tile_f32.hpp, tile_lowp.hpp,
// tile_fp8.hpp).  This header holds what they share: vector types and the
// block-to-tile mappings.
//
#pragma once

#include <hip/hip_runtime.h>

#include "devptr.hpp"
#include "kernels.hpp"

namespace rbc {
namespace tiles {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x8 __attribute__((ext_vector_type(8)));

// Block id -> logical tile id such that consecutive logical tiles share an XCD
// (workgroups are dispatched round robin over the 8 XCDs).
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nb) {
  const int64_t per = nb / 8, rem = nb % 8;
  const int64_t xcd = bid % 8, local = bid / 8;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// Launches whose tiles do not fill whole rounds of the resident grid: the
// first n_big blocks compute full tiles (ids 0 .. n_big - 1, whole rounds),
// the remaining blocks the last tiles split in quarters (tiles of half the
// side), so that the last round is spread over every CU.  Every output gets
// the same arithmetic in either tile size.  Returns true and the full-size
// tile id for a full tile, false and the half-size tile id (leaf-major over
// the half-size tile grid) for a quarter.
__device__ __forceinline__ bool split_tail(int64_t b, int64_t n_big, int64_t n_small, int tiles_n,
                                          int tiles_per_leaf, int64_t* bid) {
  if (b < n_big) {
    *bid = xcd_remap(b, n_big);
    return true;
  }
  const int64_t sq = xcd_remap(b - n_big, n_small);
  const int64_t big = n_big + sq / 4;
  const int q = (int)(sq % 4);
  const int64_t leaf = big / tiles_per_leaf;
  const int t = (int)(big - leaf * tiles_per_leaf), tm = t / tiles_n, tn = t - (t / tiles_n) * tiles_n;
  *bid = leaf * 4 * (int64_t)tiles_per_leaf + (int64_t)(2 * tm + q / 2) * (2 * tiles_n) + 2 * tn + q % 2;
  return false;
}

}  // namespace tiles
}  // namespace rbc

