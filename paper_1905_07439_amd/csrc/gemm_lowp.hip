// Reduced-precision leaf products on CDNA4 matrix cores, f32 accumulation.
//
//   bf16x3: P = S_hi T_hi + S_hi T_lo + S_lo T_hi, operands split by the gather
//           (S = S_hi + S_lo, each part rounded to bf16); v_mfma_f32_16x16x32_bf16.
//           The dropped term S_lo T_lo is below 2^-16 relative to |S||T|.
//   f16s:   P = 2^-(eS + eT) (S' T') with S' = rn_f16(2^eS S), T' = rn_f16(2^eT T),
//           one power-of-two scale per leaf operand chosen by the gather so that
//           no value can overflow; v_mfma_f32_16x16x32_f16.  The unscaling is exact.
//
// Tile BM x BN (32, 64, 96 or 128) per workgroup of 4 wavefronts, each a
// (BM/2) x (BN/2) quarter of 16x16 MFMA tiles, K slabs of 32 (the tile is
// described in tile_lowp.hpp: S operands are 16-byte LDS reads, T operands
// transposing LDS reads).  Two LDS buffers: a slab held in registers is
// written to one, one barrier, then the next slab's global loads stay in
// flight while the MFMAs consume the buffer.  Block ids are remapped so that
// one leaf's tiles run on one XCD.  128- and 64-tile launches run the partial
// last round of the resident grid as tiles of half the side (split_tail).
#include <hip/hip_runtime.h>

#include "tile_lowp.hpp"
#include "occupancy.hpp"

namespace rbc {
namespace {

using tiles::LowpTile;

template <int KIND, int BM, int BN>
__global__ __launch_bounds__(256) void k_gemm_lowp(const uint16_t* __restrict__ S,
                                                   const uint16_t* __restrict__ T,
                                                   float* __restrict__ P, int m, int n, int k,
                                                   int64_t plane_s, int64_t plane_t,
                                                   const int32_t* __restrict__ eS,
                                                   const int32_t* __restrict__ eT, int tiles_n,
                                                   int tiles_per_leaf, int64_t nblocks) {
  __shared__ __attribute__((aligned(16))) uint16_t smem[LowpTile<KIND, BM, BN>::SMEM_HALVES];
  tiles::gemm_lowp_tile<KIND, BM, BN>(S, T, P, m, n, k, plane_s, plane_t, eS, eT, tiles_n,
                                      tiles_per_leaf, tiles::xcd_remap(blockIdx.x, nblocks), smem);
}

// Tiles of BM with the last partial round as tiles of BM / 2 (split_tail).
template <int KIND, int BM>
__global__ __launch_bounds__(256) void k_gemm_lowp_split(const uint16_t* __restrict__ S,
                                                         const uint16_t* __restrict__ T, float* __restrict__ P,
                                                         int m, int n, int k, int64_t plane_s, int64_t plane_t,
                                                         const int32_t* __restrict__ eS,
                                                         const int32_t* __restrict__ eT, int tiles_n,
                                                         int tiles_per_leaf, int64_t n_big, int64_t n_small) {
  constexpr int H = BM / 2;
  constexpr int SB = LowpTile<KIND, BM, BM>::SMEM_HALVES, SH = LowpTile<KIND, H, H>::SMEM_HALVES;
  __shared__ __attribute__((aligned(16))) uint16_t smem[SB > SH ? SB : SH];
  int64_t bid;
  if (tiles::split_tail(blockIdx.x, n_big, n_small, tiles_n, tiles_per_leaf, &bid))
    tiles::gemm_lowp_tile<KIND, BM, BM>(S, T, P, m, n, k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf, bid,
                                        smem);
  else
    tiles::gemm_lowp_tile<KIND, H, H>(S, T, P, m, n, k, plane_s, plane_t, eS, eT, 2 * tiles_n,
                                      4 * tiles_per_leaf, bid, smem);
}

// Large tiles BM x BN on NWM x NWN wavefronts with the partial last round as (BM/2) x
// (BN/2) tiles on SWM x SWN wavefronts (LowpTileW; same bits as the 128-tiles).
template <int KIND, int BM, int BN, int NWM, int NWN, int SWM, int SWN>
__global__ __launch_bounds__(64 * NWM * NWN) void k_gemm_lowp_wide(
    const uint16_t* __restrict__ S, const uint16_t* __restrict__ T, float* __restrict__ P, int m, int n, int k,
    int64_t plane_s, int64_t plane_t, const int32_t* __restrict__ eS, const int32_t* __restrict__ eT, int tiles_n,
    int tiles_per_leaf, int64_t n_big, int64_t n_small) {
  static_assert(NWM * NWN == SWM * SWN, "one thread count for both tile sizes");
  constexpr int SB = tiles::LowpTileW<KIND, BM, BN, NWM, NWN>::SMEM_HALVES;
  constexpr int SH = tiles::LowpTileW<KIND, BM / 2, BN / 2, SWM, SWN>::SMEM_HALVES;
  __shared__ __attribute__((aligned(16))) uint16_t smem[SB > SH ? SB : SH];
  int64_t bid;
  if (tiles::split_tail(blockIdx.x, n_big, n_small, tiles_n, tiles_per_leaf, &bid))
    tiles::gemm_lowp_tile_w<KIND, BM, BN, NWM, NWN>(S, T, P, m, n, k, plane_s, plane_t, eS, eT, tiles_n,
                                                    tiles_per_leaf, bid, smem);
  else
    tiles::gemm_lowp_tile_w<KIND, BM / 2, BN / 2, SWM, SWN>(S, T, P, m, n, k, plane_s, plane_t, eS, eT,
                                                            2 * tiles_n, 4 * tiles_per_leaf, bid, smem);
}

template <int KIND, int BM, int BN, int NWM, int NWN, int SWM, int SWN>
void launch_wide(hipStream_t stream, const uint16_t* S, const uint16_t* T, float* P, int64_t m, int64_t n, int64_t k,
                 int64_t batch, const int32_t* eS, const int32_t* eT) {
  const int tiles_n = (int)(n / BN), tiles_per_leaf = (int)((m / BM) * tiles_n);
  const int64_t nblocks = batch * tiles_per_leaf;
  const int64_t plane_s = batch * m * k, plane_t = batch * k * n;
  const void* kern = (const void*)k_gemm_lowp_wide<KIND, BM, BN, NWM, NWN, SWM, SWN>;
  const TailSplit sp = tail_split(nblocks, resident_blocks(kern, 64 * NWM * NWN));
  hipLaunchKernelGGL((k_gemm_lowp_wide<KIND, BM, BN, NWM, NWN, SWM, SWN>), dim3((unsigned)(sp.n_big + sp.n_small)),
                     dim3(64 * NWM * NWN), 0, stream, S, T, P, (int)m, (int)n, (int)k, plane_s, plane_t, eS, eT,
                     tiles_n, tiles_per_leaf, sp.n_big, sp.n_small);
}

template <int KIND, int BM>
void launch_split(int64_t nblocks, hipStream_t stream, const uint16_t* S, const uint16_t* T, float* P, int64_t m,
                  int64_t n, int64_t k, int64_t plane_s, int64_t plane_t, const int32_t* eS, const int32_t* eT,
                  int tiles_n, int tiles_per_leaf) {
  const TailSplit sp = tail_split(nblocks, resident_blocks((const void*)k_gemm_lowp_split<KIND, BM>, 256));
  hipLaunchKernelGGL((k_gemm_lowp_split<KIND, BM>), dim3((unsigned)(sp.n_big + sp.n_small)), dim3(256), 0, stream,
                     S, T, P, (int)m, (int)n, (int)k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf, sp.n_big,
                     sp.n_small);
}

template <int KIND>
hipError_t launch_lowp(const uint16_t* S, const uint16_t* T, float* P, int64_t m, int64_t n, int64_t k,
                       int64_t batch, int tile, const int32_t* eS, const int32_t* eT,
                       hipStream_t stream) {
  if (batch == 0 || m == 0 || n == 0) return hipSuccess;
  if (m % tile || n % tile || k % 32 || (tile != 32 && tile != 64 && tile != 96 && tile != 128))
    return hipErrorInvalidValue;
  const int tiles_n = (int)(n / tile), tiles_per_leaf = (int)((m / tile) * tiles_n);
  const int64_t nblocks = batch * tiles_per_leaf;
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  const int64_t plane_s = batch * m * k, plane_t = batch * k * n;
  const dim3 grid((unsigned)nblocks), block(256);
  // 128-tile plans whose leaves allow it run on the larger tiles (same bits)
  bool wide = false;
  if constexpr (KIND == tiles::LOWP_F16S) {
    if ((wide = tile == 128 && m % 256 == 0 && n % 256 == 0))
      launch_wide<KIND, 256, 256, 2, 4, 2, 4>(stream, S, T, P, m, n, k, batch, eS, eT);
  } else {
    if ((wide = tile == 128 && n % 256 == 0))
      launch_wide<KIND, 128, 256, 4, 2, 2, 4>(stream, S, T, P, m, n, k, batch, eS, eT);
  }
  if (wide)
    ;
  else if (tile == 128)
    launch_split<KIND, 128>(nblocks, stream, S, T, P, m, n, k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf);
  else if (tile == 64)
    launch_split<KIND, 64>(nblocks, stream, S, T, P, m, n, k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf);
  else if (tile == 96)
    hipLaunchKernelGGL((k_gemm_lowp<KIND, 96, 96>), grid, block, 0, stream, S, T, P, (int)m, (int)n,
                       (int)k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf, nblocks);
  else
    hipLaunchKernelGGL((k_gemm_lowp<KIND, 32, 32>), grid, block, 0, stream, S, T, P, (int)m, (int)n,
                       (int)k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf, nblocks);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_bf16x3(const uint16_t* S, const uint16_t* T, float* P, int64_t m, int64_t n,
                              int64_t k, int64_t batch, int tile, hipStream_t stream) {
  return launch_lowp<tiles::LOWP_BF16X3>(S, T, P, m, n, k, batch, tile, nullptr, nullptr, stream);
}

hipError_t launch_gemm_f16s(const uint16_t* S, const uint16_t* T, float* P, int64_t m, int64_t n,
                            int64_t k, int64_t batch, int tile, const int32_t* eS, const int32_t* eT,
                            hipStream_t stream) {
  if (!eS || !eT) return hipErrorInvalidValue;
  return launch_lowp<tiles::LOWP_F16S>(S, T, P, m, n, k, batch, tile, eS, eT, stream);
}

}  // namespace rbc
