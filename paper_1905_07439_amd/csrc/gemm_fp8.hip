// fp8 leaf products with one correction pass on CDNA4 matrix cores (the tile
// is described in tile_fp8.hpp): P = 2^-(eS + eT) (hi hi + (hi lo + lo hi) / 16)
// with S = 2^-eS (hi + lo / 16) and likewise T, every byte an OCP e4m3 value.
// The dropped lo lo term is below 2^-8 relative to |S||T|.
#include <hip/hip_runtime.h>

#include "tile_fp8.hpp"
#include "occupancy.hpp"

namespace rbc {
namespace {

using tiles::Fp8Tile;

template <int BM, int BN>
__global__ __launch_bounds__(256, 2) void k_gemm_fp8c(const uint8_t* __restrict__ S, const uint8_t* __restrict__ T,
                                                   float* __restrict__ P, int m, int n, int k, int64_t plane_s,
                                                   int64_t plane_t, const int32_t* __restrict__ eS,
                                                   const int32_t* __restrict__ eT, int tiles_n,
                                                   int tiles_per_leaf, int64_t nblocks) {
  __shared__ __attribute__((aligned(16))) uint8_t smem[Fp8Tile<BM, BN>::SMEM_BYTES];
  tiles::gemm_fp8c_tile<BM, BN>(S, T, P, m, n, k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf,
                                tiles::xcd_remap(blockIdx.x, nblocks), smem);
}

// 128-tiles with the last partial round as 64-tiles (split_tail; both sizes
// use the same fragment shape, so the products are the same bits).
constexpr int kSmem128 = Fp8Tile<128, 128>::SMEM_BYTES, kSmem64 = Fp8Tile<64, 64>::SMEM_BYTES;
__global__ __launch_bounds__(256, 2) void k_gemm_fp8c_128(const uint8_t* __restrict__ S, const uint8_t* __restrict__ T,
                                                          float* __restrict__ P, int m, int n, int k, int64_t plane_s,
                                                          int64_t plane_t, const int32_t* __restrict__ eS,
                                                          const int32_t* __restrict__ eT, int tiles_n,
                                                          int tiles_per_leaf, int64_t n_big, int64_t n_small) {
  __shared__ __attribute__((aligned(16))) uint8_t smem[kSmem128 > kSmem64 ? kSmem128 : kSmem64];
  int64_t bid;
  if (tiles::split_tail(blockIdx.x, n_big, n_small, tiles_n, tiles_per_leaf, &bid))
    tiles::gemm_fp8c_tile<128, 128>(S, T, P, m, n, k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf, bid, smem);
  else
    tiles::gemm_fp8c_tile<64, 64>(S, T, P, m, n, k, plane_s, plane_t, eS, eT, 2 * tiles_n, 4 * tiles_per_leaf, bid,
                                  smem);
}

template <int TILE>
void launch_tile(dim3 grid, hipStream_t stream, const uint8_t* S, const uint8_t* T, float* P, int64_t m,
                 int64_t n, int64_t k, int64_t plane_s, int64_t plane_t, const int32_t* eS, const int32_t* eT,
                 int tiles_n, int tiles_per_leaf, int64_t nblocks) {
  hipLaunchKernelGGL((k_gemm_fp8c<TILE, TILE>), grid, dim3(256), 0, stream, S, T, P, (int)m, (int)n, (int)k,
                     plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf, nblocks);
}

}  // namespace

hipError_t launch_gemm_fp8c(const uint8_t* S, const uint8_t* T, float* P, int64_t m, int64_t n, int64_t k,
                            int64_t batch, int tile, const int32_t* eS, const int32_t* eT, hipStream_t stream) {
  if (batch == 0 || m == 0 || n == 0) return hipSuccess;
  if (!eS || !eT) return hipErrorInvalidValue;
  if (m % tile || n % tile || k % 64 || (tile != 32 && tile != 64 && tile != 96 && tile != 128))
    return hipErrorInvalidValue;
  const int tiles_n = (int)(n / tile), tiles_per_leaf = (int)((m / tile) * tiles_n);
  const int64_t nblocks = batch * tiles_per_leaf;
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  const int64_t plane_s = batch * m * k, plane_t = batch * k * n;
  const dim3 grid((unsigned)nblocks);
  if (tile == 128) {
    const TailSplit sp = tail_split(nblocks, resident_blocks((const void*)k_gemm_fp8c_128, 256));
    hipLaunchKernelGGL(k_gemm_fp8c_128, dim3((unsigned)(sp.n_big + sp.n_small)), dim3(256), 0, stream, S, T, P,
                       (int)m, (int)n, (int)k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf, sp.n_big,
                       sp.n_small);
  } else if (tile == 96)
    launch_tile<96>(grid, stream, S, T, P, m, n, k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf, nblocks);
  else if (tile == 64)
    launch_tile<64>(grid, stream, S, T, P, m, n, k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf, nblocks);
  else
    launch_tile<32>(grid, stream, S, T, P, m, n, k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf, nblocks);
  return hipGetLastError();
}

}  // namespace rbc
