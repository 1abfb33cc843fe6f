// Leaf products P_l = S_l T_l (the standard product at the bottom of the
// recursion, F-hat^(0) in Section 2.1.1) for every leaf of a plan in one
// batched launch, on CDNA4 matrix cores.
//
// f32: v_mfma_f32_16x16x4_f32.  A workgroup of 4 wavefronts computes a BM x BN
// tile (BM = BN = 64 or 128), each wavefront a (BM/2) x (BN/2) quarter as a
// grid of 16x16 MFMA tiles.  K advances in slabs (16 for 128-tiles; 32 for
// 64-tiles when K is a multiple of 32, else 16) through two LDS buffers: a
// slab held in registers is written to one buffer, one barrier, then the next
// slab's global loads are issued and stay in flight while the MFMAs consume
// the buffer.  Both slabs keep their memory layout in LDS (16-byte stores):
// the k order inside each group of 16 is permuted identically for both
// operands so that an S operand is one 16-byte LDS read per four MFMA steps;
// S rows are padded to BK + 4 words and T rows to BN + 4, which spreads each
// read over all banks.  The slab depth does not change any product's bits
// (the MFMA chain runs over the same k order).
//
// Workgroups are dispatched round robin over the 8 XCDs; block ids are
// remapped so that the tiles of one leaf run on the same XCD and share its L2.
// 128-tile launches run whole rounds of the resident grid as 128-tiles and a
// partial last round as 64-tiles (split_tail): at N = 4096, Q = 3 (5488 tiles
// on 768 resident workgroups) that took the leaf stage from 0.86 to 0.78 ms,
// with bitwise the same products.
//
// f64: v_mfma_f64_16x16x4_f64, one wavefront per 16x16 output tile, operands
// read straight from global memory (small leaves; latency bound).
#include <hip/hip_runtime.h>

#include "tile_f32.hpp"
#include "leaf_scatter.hpp"
#include "occupancy.hpp"

namespace rbc {
namespace {

using tiles::doublex4;
using tiles::F32Tile;

// MINB workgroups per CU (register cap), EPI epilogue passes (LDS cap): chosen by
// timing on 343 leaves of 512^3 -- 128 x 128 x 16 at 3 per CU with a 4-pass
// epilogue (37 KB of LDS) ran 0.72 ms against 0.88 ms for 128 x 128 x 32 at
// 1 per CU with a one-pass epilogue (69 KB of LDS: two per CU).
// 128-tiles with the last partial round as 64-tiles (split_tail).
constexpr int kSmem128 = F32Tile<128, 128, 16, 4>::SMEM, kSmem64 = F32Tile<64, 64, 32, 2>::SMEM;
__global__ __launch_bounds__(256, 3) void k_gemm_f32_128(const float* __restrict__ S, const float* __restrict__ T,
                                                         float* __restrict__ P, int m, int n, int k, int tiles_n,
                                                         int tiles_per_leaf, int64_t n_big, int64_t n_small) {
  __shared__ __attribute__((aligned(16))) float smem[kSmem128 > kSmem64 ? kSmem128 : kSmem64];
  int64_t bid;
  if (tiles::split_tail(blockIdx.x, n_big, n_small, tiles_n, tiles_per_leaf, &bid))
    tiles::gemm_f32_tile<128, 128, 16, 4>(S, T, P, m, n, k, tiles_n, tiles_per_leaf, bid, smem);
  else if (k % 32 == 0)
    tiles::gemm_f32_tile<64, 64, 32, 2>(S, T, P, m, n, k, 2 * tiles_n, 4 * tiles_per_leaf, bid, smem);
  else
    tiles::gemm_f32_tile<64, 64, 16, 2>(S, T, P, m, n, k, 2 * tiles_n, 4 * tiles_per_leaf, bid, smem);
}

// The same tiles with the operands gathered while they are loaded (LeafGather).
// BUF: 128-tiles through buffer loads (gemm_f32_gathered_tile; parents under 2 GiB).
// SCAT: the deepest level's scatter follows each tile (LeafScatter).
template <bool BUF, bool SCAT>
__global__ __launch_bounds__(256, 3) void k_gemm_f32_128_gathered(const LeafGather g, const LeafScatter ls,
                                                                  float* __restrict__ P, int m, int n, int k,
                                                                  int tiles_n, int tiles_per_leaf, int64_t n_big,
                                                                  int64_t n_small) {
  __shared__ __attribute__((aligned(16))) float smem[kSmem128 > kSmem64 ? kSmem128 : kSmem64];
  __shared__ int32_t flags[4];
  int64_t bid;
  if (tiles::split_tail(blockIdx.x, n_big, n_small, tiles_n, tiles_per_leaf, &bid)) {
    if constexpr (BUF)
      tiles::gemm_f32_gathered_tile<128, 128, 16, 4>(&g, P, m, n, k, tiles_n, tiles_per_leaf, bid, smem);
    else
      tiles::gemm_f32_tile<128, 128, 16, 4, true>(g.A, g.B, P, m, n, k, tiles_n, tiles_per_leaf, bid, smem, &g);
    if constexpr (SCAT) {
      const int64_t leaf = bid / tiles_per_leaf;
      const int t = (int)(bid - leaf * tiles_per_leaf);
      tiles::leaf_scatter_tile<128, 128>(ls, P, m, n, g.R, leaf, t / tiles_n, t % tiles_n, flags);
    }
    return;
  }
  if constexpr (BUF)  // the quarter tiles through buffer loads as well (0.773 -> 0.768 ms at N = 4096, Q = 3)
    tiles::gemm_f32_gathered_tile<64, 64, 16, 2>(&g, P, m, n, k, 2 * tiles_n, 4 * tiles_per_leaf, bid, smem);
  else if (k % 32 == 0)
    tiles::gemm_f32_tile<64, 64, 32, 2, true>(g.A, g.B, P, m, n, k, 2 * tiles_n, 4 * tiles_per_leaf, bid, smem,
                                              &g);
  else
    tiles::gemm_f32_tile<64, 64, 16, 2, true>(g.A, g.B, P, m, n, k, 2 * tiles_n, 4 * tiles_per_leaf, bid, smem,
                                              &g);
  if constexpr (SCAT) {
    const int64_t leaf = bid / (4 * tiles_per_leaf);
    const int t = (int)(bid - leaf * 4 * tiles_per_leaf);
    tiles::leaf_scatter_tile<64, 64>(ls, P, m, n, g.R, leaf, t / (2 * tiles_n), t % (2 * tiles_n), flags);
  }
}

template <int BK, int MINB, bool SCAT>
__global__ __launch_bounds__(256, MINB) void k_gemm_f32_64_gathered(const LeafGather g, const LeafScatter ls,
                                                                    float* __restrict__ P, int m, int n, int k,
                                                                    int tiles_n, int tiles_per_leaf,
                                                                    int64_t nblocks) {
  __shared__ __attribute__((aligned(16))) float smem[F32Tile<64, 64, BK, 2>::SMEM];
  __shared__ int32_t flags[1];
  const int64_t bid = tiles::xcd_remap(blockIdx.x, nblocks);
  tiles::gemm_f32_tile<64, 64, BK, 2, true>(g.A, g.B, P, m, n, k, tiles_n, tiles_per_leaf, bid, smem, &g);
  if constexpr (SCAT) {
    const int64_t leaf = bid / tiles_per_leaf;
    const int t = (int)(bid - leaf * tiles_per_leaf);
    tiles::leaf_scatter_tile<64, 64>(ls, P, m, n, g.R, leaf, t / tiles_n, t % tiles_n, flags);
  }
}

// Zero n words (the leaf scatter's counters, before its launch).
__global__ __launch_bounds__(256) void k_zero_i32(int32_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0;
}

template <int BM, int BN, int BK, int MINB, int EPI>
__global__ __launch_bounds__(256, MINB) void k_gemm_f32(const float* __restrict__ S,
                                                        const float* __restrict__ T, float* __restrict__ P,
                                                        int m, int n, int k, int tiles_n,
                                                        int tiles_per_leaf, int64_t nblocks) {
  __shared__ __attribute__((aligned(16))) float smem[F32Tile<BM, BN, BK, EPI>::SMEM];
  tiles::gemm_f32_tile<BM, BN, BK, EPI>(S, T, P, m, n, k, tiles_n, tiles_per_leaf,
                                        tiles::xcd_remap(blockIdx.x, nblocks), smem);
}

__global__ __launch_bounds__(256) void k_gemm_f64(const double* __restrict__ S,
                                                  const double* __restrict__ T,
                                                  double* __restrict__ P, int m, int n, int k,
                                                  int tiles_n, int tiles_per_leaf, int64_t ntiles) {
  const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= ntiles) return;  // whole wavefront
  const int lane = threadIdx.x & 63;
  const int64_t leaf = tile / tiles_per_leaf;
  const int t = (int)(tile - leaf * tiles_per_leaf);
  const int tm = t / tiles_n, tn = t - (t / tiles_n) * tiles_n;
  const double* Sl = S + leaf * (int64_t)m * k + (int64_t)(tm * 16 + (lane & 15)) * k + (lane >> 4);
  const double* Tl = T + leaf * (int64_t)k * n + (int64_t)(lane >> 4) * n + tn * 16 + (lane & 15);
  doublex4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < k; k0 += 4) {
    const double a = Sl[k0];
    const double b = Tl[(int64_t)k0 * n];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  // D layout of the f64 16x16 MFMA: lane holds column (lane & 15), rows (lane >> 4) + 4 v.
  double* Pl = P + leaf * (int64_t)m * n + (int64_t)(tm * 16) * n + tn * 16;
#pragma unroll
  for (int v = 0; v < 4; ++v) Pl[(int64_t)((lane >> 4) + 4 * v) * n + (lane & 15)] = acc[v];
}

// Leaves of any size (plans with exact blocks, where the recursion's blocks are
// not padded to the tile): one wavefront per 16 x 16 output tile, operands read
// straight from global memory, reads outside the leaf return zero and writes
// outside it are dropped.  Small leaves only (latency bound).
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_masked(const T* __restrict__ S, const T* __restrict__ Tm,
                                                     T* __restrict__ P, int m, int n, int k, int tiles_n,
                                                     int tiles_per_leaf, int64_t ntiles) {
  const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= ntiles) return;  // whole wavefront
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int64_t leaf = tile / tiles_per_leaf;
  const int t = (int)(tile - leaf * tiles_per_leaf);
  const int tm = t / tiles_n, tn = t - (t / tiles_n) * tiles_n;
  const int row = tm * 16 + lr, col = tn * 16 + lr;
  const T* Sl = S + leaf * (int64_t)m * k + (int64_t)row * k;
  const T* Tl = Tm + leaf * (int64_t)k * n + col;
  typedef T Tx4 __attribute__((ext_vector_type(4)));
  Tx4 acc = {T(0), T(0), T(0), T(0)};
  for (int k0 = 0; k0 < k; k0 += 4) {
    const int kk = k0 + lg;  // lane group lg carries k = k0 + lg
    const T a = (row < m && kk < k) ? Sl[kk] : T(0);
    const T b = (col < n && kk < k) ? Tl[(int64_t)kk * n] : T(0);
    if constexpr (sizeof(T) == 8)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    else
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
  // D layout: lane holds column lane & 15; rows lg + 4 v (f64), 4 lg + v (f32)
  T* Pl = P + leaf * (int64_t)m * n;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = tm * 16 + (sizeof(T) == 8 ? lg + 4 * v : 4 * lg + v);
    if (r < m && col < n) Pl[(int64_t)r * n + col] = acc[v];
  }
}

}  // namespace

template <typename T>
static hipError_t launch_masked(const T* S, const T* Tm, T* P, int64_t m, int64_t n, int64_t k, int64_t batch,
                                hipStream_t stream) {
  if (batch == 0 || m == 0 || n == 0) return hipSuccess;
  if (m > (1 << 30) || n > (1 << 30) || k > (1 << 30)) return hipErrorInvalidValue;
  const int tiles_n = (int)((n + 15) / 16), tiles_per_leaf = (int)(((m + 15) / 16) * tiles_n);
  const int64_t ntiles = batch * tiles_per_leaf;
  const int64_t nblocks = (ntiles + 3) / 4;
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gemm_masked<T>, dim3((unsigned)nblocks), dim3(256), 0, stream, S, Tm, P, (int)m, (int)n,
                     (int)k, tiles_n, tiles_per_leaf, ntiles);
  return hipGetLastError();
}

hipError_t launch_gemm_f32_masked(const float* S, const float* T, float* P, int64_t m, int64_t n, int64_t k,
                                  int64_t batch, hipStream_t stream) {
  return launch_masked<float>(S, T, P, m, n, k, batch, stream);
}

hipError_t launch_gemm_f64_masked(const double* S, const double* T, double* P, int64_t m, int64_t n, int64_t k,
                                  int64_t batch, hipStream_t stream) {
  return launch_masked<double>(S, T, P, m, n, k, batch, stream);
}

hipError_t launch_gemm_f32(const float* S, const float* T, float* P, int64_t m, int64_t n, int64_t k,
                           int64_t batch, int tile, hipStream_t stream) {
  if (batch == 0 || m == 0 || n == 0) return hipSuccess;
  if (m % tile || n % tile || k % 16 || (tile != 64 && tile != 128)) return hipErrorInvalidValue;
  const bool deep = k % 32 == 0;  // 64-tiles: K slabs of 32 when K allows, else 16
  const int tiles_n = (int)(n / tile), tiles_per_leaf = (int)((m / tile) * tiles_n);
  const int64_t nblocks = batch * tiles_per_leaf;
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nblocks), block(256);
  if (tile == 128) {
    const TailSplit sp = tail_split(nblocks, resident_blocks((const void*)k_gemm_f32_128, 256));
    hipLaunchKernelGGL(k_gemm_f32_128, dim3((unsigned)(sp.n_big + sp.n_small)), block, 0, stream, S, T, P, (int)m,
                       (int)n, (int)k, tiles_n, tiles_per_leaf, sp.n_big, sp.n_small);
  } else if (deep)
    hipLaunchKernelGGL((k_gemm_f32<64, 64, 32, 4, 2>), grid, block, 0, stream, S, T, P, (int)m, (int)n,
                       (int)k, tiles_n, tiles_per_leaf, nblocks);
  else
    hipLaunchKernelGGL((k_gemm_f32<64, 64, 16, 8, 2>), grid, block, 0, stream, S, T, P, (int)m, (int)n,
                       (int)k, tiles_n, tiles_per_leaf, nblocks);
  return hipGetLastError();
}

template <bool SCAT>
static hipError_t launch_gathered(const LeafGather& g, const LeafScatter& ls, float* P, int64_t m, int64_t n,
                                  int64_t k, int tile, int64_t nblocks, hipStream_t stream) {
  const int tiles_n = (int)(n / tile), tiles_per_leaf = (int)((m / tile) * tiles_n);
  const dim3 block(256);
  if (tile == 128) {
    // buffer loads address a parent with 32-bit byte offsets
    const bool buf = g.a_batch < (int64_t(1) << 29) && g.b_batch < (int64_t(1) << 29);
    const void* kern = buf ? (const void*)k_gemm_f32_128_gathered<true, SCAT>
                           : (const void*)k_gemm_f32_128_gathered<false, SCAT>;
    const TailSplit sp = tail_split(nblocks, resident_blocks(kern, 256));
    if (buf)
      hipLaunchKernelGGL((k_gemm_f32_128_gathered<true, SCAT>), dim3((unsigned)(sp.n_big + sp.n_small)), block, 0,
                         stream, g, ls, P, (int)m, (int)n, (int)k, tiles_n, tiles_per_leaf, sp.n_big, sp.n_small);
    else
      hipLaunchKernelGGL((k_gemm_f32_128_gathered<false, SCAT>), dim3((unsigned)(sp.n_big + sp.n_small)), block, 0,
                         stream, g, ls, P, (int)m, (int)n, (int)k, tiles_n, tiles_per_leaf, sp.n_big, sp.n_small);
  } else if (k % 32 == 0)
    hipLaunchKernelGGL((k_gemm_f32_64_gathered<32, 4, SCAT>), dim3((unsigned)nblocks), block, 0, stream, g, ls, P,
                       (int)m, (int)n, (int)k, tiles_n, tiles_per_leaf, nblocks);
  else
    hipLaunchKernelGGL((k_gemm_f32_64_gathered<16, 4, SCAT>), dim3((unsigned)nblocks), block, 0, stream, g, ls, P,
                       (int)m, (int)n, (int)k, tiles_n, tiles_per_leaf, nblocks);
  return hipGetLastError();
}

hipError_t launch_gemm_f32_gathered(const LeafGather& g, float* P, int64_t m, int64_t n, int64_t k,
                                    int64_t batch, int tile, hipStream_t stream, const LeafScatter* ls) {
  if (batch == 0 || m == 0 || n == 0) return hipSuccess;
  if (m % tile || n % tile || k % 16 || (tile != 64 && tile != 128)) return hipErrorInvalidValue;
  if (!g.A || !g.B || !g.la.tab || !g.lb.tab || g.R < 1 || batch % g.R) return hipErrorInvalidValue;
  const int64_t nblocks = batch * (m / tile) * (n / tile);
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  if (!ls) return launch_gathered<false>(g, LeafScatter{}, P, m, n, k, tile, nblocks, stream);
  if (!ls->out || !ls->cnt || !ls->lw.tab || ls->br < 1 || ls->bc < 1 || ls->br > kMaxB || ls->bc > kMaxB)
    return hipErrorInvalidValue;
  const int64_t n_cnt = batch / g.R * (m / 64) * (n / 64);
  const int64_t zb = (n_cnt + 255) / 256;
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)(zb < 1024 ? zb : 1024)), dim3(256), 0, stream, ls->cnt, n_cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_gathered<true>(g, *ls, P, m, n, k, tile, nblocks, stream);
}

hipError_t launch_gemm_f64(const double* S, const double* T, double* P, int64_t m, int64_t n,
                           int64_t k, int64_t batch, hipStream_t stream) {
  if (batch == 0 || m == 0 || n == 0) return hipSuccess;
  if (m % 16 || n % 16 || k % 4) return hipErrorInvalidValue;
  const int tiles_n = (int)(n / 16), tiles_per_leaf = (int)((m / 16) * tiles_n);
  const int64_t ntiles = batch * tiles_per_leaf;
  const int64_t nblocks = (ntiles + 3) / 4;
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gemm_f64, dim3((unsigned)nblocks), dim3(256), 0, stream, S, T, P, (int)m,
                     (int)n, (int)k, tiles_n, tiles_per_leaf, ntiles);
  return hipGetLastError();
}

}  // namespace rbc
