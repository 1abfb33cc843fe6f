// Split-precision leaf products: P = S_hi T_hi + S_hi T_lo + S_lo T_hi with
// bf16 operands (S = S_hi + S_lo, each part rounded to bf16 by the gather) and
// f32 accumulation, on v_mfma_f32_16x16x32_bf16.  The dropped term
// S_lo T_lo is below 2^-16 relative to |S||T|.
//
// Tile BM x BN (64 or 128) per workgroup of 4 wavefronts, K slabs of 32.
// Both operands are staged k-contiguous in LDS so that every MFMA operand is
// one 16-byte LDS read (8 consecutive k of one row or column): S slabs are
// already k-contiguous in memory; T slabs are transposed on the way into LDS,
// four k rows at a time, so each LDS store writes 8 bytes.  Two LDS buffers:
// a slab held in registers is written to one, one barrier, then the next
// slab's global loads stay in flight while the MFMAs consume the buffer.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace rbc {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nb) {
  const int64_t per = nb / 8, rem = nb % 8;
  const int64_t xcd = bid % 8, local = bid / 8;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

template <int BM, int BN>
__global__ __launch_bounds__(256) void k_gemm_bf16x3(const uint16_t* __restrict__ S,
                                                     const uint16_t* __restrict__ T,
                                                     float* __restrict__ P, int m, int n, int k,
                                                     int64_t plane_s, int64_t plane_t, int tiles_n,
                                                     int tiles_per_leaf, int64_t nblocks) {
  constexpr int BK = 32;
  constexpr int LDK = BK + 8;  // padded row of 40 bf16 (80 bytes)
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int A_CHUNKS = 2 * BM * BK / 8 / 256;  // 16-byte loads per thread (both planes)
  constexpr int B_TOTAL = 2 * (BK / 4) * (BN / 8);           // 4k x 8n groups, both planes
  constexpr int B_GROUPS = (B_TOTAL + 255) / 256;
  __shared__ __attribute__((aligned(16))) uint16_t As[2][2][BM][LDK];  // [buf][plane][row][k]
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][2][BN][LDK];  // [buf][plane][col][k]

  const int64_t bid = xcd_remap(blockIdx.x, nblocks);
  const int64_t leaf = bid / tiles_per_leaf;
  const int t = (int)(bid - leaf * tiles_per_leaf);
  const int tm = t / tiles_n, tn = t - (t / tiles_n) * tiles_n;
  const uint16_t* Sl = S + leaf * (int64_t)m * k + (int64_t)tm * BM * k;
  const uint16_t* Tl = T + leaf * (int64_t)k * n + (int64_t)tn * BN;
  float* Pl = P + leaf * (int64_t)m * n + (int64_t)tm * BM * n + (int64_t)tn * BN;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // Per-thread slab sources.  S: chunk (tid + 256 i) -> plane, row, 8-element k chunk.
  // T: group (tid + 256 i) -> plane, 4 k rows, 8 columns.
  const uint16_t* a_src[A_CHUNKS];
#pragma unroll
  for (int i = 0; i < A_CHUNKS; ++i) {
    const int idx = tid + 256 * i;
    const int pl = idx / (BM * BK / 8), rem = idx % (BM * BK / 8);
    a_src[i] = Sl + pl * plane_s + (int64_t)(rem / (BK / 8)) * k + (rem % (BK / 8)) * 8;
  }
  const uint16_t* b_src[B_GROUPS];
#pragma unroll
  for (int i = 0; i < B_GROUPS; ++i) {
    const int idx = (tid + 256 * i) % B_TOTAL;  // threads past B_TOTAL mirror a valid group
    const int pl = idx / ((BK / 4) * (BN / 8)), rem = idx % ((BK / 4) * (BN / 8));
    b_src[i] = Tl + pl * plane_t + (int64_t)((rem / (BN / 8)) * 4) * n + (rem % (BN / 8)) * 8;
  }

  // clang vector types (not HIP's uint4 struct) so the staging stays in registers
  u32x4 ra[A_CHUNKS];
  u32x4 rb[B_GROUPS][4];
#pragma unroll
  for (int i = 0; i < A_CHUNKS; ++i) ra[i] = *reinterpret_cast<const u32x4*>(a_src[i]);
#pragma unroll
  for (int i = 0; i < B_GROUPS; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) rb[i][r] = *reinterpret_cast<const u32x4*>(b_src[i] + (int64_t)r * n);

  floatx4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int nk = k / BK;
  const int lr = lane & 15, lg = lane >> 4;
  int cur = 0;
  for (int kt = 0; kt < nk; ++kt) {
    // registers -> LDS buffer `cur`; T is transposed so that k is contiguous
#pragma unroll
    for (int i = 0; i < A_CHUNKS; ++i) {
      const int idx = tid + 256 * i;
      const int pl = idx / (BM * BK / 8), rem = idx % (BM * BK / 8);
      *reinterpret_cast<u32x4*>(&As[cur][pl][rem / (BK / 8)][(rem % (BK / 8)) * 8]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < B_GROUPS; ++i) {
      const int idx = tid + 256 * i;
      if (B_TOTAL % 256 && idx >= B_TOTAL) break;
      const int pl = idx / ((BK / 4) * (BN / 8)), rem = idx % ((BK / 4) * (BN / 8));
      const int kg = rem / (BN / 8), cg = rem % (BN / 8);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        // element c of each of the 4 rows: 16-bit halves of 32-bit word c / 2
        const int w = c >> 1, sh = (c & 1) * 16;
        u32x2 v;
        v[0] = ((rb[i][0][w] >> sh) & 0xFFFFu) | (((rb[i][1][w] >> sh) & 0xFFFFu) << 16);
        v[1] = ((rb[i][2][w] >> sh) & 0xFFFFu) | (((rb[i][3][w] >> sh) & 0xFFFFu) << 16);
        *reinterpret_cast<u32x2*>(&Bs[cur][pl][cg * 8 + c][kg * 4]) = v;
      }
    }
    __syncthreads();
    if (kt + 1 < nk) {
      const int k1 = (kt + 1) * BK;
#pragma unroll
      for (int i = 0; i < A_CHUNKS; ++i) ra[i] = *reinterpret_cast<const u32x4*>(a_src[i] + k1);
#pragma unroll
      for (int i = 0; i < B_GROUPS; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          rb[i][r] = *reinterpret_cast<const u32x4*>(b_src[i] + (int64_t)(k1 + r) * n);
    }
    bf16x8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      ah[i] = *reinterpret_cast<const bf16x8*>(&As[cur][0][wm * WM + i * 16 + lr][lg * 8]);
      al[i] = *reinterpret_cast<const bf16x8*>(&As[cur][1][wm * WM + i * 16 + lr][lg * 8]);
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      bh[j] = *reinterpret_cast<const bf16x8*>(&Bs[cur][0][wn * WN + j * 16 + lr][lg * 8]);
      bl[j] = *reinterpret_cast<const bf16x8*>(&Bs[cur][1][wn * WN + j * 16 + lr][lg * 8]);
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
    cur ^= 1;
  }

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wm * WM + i * 16 + lg * 4 + v, col = wn * WN + j * 16 + lr;
        Pl[(int64_t)row * n + col] = acc[i][j][v];
      }
}

}  // namespace

hipError_t launch_gemm_bf16x3(const uint16_t* S, const uint16_t* T, float* P, int64_t m, int64_t n,
                              int64_t k, int64_t batch, int tile, hipStream_t stream) {
  if (batch == 0 || m == 0 || n == 0) return hipSuccess;
  if (m % tile || n % tile || k % 32 || (tile != 64 && tile != 128)) return hipErrorInvalidValue;
  const int tiles_n = (int)(n / tile), tiles_per_leaf = (int)((m / tile) * tiles_n);
  const int64_t nblocks = batch * tiles_per_leaf;
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  const int64_t plane_s = batch * m * k, plane_t = batch * k * n;
  if (tile == 128)
    hipLaunchKernelGGL((k_gemm_bf16x3<128, 128>), dim3((unsigned)nblocks), dim3(256), 0, stream, S, T,
                       P, (int)m, (int)n, (int)k, plane_s, plane_t, tiles_n, tiles_per_leaf, nblocks);
  else
    hipLaunchKernelGGL((k_gemm_bf16x3<64, 64>), dim3((unsigned)nblocks), dim3(256), 0, stream, S, T,
                       P, (int)m, (int)n, (int)k, plane_s, plane_t, tiles_n, tiles_per_leaf, nblocks);
  return hipGetLastError();
}

}  // namespace rbc
