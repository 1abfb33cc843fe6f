// Reduced-precision leaf products on CDNA4 matrix cores, f32 accumulation.
//
//   bf16x3: P = S_hi T_hi + S_hi T_lo + S_lo T_hi, operands split by the gather
//           (S = S_hi + S_lo, each part rounded to bf16); v_mfma_f32_16x16x32_bf16.
//           The dropped term S_lo T_lo is below 2^-16 relative to |S||T|.
//   f16s:   P = 2^-(eS + eT) (S' T') with S' = rn_f16(2^eS S), T' = rn_f16(2^eT T),
//           one power-of-two scale per leaf operand chosen by the gather so that
//           no value can overflow; v_mfma_f32_16x16x32_f16.  The unscaling is exact.
//
// Tile BM x BN (32, 64 or 128) per workgroup of 4 wavefronts, each a
// (BM/2) x (BN/2) quarter of 16x16 MFMA tiles, K slabs of 32.  Both operands
// are staged k-contiguous in LDS so that every MFMA operand is one 16-byte LDS
// read (8 consecutive k of one row or column): S slabs are already k-contiguous
// in memory; T slabs are transposed on the way into LDS, four k rows at a
// time, so each LDS store writes 8 bytes.  Two LDS buffers: a slab held in
// registers is written to one, one barrier, then the next slab's global loads
// stay in flight while the MFMAs consume the buffer.  Block ids are remapped
// so that one leaf's tiles run on one XCD.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace rbc {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nb) {
  const int64_t per = nb / 8, rem = nb % 8;
  const int64_t xcd = bid % 8, local = bid / 8;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

enum LowpKind { LOWP_BF16X3 = 0, LOWP_F16S = 1 };

template <int KIND>
__device__ __forceinline__ floatx4 mfma16(u32x4 a, u32x4 b, floatx4 c) {
  if constexpr (KIND == LOWP_BF16X3)
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                    c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b),
                                                   c, 0, 0, 0);
}

template <int KIND, int BM, int BN>
__global__ __launch_bounds__(256) void k_gemm_lowp(const uint16_t* __restrict__ S,
                                                   const uint16_t* __restrict__ T,
                                                   float* __restrict__ P, int m, int n, int k,
                                                   int64_t plane_s, int64_t plane_t,
                                                   const int32_t* __restrict__ eS,
                                                   const int32_t* __restrict__ eT, int tiles_n,
                                                   int tiles_per_leaf, int64_t nblocks) {
  constexpr int NP = KIND == LOWP_BF16X3 ? 2 : 1;  // operand planes (hi, lo)
  constexpr int BK = 32;
  constexpr int LDK = BK + 8;  // padded row of 40 halves (80 bytes)
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int A_TOTAL = NP * BM * BK / 8;          // 16-byte chunks of an S slab
  constexpr int A_ITER = (A_TOTAL + 255) / 256;
  constexpr int B_TOTAL = NP * (BK / 4) * (BN / 8);  // 4k x 8n groups of a T slab
  constexpr int B_ITER = (B_TOTAL + 255) / 256;
  __shared__ __attribute__((aligned(16))) uint16_t As[2][NP][BM][LDK];  // [buf][plane][row][k]
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][NP][BN][LDK];  // [buf][plane][col][k]

  const int64_t bid = xcd_remap(blockIdx.x, nblocks);
  const int64_t leaf = bid / tiles_per_leaf;
  const int t = (int)(bid - leaf * tiles_per_leaf);
  const int tm = t / tiles_n, tn = t - (t / tiles_n) * tiles_n;
  const uint16_t* Sl = S + leaf * (int64_t)m * k + (int64_t)tm * BM * k;
  const uint16_t* Tl = T + leaf * (int64_t)k * n + (int64_t)tn * BN;
  float* Pl = P + leaf * (int64_t)m * n + (int64_t)tm * BM * n + (int64_t)tn * BN;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // Per-thread slab sources (threads past a total mirror a valid chunk and do not store).
  const uint16_t* a_src[A_ITER];
#pragma unroll
  for (int i = 0; i < A_ITER; ++i) {
    const int idx = (tid + 256 * i) % A_TOTAL;
    const int pl = idx / (BM * BK / 8), rem = idx % (BM * BK / 8);
    a_src[i] = Sl + pl * plane_s + (int64_t)(rem / (BK / 8)) * k + (rem % (BK / 8)) * 8;
  }
  const uint16_t* b_src[B_ITER];
#pragma unroll
  for (int i = 0; i < B_ITER; ++i) {
    const int idx = (tid + 256 * i) % B_TOTAL;
    const int pl = idx / ((BK / 4) * (BN / 8)), rem = idx % ((BK / 4) * (BN / 8));
    b_src[i] = Tl + pl * plane_t + (int64_t)((rem / (BN / 8)) * 4) * n + (rem % (BN / 8)) * 8;
  }

  // clang vector types (not HIP's uint4 struct) so the staging stays in registers
  u32x4 ra[A_ITER];
  u32x4 rb[B_ITER][4];
#pragma unroll
  for (int i = 0; i < A_ITER; ++i) ra[i] = *reinterpret_cast<const u32x4*>(a_src[i]);
#pragma unroll
  for (int i = 0; i < B_ITER; ++i)
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
    for (int i = 0; i < A_ITER; ++i) {
      const int idx = tid + 256 * i;
      if (A_TOTAL % 256 && idx >= A_TOTAL) break;
      const int pl = idx / (BM * BK / 8), rem = idx % (BM * BK / 8);
      *reinterpret_cast<u32x4*>(&As[cur][pl][rem / (BK / 8)][(rem % (BK / 8)) * 8]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < B_ITER; ++i) {
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
      for (int i = 0; i < A_ITER; ++i) ra[i] = *reinterpret_cast<const u32x4*>(a_src[i] + k1);
#pragma unroll
      for (int i = 0; i < B_ITER; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          rb[i][r] = *reinterpret_cast<const u32x4*>(b_src[i] + (int64_t)(k1 + r) * n);
    }
    u32x4 ah[FM], bh[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
      ah[i] = *reinterpret_cast<const u32x4*>(&As[cur][0][wm * WM + i * 16 + lr][lg * 8]);
#pragma unroll
    for (int j = 0; j < FN; ++j)
      bh[j] = *reinterpret_cast<const u32x4*>(&Bs[cur][0][wn * WN + j * 16 + lr][lg * 8]);
    if constexpr (NP == 2) {
      u32x4 al[FM], bl[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        al[i] = *reinterpret_cast<const u32x4*>(&As[cur][NP - 1][wm * WM + i * 16 + lr][lg * 8]);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        bl[j] = *reinterpret_cast<const u32x4*>(&Bs[cur][NP - 1][wn * WN + j * 16 + lr][lg * 8]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          acc[i][j] = mfma16<KIND>(al[i], bh[j], acc[i][j]);
          acc[i][j] = mfma16<KIND>(ah[i], bl[j], acc[i][j]);
        }
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = mfma16<KIND>(ah[i], bh[j], acc[i][j]);
    cur ^= 1;
  }

  int unscale = 0;
  if constexpr (KIND == LOWP_F16S) unscale = -(eS[leaf] + eT[leaf]);
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wm * WM + i * 16 + lg * 4 + v, col = wn * WN + j * 16 + lr;
        float x = acc[i][j][v];
        if constexpr (KIND == LOWP_F16S) x = ldexpf(x, unscale);
        Pl[(int64_t)row * n + col] = x;
      }
}

template <int KIND>
hipError_t launch_lowp(const uint16_t* S, const uint16_t* T, float* P, int64_t m, int64_t n, int64_t k,
                       int64_t batch, int tile, const int32_t* eS, const int32_t* eT,
                       hipStream_t stream) {
  if (batch == 0 || m == 0 || n == 0) return hipSuccess;
  if (m % tile || n % tile || k % 32 || (tile != 32 && tile != 64 && tile != 128))
    return hipErrorInvalidValue;
  const int tiles_n = (int)(n / tile), tiles_per_leaf = (int)((m / tile) * tiles_n);
  const int64_t nblocks = batch * tiles_per_leaf;
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  const int64_t plane_s = batch * m * k, plane_t = batch * k * n;
  const dim3 grid((unsigned)nblocks), block(256);
  if (tile == 128)
    hipLaunchKernelGGL((k_gemm_lowp<KIND, 128, 128>), grid, block, 0, stream, S, T, P, (int)m, (int)n,
                       (int)k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf, nblocks);
  else if (tile == 64)
    hipLaunchKernelGGL((k_gemm_lowp<KIND, 64, 64>), grid, block, 0, stream, S, T, P, (int)m, (int)n,
                       (int)k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf, nblocks);
  else
    hipLaunchKernelGGL((k_gemm_lowp<KIND, 32, 32>), grid, block, 0, stream, S, T, P, (int)m, (int)n,
                       (int)k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf, nblocks);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_bf16x3(const uint16_t* S, const uint16_t* T, float* P, int64_t m, int64_t n,
                              int64_t k, int64_t batch, int tile, hipStream_t stream) {
  return launch_lowp<LOWP_BF16X3>(S, T, P, m, n, k, batch, tile, nullptr, nullptr, stream);
}

hipError_t launch_gemm_f16s(const uint16_t* S, const uint16_t* T, float* P, int64_t m, int64_t n,
                            int64_t k, int64_t batch, int tile, const int32_t* eS, const int32_t* eT,
                            hipStream_t stream) {
  if (!eS || !eT) return hipErrorInvalidValue;
  return launch_lowp<LOWP_F16S>(S, T, P, m, n, k, batch, tile, eS, eT, stream);
}

}  // namespace rbc
