// 16-bit leaf product tiles: bf16 hi+lo (three products) and f16 with per-leaf
// power-of-two scales, on the 16x16x32 matrix-core instructions.
//
#pragma once

#include "gemm_tiles.hpp"

namespace rbc {
namespace tiles {

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

// 16-bit leaf operands: S slabs keep their k-contiguous rows in LDS; T slabs
// keep their n-contiguous rows and every T operand (8 k values of one column)
// is two transposing LDS reads (ds_read_b64_tr_b16): in each group of 16
// lanes, lane s reads 4 halves of k row s / 4 at column offset 4 (s % 4), and
// lane t receives half t % 4 of the reads of lanes 4j + t / 4, j = 0..3, which
// is column t over the 4 k rows.
template <int KIND, int BM, int BN, int BK_ = 32>
struct LowpTile {
  static constexpr int NP = KIND == LOWP_BF16X3 ? 2 : 1, BK = BK_, LDK = BK + 8, LDB = BN + 16;
  static constexpr int A_HALVES = NP * BM * LDK, B_HALVES = NP * BK * LDB;  // one buffer
  static constexpr int SMEM_HALVES = 2 * (A_HALVES + B_HALVES);             // two buffers
};

typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) i16x4 lds_i16x4;

__device__ __forceinline__ u32x2 lds_read_tr16(const uint16_t* p) {
  return __builtin_bit_cast(u32x2, __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4*)(p)));
}

// Output tile `bid` of the batched reduced-precision leaf product; K slabs of
// BK (32 or 64), one MFMA k-step of 32 per 32 of the slab, in k order.
template <int KIND, int BM, int BN, int BK_ = 32>
__device__ __forceinline__ void gemm_lowp_tile(const uint16_t* __restrict__ S,
                                               const uint16_t* __restrict__ T, float* __restrict__ P,
                                               int m, int n, int k, int64_t plane_s, int64_t plane_t,
                                               const int32_t* __restrict__ eS,
                                               const int32_t* __restrict__ eT, int tiles_n,
                                               int tiles_per_leaf, int64_t bid, uint16_t* smem) {
  using Tile = LowpTile<KIND, BM, BN, BK_>;
  static_assert(BK_ % 32 == 0, "slabs of whole MFMA k-steps");
  constexpr int NP = Tile::NP;  // operand planes (hi, lo)
  constexpr int BK = Tile::BK, LDK = Tile::LDK, LDB = Tile::LDB;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int A_TOTAL = NP * BM * BK / 8;  // 16-byte chunks of an S slab
  constexpr int A_ITER = (A_TOTAL + 255) / 256;
  constexpr int B_TOTAL = NP * BK * BN / 8;  // 16-byte chunks of a T slab
  constexpr int B_ITER = (B_TOTAL + 255) / 256;
  uint16_t(*As)[NP][BM][LDK] = reinterpret_cast<uint16_t(*)[NP][BM][LDK]>(smem);  // [buf][plane][row][k]
  uint16_t(*Bs)[NP][BK][LDB] =
      reinterpret_cast<uint16_t(*)[NP][BK][LDB]>(smem + 2 * Tile::A_HALVES);      // [buf][plane][k][col]
  const int64_t leaf = bid / tiles_per_leaf;
  const int t = (int)(bid - leaf * tiles_per_leaf);
  const int tm = t / tiles_n, tn = t - (t / tiles_n) * tiles_n;
  const gbl<const uint16_t>* Sl = global_ptr(S) + leaf * (int64_t)m * k + (int64_t)tm * BM * k;
  const gbl<const uint16_t>* Tl = global_ptr(T) + leaf * (int64_t)k * n + (int64_t)tn * BN;
  gbl<float>* Pl = global_ptr(P) + leaf * (int64_t)m * n + (int64_t)tm * BM * n + (int64_t)tn * BN;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // Per-thread slab sources (threads past a total mirror a valid chunk and do not store).
  const gbl<const uint16_t>* a_src[A_ITER];
#pragma unroll
  for (int i = 0; i < A_ITER; ++i) {
    const int idx = (tid + 256 * i) % A_TOTAL;
    const int pl = idx / (BM * BK / 8), rem = idx % (BM * BK / 8);
    a_src[i] = Sl + pl * plane_s + (int64_t)(rem / (BK / 8)) * k + (rem % (BK / 8)) * 8;
  }
  const gbl<const uint16_t>* b_src[B_ITER];
#pragma unroll
  for (int i = 0; i < B_ITER; ++i) {
    const int idx = (tid + 256 * i) % B_TOTAL;
    const int pl = idx / (BK * BN / 8), rem = idx % (BK * BN / 8);
    b_src[i] = Tl + pl * plane_t + (int64_t)(rem / (BN / 8)) * n + (rem % (BN / 8)) * 8;
  }

  // clang vector types (not HIP's uint4 struct) so the staging stays in registers
  u32x4 ra[A_ITER], rb[B_ITER];
#pragma unroll
  for (int i = 0; i < A_ITER; ++i) ra[i] = *reinterpret_cast<const gbl<const u32x4>*>(a_src[i]);
#pragma unroll
  for (int i = 0; i < B_ITER; ++i) rb[i] = *reinterpret_cast<const gbl<const u32x4>*>(b_src[i]);

  floatx4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int nk = k / BK;
  const int lr = lane & 15, lg = lane >> 4;
  // this lane's part of the transposing T reads: k rows lg * 8 + lr / 4 (+ 4), column offset 4 (lr % 4)
  const int tr_row = lg * 8 + (lr >> 2), tr_col = wn * WN + (lr & 3) * 4;
  int cur = 0;
  for (int kt = 0; kt < nk; ++kt) {
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
      const int pl = idx / (BK * BN / 8), rem = idx % (BK * BN / 8);
      *reinterpret_cast<u32x4*>(&Bs[cur][pl][rem / (BN / 8)][(rem % (BN / 8)) * 8]) = rb[i];
    }
    // the staging registers are free once stored: the next slab's loads go out before the
    // barrier (f16s, 49 leaves of 1024^3: 180 -> 172 us; bf16x3, 10 of 1024 x 1536 x 1536:
    // 193 -> 185 us)
    if (kt + 1 < nk) {
      const int k1 = (kt + 1) * BK;
#pragma unroll
      for (int i = 0; i < A_ITER; ++i) ra[i] = *reinterpret_cast<const gbl<const u32x4>*>(a_src[i] + k1);
#pragma unroll
      for (int i = 0; i < B_ITER; ++i)
        rb[i] = *reinterpret_cast<const gbl<const u32x4>*>(b_src[i] + (int64_t)k1 * n);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK / 32; ++kk) {
      u32x4 ah[FM], bh[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        ah[i] = *reinterpret_cast<const u32x4*>(&As[cur][0][wm * WM + i * 16 + lr][kk * 32 + lg * 8]);
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const u32x2 lo = lds_read_tr16(&Bs[cur][0][kk * 32 + tr_row][tr_col + j * 16]);
        const u32x2 hi = lds_read_tr16(&Bs[cur][0][kk * 32 + tr_row + 4][tr_col + j * 16]);
        bh[j] = u32x4{lo[0], lo[1], hi[0], hi[1]};
      }
      if constexpr (NP == 2) {
        u32x4 al[FM], bl[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
          al[i] = *reinterpret_cast<const u32x4*>(&As[cur][NP - 1][wm * WM + i * 16 + lr][kk * 32 + lg * 8]);
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const u32x2 lo = lds_read_tr16(&Bs[cur][NP - 1][kk * 32 + tr_row][tr_col + j * 16]);
          const u32x2 hi = lds_read_tr16(&Bs[cur][NP - 1][kk * 32 + tr_row + 4][tr_col + j * 16]);
          bl[j] = u32x4{lo[0], lo[1], hi[0], hi[1]};
        }
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
    }
    cur ^= 1;
  }

  int unscale = 0;
  if constexpr (KIND == LOWP_F16S) unscale = -(global_ptr(eS)[leaf] + global_ptr(eT)[leaf]);
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


// The same product on larger workgroup tiles: BM x BN on NWM x NWN wavefronts (64 NWM NWN
// threads), each wavefront a (BM / NWM) x (BN / NWN) block of 16x16x32 MFMA tiles, K
// slabs of 32 through two LDS buffers.  Same instruction and k order as gemm_lowp_tile,
// so the same bits; larger tiles read fewer operand bytes per flop from L2 (49 f16s
// leaves of 1024^3: 128 x 128 on 4 wavefronts 181 us, 256 x 128 on 8 162 us, 256 x 256
// on 16 154 us; bf16x3, 10 leaves of 1024 x 1536^2: 128 x 256 on 8 wavefronts 173 us
// against 177 us).  Larger wavefront blocks read fewer LDS bytes per flop but gain
// little: f16s 256 x 256 on 2 x 4 wavefronts (128 x 64 each, 188 VGPRs) 149.7 us
// against 153.0 on 4 x 4, 128 x 128 each 165 us (spills); bf16x3 on 64 x 128 or
// 128 x 64 per wavefront (one wavefront per SIMD) 219-227 us against 185.
template <int KIND, int BM, int BN, int NWM, int NWN>
struct LowpTileW {
  static constexpr int NP = KIND == LOWP_BF16X3 ? 2 : 1, BK = 32, LDK = BK + 8, LDB = BN + 16;
  static constexpr int A_HALVES = NP * BM * LDK, B_HALVES = NP * BK * LDB;
  static constexpr int SMEM_HALVES = 2 * (A_HALVES + B_HALVES);
};

template <int KIND, int BM, int BN, int NWM, int NWN>
__device__ __forceinline__ void gemm_lowp_tile_w(const uint16_t* __restrict__ S, const uint16_t* __restrict__ T,
                                                 float* __restrict__ P, int m, int n, int k, int64_t plane_s,
                                                 int64_t plane_t, const int32_t* __restrict__ eS,
                                                 const int32_t* __restrict__ eT, int tiles_n, int tiles_per_leaf,
                                                 int64_t bid, uint16_t* smem) {
  using Tile = LowpTileW<KIND, BM, BN, NWM, NWN>;
  constexpr int NT = 64 * NWM * NWN;
  constexpr int NP = Tile::NP, BK = Tile::BK, LDK = Tile::LDK, LDB = Tile::LDB;
  constexpr int WM = BM / NWM, WN = BN / NWN, FM = WM / 16, FN = WN / 16;
  static_assert(FM >= 1 && FN >= 1 && WM % 16 == 0 && WN % 16 == 0, "wavefront tiles of 16 x 16 blocks");
  constexpr int A_TOTAL = NP * BM * BK / 8, A_ITER = (A_TOTAL + NT - 1) / NT;
  constexpr int B_TOTAL = NP * BK * BN / 8, B_ITER = (B_TOTAL + NT - 1) / NT;
  uint16_t(*As)[NP][BM][LDK] = reinterpret_cast<uint16_t(*)[NP][BM][LDK]>(smem);
  uint16_t(*Bs)[NP][BK][LDB] = reinterpret_cast<uint16_t(*)[NP][BK][LDB]>(smem + 2 * Tile::A_HALVES);
  const int64_t leaf = bid / tiles_per_leaf;
  const int t = (int)(bid - leaf * tiles_per_leaf);
  const int tm = t / tiles_n, tn = t - (t / tiles_n) * tiles_n;
  const gbl<const uint16_t>* Sl = global_ptr(S) + leaf * (int64_t)m * k + (int64_t)tm * BM * k;
  const gbl<const uint16_t>* Tl = global_ptr(T) + leaf * (int64_t)k * n + (int64_t)tn * BN;
  gbl<float>* Pl = global_ptr(P) + leaf * (int64_t)m * n + (int64_t)tm * BM * n + (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / NWN, wn = wave % NWN;
  const gbl<const uint16_t>* a_src[A_ITER];
#pragma unroll
  for (int i = 0; i < A_ITER; ++i) {
    const int idx = (tid + NT * i) % A_TOTAL;
    const int pl = idx / (BM * BK / 8), rem = idx % (BM * BK / 8);
    a_src[i] = Sl + pl * plane_s + (int64_t)(rem / (BK / 8)) * k + (rem % (BK / 8)) * 8;
  }
  const gbl<const uint16_t>* b_src[B_ITER];
#pragma unroll
  for (int i = 0; i < B_ITER; ++i) {
    const int idx = (tid + NT * i) % B_TOTAL;
    const int pl = idx / (BK * BN / 8), rem = idx % (BK * BN / 8);
    b_src[i] = Tl + pl * plane_t + (int64_t)(rem / (BN / 8)) * n + (rem % (BN / 8)) * 8;
  }
  u32x4 ra[A_ITER], rb[B_ITER];
#pragma unroll
  for (int i = 0; i < A_ITER; ++i) ra[i] = *reinterpret_cast<const gbl<const u32x4>*>(a_src[i]);
#pragma unroll
  for (int i = 0; i < B_ITER; ++i) rb[i] = *reinterpret_cast<const gbl<const u32x4>*>(b_src[i]);
  floatx4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int nk = k / BK;
  const int lr = lane & 15, lg = lane >> 4;
  const int tr_row = lg * 8 + (lr >> 2), tr_col = wn * WN + (lr & 3) * 4;
  int cur = 0;
  for (int kt = 0; kt < nk; ++kt) {
#pragma unroll
    for (int i = 0; i < A_ITER; ++i) {
      const int idx = tid + NT * i;
      if (A_TOTAL % NT && idx >= A_TOTAL) break;
      const int pl = idx / (BM * BK / 8), rem = idx % (BM * BK / 8);
      *reinterpret_cast<u32x4*>(&As[cur][pl][rem / (BK / 8)][(rem % (BK / 8)) * 8]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < B_ITER; ++i) {
      const int idx = tid + NT * i;
      if (B_TOTAL % NT && idx >= B_TOTAL) break;
      const int pl = idx / (BK * BN / 8), rem = idx % (BK * BN / 8);
      *reinterpret_cast<u32x4*>(&Bs[cur][pl][rem / (BN / 8)][(rem % (BN / 8)) * 8]) = rb[i];
    }
    if (kt + 1 < nk) {
      const int k1 = (kt + 1) * BK;
#pragma unroll
      for (int i = 0; i < A_ITER; ++i) ra[i] = *reinterpret_cast<const gbl<const u32x4>*>(a_src[i] + k1);
#pragma unroll
      for (int i = 0; i < B_ITER; ++i)
        rb[i] = *reinterpret_cast<const gbl<const u32x4>*>(b_src[i] + (int64_t)k1 * n);
    }
    __syncthreads();
    u32x4 ah[FM], bh[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) ah[i] = *reinterpret_cast<const u32x4*>(&As[cur][0][wm * WM + i * 16 + lr][lg * 8]);
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const u32x2 lo = lds_read_tr16(&Bs[cur][0][tr_row][tr_col + j * 16]);
      const u32x2 hi = lds_read_tr16(&Bs[cur][0][tr_row + 4][tr_col + j * 16]);
      bh[j] = u32x4{lo[0], lo[1], hi[0], hi[1]};
    }
    if constexpr (NP == 2) {
      u32x4 al[FM], bl[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        al[i] = *reinterpret_cast<const u32x4*>(&As[cur][1][wm * WM + i * 16 + lr][lg * 8]);
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const u32x2 lo = lds_read_tr16(&Bs[cur][1][tr_row][tr_col + j * 16]);
        const u32x2 hi = lds_read_tr16(&Bs[cur][1][tr_row + 4][tr_col + j * 16]);
        bl[j] = u32x4{lo[0], lo[1], hi[0], hi[1]};
      }
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
  if constexpr (KIND == LOWP_F16S) unscale = -(global_ptr(eS)[leaf] + global_ptr(eT)[leaf]);
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

}  // namespace tiles
}  // namespace rbc

