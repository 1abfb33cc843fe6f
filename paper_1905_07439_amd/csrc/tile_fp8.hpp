// fp8 (OCP e4m3) leaf product tiles with one correction pass.
//
#pragma once

#include "gemm_tiles.hpp"

namespace rbc {
namespace tiles {

// ---- fp8 (OCP e4m3) leaves with one correction pass ------------------------
//
// S and T hold a hi plane and a lo plane of bytes (lo scaled by 16).  Per
// output: acc = sum hi_S hi_T and cor = sum (hi_S lo_T + lo_S hi_T), both f32,
// on fp8 matrix-core instructions; P = 2^-(eS + eT) (acc + cor / 16).  K
// advances in slabs of 64 bytes.  Both slabs are copied to LDS as they lie in
// memory (S rows k-contiguous, T rows n-contiguous), in 16-byte chunks.  T
// operands are read with the transposing LDS load ds_read_b64_tr_b8: in each
// group of 16 lanes, lane s reads 8 bytes of k row s / 2 at column offset
// 8 (s % 2), and lane t receives byte t % 8 of the reads of lanes 2j + t / 8,
// j = 0..7, which is column t over the 8 k rows.
//
// Tiles of 64 and 128 use v_mfma_scale_f32_32x32x64_f8f6f4 with unit scales
// (the full fp8 rate of CDNA4): per wavefront 32 x 32 fragments, lane l holds
// row (A) or column (B) l % 32 and the 32 consecutive k of group l / 32
// (two 16-byte LDS reads of S; four transposing reads of T), and result v of
// lane l is row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32.  Tiles of 32
// and 96 (wavefront quarters of 16 and 48 rows) use v_mfma_f32_16x16x32_fp8_fp8:
// lane l holds row / column l % 16 and the 8 k of group l / 16.
template <int BM, int BN>
struct Fp8Tile {
  static constexpr bool WIDE = BM % 64 == 0 && BN % 64 == 0;  // 32 x 32 x 64 fragments
  // S rows padded so that eight lanes' 16-byte reads (wide) or sixteen lanes'
  // 8-byte reads (narrow) of consecutive rows hit distinct banks
  static constexpr int BK = 64, LDK = WIDE ? BK + 16 : BK + 8, LDB = BN + 16;
  static constexpr int A_BYTES = 2 * BM * LDK, B_BYTES = 2 * BK * LDB;  // one buffer, both planes
  static constexpr int SMEM_BYTES = 2 * (A_BYTES + B_BYTES);            // two buffers
};

typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ floatx16 mfma_fp8_32(i32x8 a, i32x8 b, floatx16 c) {
  // operand formats 0 (e4m3), scales 127 (E8M0 2^0)
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}

__device__ __forceinline__ floatx4 mfma_fp8(u32x2 a, u32x2 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(__builtin_bit_cast(long, a), __builtin_bit_cast(long, b), c,
                                                     0, 0, 0);
}

typedef int i32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) i32x2 lds_i32x2;

__device__ __forceinline__ u32x2 lds_read_tr8(const uint8_t* p) {
  return __builtin_bit_cast(u32x2, __builtin_amdgcn_ds_read_tr8_b64_v2i32((lds_i32x2*)(p)));
}

template <int BM, int BN>
__device__ __forceinline__ void gemm_fp8c_tile16(const uint8_t* __restrict__ S, const uint8_t* __restrict__ T,
                                               float* __restrict__ P, int m, int n, int k, int64_t plane_s,
                                               int64_t plane_t, const int32_t* __restrict__ eS,
                                               const int32_t* __restrict__ eT, int tiles_n, int tiles_per_leaf,
                                               int64_t bid, uint8_t* smem) {
  using Tile = Fp8Tile<BM, BN>;
  constexpr int BK = Tile::BK, LDK = Tile::LDK, LDB = Tile::LDB;
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
  constexpr int A_TOTAL = 2 * BM * (BK / 16);  // 16-byte chunks of an S slab (both planes)
  constexpr int A_ITER = (A_TOTAL + 255) / 256;
  constexpr int B_TOTAL = 2 * BK * (BN / 16);  // 16-byte chunks of a T slab (both planes)
  constexpr int B_ITER = (B_TOTAL + 255) / 256;
  // [buf][plane][row][k] and [buf][plane][k][col]
  uint8_t(*As)[2][BM][LDK] = reinterpret_cast<uint8_t(*)[2][BM][LDK]>(smem);
  uint8_t(*Bs)[2][BK][LDB] = reinterpret_cast<uint8_t(*)[2][BK][LDB]>(smem + 2 * Tile::A_BYTES);
  const int64_t leaf = bid / tiles_per_leaf;
  const int t = (int)(bid - leaf * tiles_per_leaf);
  const int tm = t / tiles_n, tn = t - (t / tiles_n) * tiles_n;
  const gbl<const uint8_t>* Sl = global_ptr(S) + leaf * (int64_t)m * k + (int64_t)tm * BM * k;
  const gbl<const uint8_t>* Tl = global_ptr(T) + leaf * (int64_t)k * n + (int64_t)tn * BN;
  gbl<float>* Pl = global_ptr(P) + leaf * (int64_t)m * n + (int64_t)tm * BM * n + (int64_t)tn * BN;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // Per-thread slab sources (threads past a total mirror a valid chunk and do not store).
  const gbl<const uint8_t>* a_src[A_ITER];
#pragma unroll
  for (int i = 0; i < A_ITER; ++i) {
    const int idx = (tid + 256 * i) % A_TOTAL;
    const int pl = idx / (BM * (BK / 16)), rem = idx % (BM * (BK / 16));
    a_src[i] = Sl + pl * plane_s + (int64_t)(rem / (BK / 16)) * k + (rem % (BK / 16)) * 16;
  }
  const gbl<const uint8_t>* b_src[B_ITER];
#pragma unroll
  for (int i = 0; i < B_ITER; ++i) {
    const int idx = (tid + 256 * i) % B_TOTAL;
    const int pl = idx / (BK * (BN / 16)), rem = idx % (BK * (BN / 16));
    b_src[i] = Tl + pl * plane_t + (int64_t)(rem / (BN / 16)) * n + (rem % (BN / 16)) * 16;
  }

  u32x4 ra[A_ITER], rb[B_ITER];
#pragma unroll
  for (int i = 0; i < A_ITER; ++i) ra[i] = *reinterpret_cast<const gbl<const u32x4>*>(a_src[i]);
#pragma unroll
  for (int i = 0; i < B_ITER; ++i) rb[i] = *reinterpret_cast<const gbl<const u32x4>*>(b_src[i]);

  floatx4 acc[FM][FN], cor[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = cor[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int nk = k / BK;
  const int lr = lane & 15, lg = lane >> 4;
  // this lane's part of a transposing T read: k row lg * 8 + lr / 2, column offset 8 (lr % 2)
  const int tr_row = lg * 8 + (lr >> 1), tr_col = wn * WN + (lr & 1) * 8;
  int cur = 0;
  for (int kt = 0; kt < nk; ++kt) {
#pragma unroll
    for (int i = 0; i < A_ITER; ++i) {
      const int idx = tid + 256 * i;
      if (A_TOTAL % 256 && idx >= A_TOTAL) break;
      const int pl = idx / (BM * (BK / 16)), rem = idx % (BM * (BK / 16));
      *reinterpret_cast<u32x4*>(&As[cur][pl][rem / (BK / 16)][(rem % (BK / 16)) * 16]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < B_ITER; ++i) {
      const int idx = tid + 256 * i;
      if (B_TOTAL % 256 && idx >= B_TOTAL) break;
      const int pl = idx / (BK * (BN / 16)), rem = idx % (BK * (BN / 16));
      *reinterpret_cast<u32x4*>(&Bs[cur][pl][rem / (BN / 16)][(rem % (BN / 16)) * 16]) = rb[i];
    }
    if (kt + 1 < nk) {  // the next slab's loads before the barrier (staging registers are free)
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
      u32x2 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        ah[i] = *reinterpret_cast<const u32x2*>(&As[cur][0][wm * WM + i * 16 + lr][kk * 32 + lg * 8]);
        al[i] = *reinterpret_cast<const u32x2*>(&As[cur][1][wm * WM + i * 16 + lr][kk * 32 + lg * 8]);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        bh[j] = lds_read_tr8(&Bs[cur][0][kk * 32 + tr_row][tr_col + j * 16]);
        bl[j] = lds_read_tr8(&Bs[cur][1][kk * 32 + tr_row][tr_col + j * 16]);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          acc[i][j] = mfma_fp8(ah[i], bh[j], acc[i][j]);
          cor[i][j] = mfma_fp8(ah[i], bl[j], cor[i][j]);
          cor[i][j] = mfma_fp8(al[i], bh[j], cor[i][j]);
        }
    }
    cur ^= 1;
  }

  const int unscale = -(global_ptr(eS)[leaf] + global_ptr(eT)[leaf]);
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wm * WM + i * 16 + lg * 4 + v, col = wn * WN + j * 16 + lr;
        Pl[(int64_t)row * n + col] = ldexpf(acc[i][j][v] + cor[i][j][v] * 0.0625f, unscale);
      }
}

template <int BM, int BN>
__device__ __forceinline__ void gemm_fp8c_tile32(const uint8_t* __restrict__ S, const uint8_t* __restrict__ T,
                                                 float* __restrict__ P, int m, int n, int k, int64_t plane_s,
                                                 int64_t plane_t, const int32_t* __restrict__ eS,
                                                 const int32_t* __restrict__ eT, int tiles_n, int tiles_per_leaf,
                                                 int64_t bid, uint8_t* smem) {
  using Tile = Fp8Tile<BM, BN>;
  static_assert(Tile::WIDE, "32 x 32 fragments need wavefront quarters of 32-multiples");
  constexpr int BK = Tile::BK, LDK = Tile::LDK, LDB = Tile::LDB;
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 32, FN = WN / 32;
  constexpr int A_TOTAL = 2 * BM * (BK / 16);  // 16-byte chunks of an S slab (both planes)
  constexpr int A_ITER = (A_TOTAL + 255) / 256;
  constexpr int B_TOTAL = 2 * BK * (BN / 16);  // 16-byte chunks of a T slab (both planes)
  constexpr int B_ITER = (B_TOTAL + 255) / 256;
  uint8_t(*As)[2][BM][LDK] = reinterpret_cast<uint8_t(*)[2][BM][LDK]>(smem);
  uint8_t(*Bs)[2][BK][LDB] = reinterpret_cast<uint8_t(*)[2][BK][LDB]>(smem + 2 * Tile::A_BYTES);
  const int64_t leaf = bid / tiles_per_leaf;
  const int t = (int)(bid - leaf * tiles_per_leaf);
  const int tm = t / tiles_n, tn = t - (t / tiles_n) * tiles_n;
  const gbl<const uint8_t>* Sl = global_ptr(S) + leaf * (int64_t)m * k + (int64_t)tm * BM * k;
  const gbl<const uint8_t>* Tl = global_ptr(T) + leaf * (int64_t)k * n + (int64_t)tn * BN;
  gbl<float>* Pl = global_ptr(P) + leaf * (int64_t)m * n + (int64_t)tm * BM * n + (int64_t)tn * BN;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const gbl<const uint8_t>* a_src[A_ITER];
#pragma unroll
  for (int i = 0; i < A_ITER; ++i) {
    const int idx = (tid + 256 * i) % A_TOTAL;
    const int pl = idx / (BM * (BK / 16)), rem = idx % (BM * (BK / 16));
    a_src[i] = Sl + pl * plane_s + (int64_t)(rem / (BK / 16)) * k + (rem % (BK / 16)) * 16;
  }
  const gbl<const uint8_t>* b_src[B_ITER];
#pragma unroll
  for (int i = 0; i < B_ITER; ++i) {
    const int idx = (tid + 256 * i) % B_TOTAL;
    const int pl = idx / (BK * (BN / 16)), rem = idx % (BK * (BN / 16));
    b_src[i] = Tl + pl * plane_t + (int64_t)(rem / (BN / 16)) * n + (rem % (BN / 16)) * 16;
  }

  u32x4 ra[A_ITER], rb[B_ITER];
#pragma unroll
  for (int i = 0; i < A_ITER; ++i) ra[i] = *reinterpret_cast<const gbl<const u32x4>*>(a_src[i]);
#pragma unroll
  for (int i = 0; i < B_ITER; ++i) rb[i] = *reinterpret_cast<const gbl<const u32x4>*>(b_src[i]);

  floatx16 acc[FM][FN], cor[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = cor[i][j] = floatx16{};

  const int nk = k / BK;
  const int l32 = lane & 31, kg = (lane >> 5) * 32;  // fragment row / column, k group
  // transposing T reads: 16-lane group G covers columns 16 (G % 2) .. + 15 of the fragment and
  // k group 32 (G / 2); its lane s reads k row s / 2 (+ 8 q) at column offset 8 (s % 2)
  const int G = lane >> 4, s16 = lane & 15;
  const int tr_row = (G >> 1) * 32 + (s16 >> 1), tr_col = wn * WN + (G & 1) * 16 + (s16 & 1) * 8;
  int cur = 0;
  for (int kt = 0; kt < nk; ++kt) {
#pragma unroll
    for (int i = 0; i < A_ITER; ++i) {
      const int idx = tid + 256 * i;
      if (A_TOTAL % 256 && idx >= A_TOTAL) break;
      const int pl = idx / (BM * (BK / 16)), rem = idx % (BM * (BK / 16));
      *reinterpret_cast<u32x4*>(&As[cur][pl][rem / (BK / 16)][(rem % (BK / 16)) * 16]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < B_ITER; ++i) {
      const int idx = tid + 256 * i;
      if (B_TOTAL % 256 && idx >= B_TOTAL) break;
      const int pl = idx / (BK * (BN / 16)), rem = idx % (BK * (BN / 16));
      *reinterpret_cast<u32x4*>(&Bs[cur][pl][rem / (BN / 16)][(rem % (BN / 16)) * 16]) = rb[i];
    }
    if (kt + 1 < nk) {  // the next slab's loads before the barrier (staging registers are free)
      const int k1 = (kt + 1) * BK;
#pragma unroll
      for (int i = 0; i < A_ITER; ++i) ra[i] = *reinterpret_cast<const gbl<const u32x4>*>(a_src[i] + k1);
#pragma unroll
      for (int i = 0; i < B_ITER; ++i)
        rb[i] = *reinterpret_cast<const gbl<const u32x4>*>(b_src[i] + (int64_t)k1 * n);
    }
    __syncthreads();
    i32x8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int row = wm * WM + i * 32 + l32;
      const u32x4 h0 = *reinterpret_cast<const u32x4*>(&As[cur][0][row][kg]);
      const u32x4 h1 = *reinterpret_cast<const u32x4*>(&As[cur][0][row][kg + 16]);
      const u32x4 o0 = *reinterpret_cast<const u32x4*>(&As[cur][1][row][kg]);
      const u32x4 o1 = *reinterpret_cast<const u32x4*>(&As[cur][1][row][kg + 16]);
      ah[i] = __builtin_bit_cast(i32x8, (u32x8{h0[0], h0[1], h0[2], h0[3], h1[0], h1[1], h1[2], h1[3]}));
      al[i] = __builtin_bit_cast(i32x8, (u32x8{o0[0], o0[1], o0[2], o0[3], o1[0], o1[1], o1[2], o1[3]}));
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      u32x2 h[4], o[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        h[q] = lds_read_tr8(&Bs[cur][0][tr_row + 8 * q][tr_col + j * 32]);
        o[q] = lds_read_tr8(&Bs[cur][1][tr_row + 8 * q][tr_col + j * 32]);
      }
      bh[j] = __builtin_bit_cast(i32x8, (u32x8{h[0][0], h[0][1], h[1][0], h[1][1], h[2][0], h[2][1], h[3][0], h[3][1]}));
      bl[j] = __builtin_bit_cast(i32x8, (u32x8{o[0][0], o[0][1], o[1][0], o[1][1], o[2][0], o[2][1], o[3][0], o[3][1]}));
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        acc[i][j] = mfma_fp8_32(ah[i], bh[j], acc[i][j]);
        cor[i][j] = mfma_fp8_32(ah[i], bl[j], cor[i][j]);
        cor[i][j] = mfma_fp8_32(al[i], bh[j], cor[i][j]);
      }
    cur ^= 1;
  }

  const int unscale = -(global_ptr(eS)[leaf] + global_ptr(eT)[leaf]);
  const int rq = (lane >> 5) * 4;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = wm * WM + i * 32 + 8 * (v >> 2) + rq + (v & 3), col = wn * WN + j * 32 + l32;
        Pl[(int64_t)row * n + col] = ldexpf(acc[i][j][v] + cor[i][j][v] * 0.0625f, unscale);
      }
}

// Output tile `bid` of the batched fp8 leaf product (the two fragment shapes above).
template <int BM, int BN>
__device__ __forceinline__ void gemm_fp8c_tile(const uint8_t* __restrict__ S, const uint8_t* __restrict__ T,
                                               float* __restrict__ P, int m, int n, int k, int64_t plane_s,
                                               int64_t plane_t, const int32_t* __restrict__ eS,
                                               const int32_t* __restrict__ eT, int tiles_n, int tiles_per_leaf,
                                               int64_t bid, uint8_t* smem) {
  if constexpr (Fp8Tile<BM, BN>::WIDE)
    gemm_fp8c_tile32<BM, BN>(S, T, P, m, n, k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf, bid, smem);
  else
    gemm_fp8c_tile16<BM, BN>(S, T, P, m, n, k, plane_s, plane_t, eS, eT, tiles_n, tiles_per_leaf, bid, smem);
}

}  // namespace tiles
}  // namespace rbc

