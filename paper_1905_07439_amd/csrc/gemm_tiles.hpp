// Device-side leaf product tiles, shared by the leaf kernels (gemm.hip,
// gemm_lowp.hip) and by the batch engine's persistent kernel (batch.hip).
// Each function computes one output tile given its logical tile index and a
// pointer to the workgroup's LDS block.
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

// EPI: the epilogue parks each wavefront's output quarter in LDS in EPI passes
// of WM / EPI rows, so that the epilogue needs no more LDS than the K loop.
template <int BM, int BN, int BK, int EPI = 1>
struct F32Tile {
  static constexpr int LDA = BK + 4, LDB = BN + 4, WM = BM / 2, WN = BN / 2, LDE = WN + 4;
  static constexpr int A_FLOATS = 2 * BM * LDA, B_FLOATS = 2 * BK * LDB, E_FLOATS = 4 * (WM / EPI) * LDE;
  // LDS floats: two S and two T slab buffers in the K loop, the output quarters in the epilogue
  static constexpr int SMEM = A_FLOATS + B_FLOATS > E_FLOATS ? A_FLOATS + B_FLOATS : E_FLOATS;
};

// The nonzero folded coefficients of product r on one side of a level, in
// row-major sub-block order, with the element offsets of their sub-blocks;
// n counts them (the host admits at most two).
struct GatherSlots {
  float c0, c1;
  int64_t off0, off1;
  int n;
};

__device__ __forceinline__ GatherSlots gather_slots(const SideLevel& L, int br, int bc, int r, int R,
                                                    int64_t row_blk, int64_t col_blk) {
  const gbl<const float>* tab = global_ptr(static_cast<const float*>(L.tab));
  GatherSlots g{0.f, 0.f, 0, 0, 0};
  for (int kr = 0; kr < br; ++kr)
    for (int kc = 0; kc < bc; ++kc) {
      float c = tab[(L.pr[kr] * bc + L.pc[kc]) * R + r];
      if (L.sr[kr] * L.sc[kc] < 0) c = -c;
      if (c != 0.f) {
        const int64_t off = kr * row_blk + kc * col_blk;
        if (g.n == 0) g.c0 = c, g.off0 = off;
        else g.c1 = c, g.off1 = off;
        ++g.n;
      }
    }
  return g;
}

// c0 x0 (+ c1 x1 when n > 1; zero when n == 0), one rounding per operation.
__device__ __forceinline__ floatx4 gather_sum(const GatherSlots& g, floatx4 x0, floatx4 x1) {
#pragma clang fp contract(off)
  const floatx4 t0 = g.c0 * x0;
  const floatx4 s = g.n > 1 ? t0 + g.c1 * x1 : t0;
  return g.n > 0 ? s : floatx4{0.f, 0.f, 0.f, 0.f};
}

// Output tile `bid` (leaf-major, then tile row, then tile column) of the batched leaf product.
// GATHER: the operands come from gsrc (LeafGather) instead of S and T.
template <int BM, int BN, int BK, int EPI = 1, bool GATHER = false>
__device__ __forceinline__ void gemm_f32_tile(const float* __restrict__ S, const float* __restrict__ T,
                                              float* __restrict__ P, int m, int n, int k, int tiles_n,
                                              int tiles_per_leaf, int64_t bid, float* smem,
                                              const LeafGather* gsrc = nullptr) {
  constexpr int LDA = F32Tile<BM, BN, BK, EPI>::LDA;  // S slab row: k-contiguous, padded
  constexpr int LDB = F32Tile<BM, BN, BK, EPI>::LDB;  // T slab row: n-contiguous, padded
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int KQ = BK / 4;                  // float4 chunks per S row of a slab
  constexpr int A_VEC = BM * KQ / 256;        // float4 loads per thread per slab
  constexpr int B_VEC = BK * (BN / 4) / 256;
  constexpr int LDE = F32Tile<BM, BN, BK, EPI>::LDE;  // epilogue row of a wavefront's quarter
  static_assert(A_VEC >= 1 && B_VEC >= 1, "tile too small for 256 threads");
  constexpr int A_FLOATS = F32Tile<BM, BN, BK, EPI>::A_FLOATS;
  float(*As)[BM][LDA] = reinterpret_cast<float(*)[BM][LDA]>(smem);
  float(*Bs)[BK][LDB] = reinterpret_cast<float(*)[BK][LDB]>(smem + A_FLOATS);

  const int64_t leaf = bid / tiles_per_leaf;
  const int t = (int)(bid - leaf * tiles_per_leaf);
  const int tm = t / tiles_n, tn = t - (t / tiles_n) * tiles_n;
  const gbl<const float>* Sl = global_ptr(S) + leaf * (int64_t)m * k + (int64_t)tm * BM * k;
  const gbl<const float>* Tl = global_ptr(T) + leaf * (int64_t)k * n + (int64_t)tn * BN;
  gbl<float>* Pl = global_ptr(P) + leaf * (int64_t)m * n + (int64_t)tm * BM * n + (int64_t)tn * BN;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // Per-thread slab sources: S row (tid + 256 i) / KQ, chunk % KQ; T row (tid + 256 i) / (BN/4).
  // With GATHER they point into the first nonzero sub-block of the leaf's parent, the
  // second at a fixed offset from the first.
  const gbl<const float>* a_src[A_VEC];
  const gbl<const float>* b_src[B_VEC];
  int64_t a_ld = k, b_ld = n, a_off1 = 0, b_off1 = 0;
  GatherSlots ga{1.f, 0.f, 0, 0, 1}, gb{1.f, 0.f, 0, 0, 1};
  if constexpr (GATHER) {
    const int64_t parent = leaf / gsrc->R;
    const int r = (int)(leaf - parent * gsrc->R);
    ga = gather_slots(gsrc->la, gsrc->bra, gsrc->bca, r, gsrc->R, gsrc->a_row_blk, gsrc->a_col_blk);
    gb = gather_slots(gsrc->lb, gsrc->brb, gsrc->bcb, r, gsrc->R, gsrc->b_row_blk, gsrc->b_col_blk);
    a_ld = gsrc->a_ld, b_ld = gsrc->b_ld;
    a_off1 = ga.off1 - ga.off0, b_off1 = gb.off1 - gb.off0;
    Sl = global_ptr(gsrc->A) + parent * gsrc->a_batch + ga.off0 + (int64_t)tm * BM * a_ld;
    Tl = global_ptr(gsrc->B) + parent * gsrc->b_batch + gb.off0 + (int64_t)tn * BN;
  }
#pragma unroll
  for (int i = 0; i < A_VEC; ++i) {
    const int idx = tid + 256 * i;
    a_src[i] = Sl + (int64_t)(idx / KQ) * a_ld + (idx % KQ) * 4;
  }
#pragma unroll
  for (int i = 0; i < B_VEC; ++i) {
    const int idx = tid + 256 * i;
    b_src[i] = Tl + (int64_t)(idx / (BN / 4)) * b_ld + (idx % (BN / 4)) * 4;
  }
  const int64_t b_step = (int64_t)BK * b_ld;

  // clang vector types (not HIP's float4 struct) so the staging stays in registers.
  // ra, rb: the slab as loaded (first sub-block with GATHER); xa, xb: second sub-block.
  floatx4 ra[A_VEC], rb[B_VEC];
  floatx4 xa[GATHER ? A_VEC : 1], xb[GATHER ? B_VEC : 1];
  auto load_slab = [&](int kt) {
#pragma unroll
    for (int i = 0; i < A_VEC; ++i) ra[i] = *reinterpret_cast<const gbl<const floatx4>*>(a_src[i] + kt * BK);
#pragma unroll
    for (int i = 0; i < B_VEC; ++i) rb[i] = *reinterpret_cast<const gbl<const floatx4>*>(b_src[i] + kt * b_step);
    if constexpr (GATHER) {
      if (ga.n > 1) {
#pragma unroll
        for (int i = 0; i < A_VEC; ++i)
          xa[i] = *reinterpret_cast<const gbl<const floatx4>*>(a_src[i] + a_off1 + kt * BK);
      }
      if (gb.n > 1) {
#pragma unroll
        for (int i = 0; i < B_VEC; ++i)
          xb[i] = *reinterpret_cast<const gbl<const floatx4>*>(b_src[i] + b_off1 + kt * b_step);
      }
    }
  };
  if constexpr (GATHER) {
#pragma unroll
    for (int i = 0; i < A_VEC; ++i) xa[i] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < B_VEC; ++i) xb[i] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
  load_slab(0);

  floatx4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int nk = k / BK;
  const int lr = lane & 15, lg = lane >> 4;
  int cur = 0;
  for (int kt = 0; kt < nk; ++kt) {
#pragma unroll
    for (int i = 0; i < A_VEC; ++i) {
      const int idx = tid + 256 * i;
      floatx4 v = ra[i];
      if constexpr (GATHER) v = gather_sum(ga, ra[i], xa[i]);
      *reinterpret_cast<floatx4*>(&As[cur][idx / KQ][(idx % KQ) * 4]) = v;
    }
#pragma unroll
    for (int i = 0; i < B_VEC; ++i) {
      const int idx = tid + 256 * i;
      floatx4 v = rb[i];
      if constexpr (GATHER) v = gather_sum(gb, rb[i], xb[i]);
      *reinterpret_cast<floatx4*>(&Bs[cur][idx / (BN / 4)][(idx % (BN / 4)) * 4]) = v;
    }
    __syncthreads();
    if (kt + 1 < nk) load_slab(kt + 1);
    // 16 k per chunk: in MFMA step j, lane group lg carries k = 16 c + 4 lg + j for both
    // operands, so one 16-byte read of S gives a lane its operands for four steps.
#pragma unroll
    for (int c = 0; c < BK / 16; ++c) {
      floatx4 a[FM];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        a[i] = *reinterpret_cast<const floatx4*>(&As[cur][wm * WM + i * 16 + lr][c * 16 + lg * 4]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float b[FN];
#pragma unroll
        for (int q = 0; q < FN; ++q) b[q] = Bs[cur][c * 16 + lg * 4 + j][wn * WN + q * 16 + lr];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int q = 0; q < FN; ++q)
            acc[i][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][j], b[q], acc[i][q], 0, 0, 0);
      }
    }
    cur ^= 1;
  }

  // Epilogue through LDS: each wavefront parks its (BM/2) x (BN/2) quarter (D layout of the
  // 16x16 MFMA: lane holds column lane & 15, rows 4 (lane >> 4) + v), WM / EPI rows per
  // pass, then writes them back row by row with 16-byte stores, 16 lanes per row.
  static_assert(FM % EPI == 0, "epilogue passes must split the fragments evenly");
  constexpr int FP = FM / EPI, WR = WM / EPI;  // fragments and rows per pass
  float* Es = smem + wave * WR * LDE;
  constexpr int LPR = WN / 4;            // lanes per row (16-byte chunks)
  constexpr int RPI = 64 / LPR;          // rows per store instruction
  gbl<float>* Pw = Pl + (int64_t)(wm * WM) * n + wn * WN;
  const int er = lane / LPR, ec = (lane % LPR) * 4;
#pragma unroll
  for (int ps = 0; ps < EPI; ++ps) {
    __syncthreads();  // every wavefront is done reading the operand buffers / the previous pass
#pragma unroll
    for (int i = 0; i < FP; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) Es[(i * 16 + lg * 4 + v) * LDE + j * 16 + lr] = acc[ps * FP + i][j][v];
    __syncthreads();
#pragma unroll
    for (int r0 = 0; r0 < WR; r0 += RPI) {
      const floatx4 v = *reinterpret_cast<const floatx4*>(&Es[(r0 + er) * LDE + ec]);
      *reinterpret_cast<gbl<floatx4>*>(Pw + (int64_t)(ps * WR + r0 + er) * n + ec) = v;
    }
  }
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
    __syncthreads();
    if (kt + 1 < nk) {
      const int k1 = (kt + 1) * BK;
#pragma unroll
      for (int i = 0; i < A_ITER; ++i) ra[i] = *reinterpret_cast<const gbl<const u32x4>*>(a_src[i] + k1);
#pragma unroll
      for (int i = 0; i < B_ITER; ++i)
        rb[i] = *reinterpret_cast<const gbl<const u32x4>*>(b_src[i] + (int64_t)k1 * n);
    }
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
    __syncthreads();
    if (kt + 1 < nk) {
      const int k1 = (kt + 1) * BK;
#pragma unroll
      for (int i = 0; i < A_ITER; ++i) ra[i] = *reinterpret_cast<const gbl<const u32x4>*>(a_src[i] + k1);
#pragma unroll
      for (int i = 0; i < B_ITER; ++i)
        rb[i] = *reinterpret_cast<const gbl<const u32x4>*>(b_src[i] + (int64_t)k1 * n);
    }
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
    __syncthreads();
    if (kt + 1 < nk) {
      const int k1 = (kt + 1) * BK;
#pragma unroll
      for (int i = 0; i < A_ITER; ++i) ra[i] = *reinterpret_cast<const gbl<const u32x4>*>(a_src[i] + k1);
#pragma unroll
      for (int i = 0; i < B_ITER; ++i)
        rb[i] = *reinterpret_cast<const gbl<const u32x4>*>(b_src[i] + (int64_t)k1 * n);
    }
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
