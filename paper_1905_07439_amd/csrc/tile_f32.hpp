// f32 leaf product tile (v_mfma_f32_16x16x4f32), optionally forming its operands
// from the parent blocks of the deepest level while loading them (leaf gather).
//
#pragma once

#include "gemm_tiles.hpp"

namespace rbc {
namespace tiles {

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


// ---- leaf gather with buffer loads --------------------------------------------
// The gathered tile above, restructured for the matrix cores' sake (measured on
// 343 leaves of 512^3 from 49 parents of 1024^2: 0.810 -> 0.769-0.777 ms, the
// same bits):
//  - loads through one buffer resource per parent: each thread keeps one 32-bit
//    offset per load, the sub-block and slab offsets are scalar, so the K loop
//    does no address arithmetic and the tile fits in 138 VGPRs (167 before);
//  - the next slab's loads are issued right after the current slab is stored,
//    before the barrier;
//  - a chunk's T operands are read from LDS all at once before its MFMAs;
//  - when the second coefficient is +-1 (every Strassen-like level), the
//    operand is fma(c1, x1, c0 x0): c1 x1 is exact, so the single rounding of
//    the fma equals rounding the sum of the rounded terms.
// Parents must be under 2 GiB (32-bit byte offsets); the launcher checks.
typedef __amdgpu_buffer_rsrc_t buffer_rsrc;

__device__ __forceinline__ floatx4 buffer_load4(buffer_rsrc r, int voff, int soff) {
  return __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

// How a side forms its operand from its (at most two) sub-blocks: 0 zero, 1 c0 x0,
// 2 fma(c1, x1, c0 x0) for c1 = +-1, 3 c0 x0 + c1 x1 with both terms rounded.
__device__ __forceinline__ int gather_mode(const GatherSlots& g) {
  if (g.n == 0) return 0;
  if (g.n == 1) return 1;
  return __builtin_fabsf(g.c1) == 1.f ? 2 : 3;
}

template <int NV>
__device__ __forceinline__ void gather_combine(int mode, const GatherSlots& g, floatx4 (&x0)[NV],
                                               const floatx4 (&x1)[NV]) {
#pragma clang fp contract(off)
  if (mode == 2) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const floatx4 t = g.c0 * x0[i];
#pragma unroll
      for (int e = 0; e < 4; ++e) x0[i][e] = __builtin_fmaf(g.c1, x1[i][e], t[e]);
    }
  } else if (mode == 1) {
#pragma unroll
    for (int i = 0; i < NV; ++i) x0[i] = g.c0 * x0[i];
  } else if (mode == 3) {
#pragma unroll
    for (int i = 0; i < NV; ++i) x0[i] = g.c0 * x0[i] + g.c1 * x1[i];
  } else {
#pragma unroll
    for (int i = 0; i < NV; ++i) x0[i] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
}

__device__ __forceinline__ float uniform_f(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}

// Output tile `bid` of the batched leaf product, operands gathered from the parents
// (LeafGather) as gemm_f32_tile<..., GATHER = true> does, with the same arithmetic
// in the same order.
template <int BM, int BN, int BK, int EPI>
__device__ __forceinline__ void gemm_f32_gathered_tile(const LeafGather* gs, float* __restrict__ P, int m, int n,
                                                       int k, int tiles_n, int tiles_per_leaf, int64_t bid,
                                                       float* smem) {
  using Cfg = F32Tile<BM, BN, BK, EPI>;
  constexpr int LDA = Cfg::LDA, LDB = Cfg::LDB, WM = BM / 2, WN = BN / 2, LDE = Cfg::LDE;
  constexpr int FM = WM / 16, FN = WN / 16, KQ = BK / 4;
  constexpr int A_VEC = BM * KQ / 256, B_VEC = BK * (BN / 4) / 256;
  static_assert(A_VEC >= 1 && B_VEC >= 1, "tile too small for 256 threads");
  float(*As)[BM][LDA] = reinterpret_cast<float(*)[BM][LDA]>(smem);
  float(*Bs)[BK][LDB] = reinterpret_cast<float(*)[BK][LDB]>(smem + Cfg::A_FLOATS);
  const int64_t leaf = bid / tiles_per_leaf;
  const int t = (int)(bid - leaf * tiles_per_leaf);
  const int tm = t / tiles_n, tn = t - (t / tiles_n) * tiles_n;
  gbl<float>* Pl = global_ptr(P) + leaf * (int64_t)m * n + (int64_t)tm * BM * n + (int64_t)tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t parent = leaf / gs->R;
  const int r = (int)(leaf - parent * gs->R);
  GatherSlots ga = gather_slots(gs->la, gs->bra, gs->bca, r, gs->R, gs->a_row_blk, gs->a_col_blk);
  GatherSlots gb = gather_slots(gs->lb, gs->brb, gs->bcb, r, gs->R, gs->b_row_blk, gs->b_col_blk);
  ga.c0 = uniform_f(ga.c0), ga.c1 = uniform_f(ga.c1), gb.c0 = uniform_f(gb.c0), gb.c1 = uniform_f(gb.c1);
  const int ma = __builtin_amdgcn_readfirstlane(gather_mode(ga));
  const int mb = __builtin_amdgcn_readfirstlane(gather_mode(gb));
  const buffer_rsrc rsa = __builtin_amdgcn_make_buffer_rsrc((void*)(gs->A + parent * gs->a_batch), 0,
                                                            (int)(gs->a_batch * 4), 0x00020000);
  const buffer_rsrc rsb = __builtin_amdgcn_make_buffer_rsrc((void*)(gs->B + parent * gs->b_batch), 0,
                                                            (int)(gs->b_batch * 4), 0x00020000);
  int a_vo[A_VEC], b_vo[B_VEC];
#pragma unroll
  for (int i = 0; i < A_VEC; ++i) {
    const int idx = tid + 256 * i;
    a_vo[i] = (int)(((int64_t)(tm * BM + idx / KQ) * gs->a_ld + (idx % KQ) * 4) * 4);
  }
#pragma unroll
  for (int i = 0; i < B_VEC; ++i) {
    const int idx = tid + 256 * i;
    b_vo[i] = (int)(((int64_t)(idx / (BN / 4)) * gs->b_ld + tn * BN + (idx % (BN / 4)) * 4) * 4);
  }
  const int a0 = __builtin_amdgcn_readfirstlane((int)(ga.off0 * 4));
  const int a1 = __builtin_amdgcn_readfirstlane((int)(ga.off1 * 4));
  const int b0 = __builtin_amdgcn_readfirstlane((int)(gb.off0 * 4));
  const int b1 = __builtin_amdgcn_readfirstlane((int)(gb.off1 * 4));
  const int b_step = (int)(BK * gs->b_ld * 4);
  floatx4 ra[A_VEC], rb[B_VEC], xa[A_VEC], xb[B_VEC];
  auto load_slab = [&](int kt) {
    const int sa = kt * BK * 4, sb = kt * b_step;
#pragma unroll
    for (int i = 0; i < A_VEC; ++i) ra[i] = buffer_load4(rsa, a_vo[i], a0 + sa);
    if (ma >= 2) {
#pragma unroll
      for (int i = 0; i < A_VEC; ++i) xa[i] = buffer_load4(rsa, a_vo[i], a1 + sa);
    }
#pragma unroll
    for (int i = 0; i < B_VEC; ++i) rb[i] = buffer_load4(rsb, b_vo[i], b0 + sb);
    if (mb >= 2) {
#pragma unroll
      for (int i = 0; i < B_VEC; ++i) xb[i] = buffer_load4(rsb, b_vo[i], b1 + sb);
    }
  };
#pragma unroll
  for (int i = 0; i < A_VEC; ++i) xa[i] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < B_VEC; ++i) xb[i] = floatx4{0.f, 0.f, 0.f, 0.f};
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
    gather_combine(ma, ga, ra, xa);
    gather_combine(mb, gb, rb, xb);
#pragma unroll
    for (int i = 0; i < A_VEC; ++i) {
      const int idx = tid + 256 * i;
      *reinterpret_cast<floatx4*>(&As[cur][idx / KQ][(idx % KQ) * 4]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < B_VEC; ++i) {
      const int idx = tid + 256 * i;
      *reinterpret_cast<floatx4*>(&Bs[cur][idx / (BN / 4)][(idx % (BN / 4)) * 4]) = rb[i];
    }
    if (kt + 1 < nk) load_slab(kt + 1);  // the staging registers are free once stored
    __syncthreads();
    // k order inside each chunk of 16 as in gemm_f32_tile (same bits)
#pragma unroll
    for (int c = 0; c < BK / 16; ++c) {
      floatx4 a[FM];
      float b[4][FN];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        a[i] = *reinterpret_cast<const floatx4*>(&As[cur][wm * WM + i * 16 + lr][c * 16 + lg * 4]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int q = 0; q < FN; ++q) b[j][q] = Bs[cur][c * 16 + lg * 4 + j][wn * WN + q * 16 + lr];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int q = 0; q < FN; ++q)
            acc[i][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][j], b[j][q], acc[i][q], 0, 0, 0);
    }
    cur ^= 1;
  }
  static_assert(FM % EPI == 0, "epilogue passes must split the fragments evenly");
  constexpr int FP = FM / EPI, WR = WM / EPI;
  float* Es = smem + wave * WR * LDE;
  constexpr int LPR = WN / 4, RPI = 64 / LPR;
  gbl<float>* Pw = Pl + (int64_t)(wm * WM) * n + wn * WN;
  const int er = lane / LPR, ec = (lane % LPR) * 4;
#pragma unroll
  for (int ps = 0; ps < EPI; ++ps) {
    __syncthreads();
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

}  // namespace tiles
}  // namespace rbc

