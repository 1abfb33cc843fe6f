// Leaf products P_l = S_l T_l (the standard product at the bottom of the
// recursion, F-hat^(0) in Section 2.1.1) for every leaf of a plan in one
// batched launch, on CDNA4 matrix cores.
//
// f32: v_mfma_f32_16x16x4_f32.  A workgroup of 4 wavefronts computes a BM x BN
// tile (BM = BN = 64 or 128), each wavefront a (BM/2) x (BN/2) quarter as a
// grid of 16x16 MFMA tiles.  K advances in slabs of 32 (16 when K is not a
// multiple of 32) through two LDS buffers: a slab held in registers is
// written to one buffer, one barrier, then the next slab's global loads are
// issued and stay in flight while the MFMAs consume the buffer.  Both slabs
// keep their memory layout in LDS (16-byte stores): the k order inside each
// group of 16 is permuted identically for both operands so that an S operand
// is one 16-byte LDS read per four MFMA steps; S rows are padded to 36 words
// and T rows to BN + 4, which spreads each read over all banks.
//
// Workgroups are dispatched round robin over the 8 XCDs; block ids are
// remapped so that the tiles of one leaf run on the same XCD and share its L2.
//
// f64: v_mfma_f64_16x16x4_f64, one wavefront per 16x16 output tile, operands
// read straight from global memory (small leaves; latency bound).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace rbc {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// Block id -> logical tile id such that consecutive logical tiles share an XCD.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nb) {
  const int64_t per = nb / 8, rem = nb % 8;
  const int64_t xcd = bid % 8, local = bid / 8;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

template <int BM, int BN, int BK>
__global__ __launch_bounds__(256) void k_gemm_f32(const float* __restrict__ S,
                                                  const float* __restrict__ T, float* __restrict__ P,
                                                  int m, int n, int k, int tiles_n,
                                                  int tiles_per_leaf, int64_t nblocks) {
  constexpr int LDA = BK + 4;                 // S slab row: k-contiguous, padded
  constexpr int LDB = BN + 4;                 // T slab row: n-contiguous, padded
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int KQ = BK / 4;                  // float4 chunks per S row of a slab
  constexpr int A_VEC = BM * KQ / 256;        // float4 loads per thread per slab
  constexpr int B_VEC = BK * (BN / 4) / 256;
  constexpr int LDE = WN + 4;                 // epilogue row of a wavefront's quarter
  static_assert(A_VEC >= 1 && B_VEC >= 1, "tile too small for 256 threads");
  // One LDS block: two S and two T slab buffers during the K loop, the four
  // wavefronts' output quarters in the epilogue.
  constexpr int A_FLOATS = 2 * BM * LDA, B_FLOATS = 2 * BK * LDB, E_FLOATS = 4 * WM * LDE;
  constexpr int SMEM = A_FLOATS + B_FLOATS > E_FLOATS ? A_FLOATS + B_FLOATS : E_FLOATS;
  __shared__ __attribute__((aligned(16))) float smem[SMEM];
  float(*As)[BM][LDA] = reinterpret_cast<float(*)[BM][LDA]>(smem);
  float(*Bs)[BK][LDB] = reinterpret_cast<float(*)[BK][LDB]>(smem + A_FLOATS);

  const int64_t bid = xcd_remap(blockIdx.x, nblocks);
  const int64_t leaf = bid / tiles_per_leaf;
  const int t = (int)(bid - leaf * tiles_per_leaf);
  const int tm = t / tiles_n, tn = t - (t / tiles_n) * tiles_n;
  const float* Sl = S + leaf * (int64_t)m * k + (int64_t)tm * BM * k;
  const float* Tl = T + leaf * (int64_t)k * n + (int64_t)tn * BN;
  float* Pl = P + leaf * (int64_t)m * n + (int64_t)tm * BM * n + (int64_t)tn * BN;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // Per-thread slab sources: S row (tid + 256 i) / KQ, chunk % KQ; T row (tid + 256 i) / (BN/4).
  const float* a_src[A_VEC];
  const float* b_src[B_VEC];
#pragma unroll
  for (int i = 0; i < A_VEC; ++i) {
    const int idx = tid + 256 * i;
    a_src[i] = Sl + (int64_t)(idx / KQ) * k + (idx % KQ) * 4;
  }
#pragma unroll
  for (int i = 0; i < B_VEC; ++i) {
    const int idx = tid + 256 * i;
    b_src[i] = Tl + (int64_t)(idx / (BN / 4)) * n + (idx % (BN / 4)) * 4;
  }
  const int64_t b_step = (int64_t)BK * n;

  // clang vector types (not HIP's float4 struct) so the staging stays in registers
  floatx4 ra[A_VEC], rb[B_VEC];
#pragma unroll
  for (int i = 0; i < A_VEC; ++i) ra[i] = *reinterpret_cast<const floatx4*>(a_src[i]);
#pragma unroll
  for (int i = 0; i < B_VEC; ++i) rb[i] = *reinterpret_cast<const floatx4*>(b_src[i]);

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
      *reinterpret_cast<floatx4*>(&As[cur][idx / KQ][(idx % KQ) * 4]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < B_VEC; ++i) {
      const int idx = tid + 256 * i;
      *reinterpret_cast<floatx4*>(&Bs[cur][idx / (BN / 4)][(idx % (BN / 4)) * 4]) = rb[i];
    }
    __syncthreads();
    if (kt + 1 < nk) {
#pragma unroll
      for (int i = 0; i < A_VEC; ++i) ra[i] = *reinterpret_cast<const floatx4*>(a_src[i] + (kt + 1) * BK);
#pragma unroll
      for (int i = 0; i < B_VEC; ++i)
        rb[i] = *reinterpret_cast<const floatx4*>(b_src[i] + (kt + 1) * b_step);
    }
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
  // 16x16 MFMA: lane holds column lane & 15, rows 4 (lane >> 4) + v), then writes it back
  // row by row with 16-byte stores, 16 lanes per row.
  __syncthreads();  // every wavefront is done reading the operand buffers
  float* Es = smem + wave * WM * LDE;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) Es[(i * 16 + lg * 4 + v) * LDE + j * 16 + lr] = acc[i][j][v];
  __syncthreads();
  constexpr int LPR = WN / 4;            // lanes per row (16-byte chunks)
  constexpr int RPI = 64 / LPR;          // rows per store instruction
  float* Pw = Pl + (int64_t)(wm * WM) * n + wn * WN;
  const int er = lane / LPR, ec = (lane % LPR) * 4;
#pragma unroll
  for (int r0 = 0; r0 < WM; r0 += RPI) {
    const floatx4 v = *reinterpret_cast<const floatx4*>(&Es[(r0 + er) * LDE + ec]);
    *reinterpret_cast<floatx4*>(Pw + (int64_t)(r0 + er) * n + ec) = v;
  }
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

}  // namespace

hipError_t launch_gemm_f32(const float* S, const float* T, float* P, int64_t m, int64_t n, int64_t k,
                           int64_t batch, int tile, hipStream_t stream) {
  if (batch == 0 || m == 0 || n == 0) return hipSuccess;
  if (m % tile || n % tile || k % 16 || (tile != 64 && tile != 128)) return hipErrorInvalidValue;
  const bool deep = k % 32 == 0;  // K slabs of 32 when K allows, else 16
  const int tiles_n = (int)(n / tile), tiles_per_leaf = (int)((m / tile) * tiles_n);
  const int64_t nblocks = batch * tiles_per_leaf;
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nblocks), block(256);
  if (tile == 128 && deep)
    hipLaunchKernelGGL((k_gemm_f32<128, 128, 32>), grid, block, 0, stream, S, T, P, (int)m, (int)n,
                       (int)k, tiles_n, tiles_per_leaf, nblocks);
  else if (tile == 128)
    hipLaunchKernelGGL((k_gemm_f32<128, 128, 16>), grid, block, 0, stream, S, T, P, (int)m, (int)n,
                       (int)k, tiles_n, tiles_per_leaf, nblocks);
  else if (deep)
    hipLaunchKernelGGL((k_gemm_f32<64, 64, 32>), grid, block, 0, stream, S, T, P, (int)m, (int)n,
                       (int)k, tiles_n, tiles_per_leaf, nblocks);
  else
    hipLaunchKernelGGL((k_gemm_f32<64, 64, 16>), grid, block, 0, stream, S, T, P, (int)m, (int)n,
                       (int)k, tiles_n, tiles_per_leaf, nblocks);
  return hipGetLastError();
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
