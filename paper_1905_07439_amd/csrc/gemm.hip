// Leaf products P_l = S_l T_l (the standard product at the bottom of the
// recursion, F-hat^(0) in Section 2.1.1) for every leaf of a plan in one
// batched launch, on CDNA4 matrix cores.
//
// f32: v_mfma_f32_16x16x4_f32.  A workgroup of 4 wavefronts computes a BM x BN
// tile (BM = BN = 64 or 128), each wavefront a (BM/2) x (BN/2) quarter as a
// grid of 16x16 MFMA tiles.  K advances in steps of 16 through a double
// buffered LDS stage: the next K slab is fetched from global memory into
// registers while the current slab feeds the MFMAs, then stored to the other
// LDS buffer.  S slabs are stored transposed (k-major) so that one MFMA
// operand is 16 consecutive LDS words per k row; rows are padded by 16 words,
// which puts the four k rows a wavefront reads in one instruction on
// disjoint banks.
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

template <int BM, int BN>
__global__ __launch_bounds__(256) void k_gemm_f32(const float* __restrict__ S,
                                                  const float* __restrict__ T, float* __restrict__ P,
                                                  int m, int n, int k, int tiles_n,
                                                  int tiles_per_leaf, int64_t nblocks) {
  constexpr int BK = 16;
  constexpr int PAD = 16;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int A_VEC = BM * BK / 4 / 256;  // float4 loads per thread per slab
  constexpr int B_VEC = BN * BK / 4 / 256;
  __shared__ float As[2][BK][BM + PAD];
  __shared__ float Bs[2][BK][BN + PAD];

  const int64_t bid = xcd_remap(blockIdx.x, nblocks);
  const int64_t leaf = bid / tiles_per_leaf;
  const int t = (int)(bid - leaf * tiles_per_leaf);
  const int tm = t / tiles_n, tn = t - (t / tiles_n) * tiles_n;
  const float* Sl = S + leaf * (int64_t)m * k + (int64_t)tm * BM * k;
  const float* Tl = T + leaf * (int64_t)k * n + (int64_t)tn * BN;
  float* Pl = P + leaf * (int64_t)m * n + (int64_t)tm * BM * n + (int64_t)tn * BN;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  float4 ra[A_VEC], rb[B_VEC];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < A_VEC; ++i) {
      const int idx = tid + 256 * i, row = idx / (BK / 4), kq = idx % (BK / 4);
      ra[i] = *reinterpret_cast<const float4*>(Sl + (int64_t)row * k + k0 + kq * 4);
    }
#pragma unroll
    for (int i = 0; i < B_VEC; ++i) {
      const int idx = tid + 256 * i, kr = idx / (BN / 4), cq = idx % (BN / 4);
      rb[i] = *reinterpret_cast<const float4*>(Tl + (int64_t)(k0 + kr) * n + cq * 4);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < A_VEC; ++i) {
      const int idx = tid + 256 * i, row = idx / (BK / 4), kq = idx % (BK / 4);
      As[buf][kq * 4 + 0][row] = ra[i].x;
      As[buf][kq * 4 + 1][row] = ra[i].y;
      As[buf][kq * 4 + 2][row] = ra[i].z;
      As[buf][kq * 4 + 3][row] = ra[i].w;
    }
#pragma unroll
    for (int i = 0; i < B_VEC; ++i) {
      const int idx = tid + 256 * i, kr = idx / (BN / 4), cq = idx % (BN / 4);
      *reinterpret_cast<float4*>(&Bs[buf][kr][cq * 4]) = rb[i];
    }
  };

  floatx4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  gload(0);
  sstore(0);
  __syncthreads();
  const int nk = k / BK;
  const int lr = lane & 15, lk = lane >> 4;
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      float a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = As[cur][kk + lk][wm * WM + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = Bs[cur][kk + lk][wn * WN + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }

  // D layout of the 16x16 MFMA: lane holds column (lane & 15), rows 4*(lane >> 4) + v.
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wm * WM + i * 16 + lk * 4 + v, col = wn * WN + j * 16 + lr;
        Pl[(int64_t)row * n + col] = acc[i][j][v];
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
  const int tiles_n = (int)(n / tile), tiles_per_leaf = (int)((m / tile) * tiles_n);
  const int64_t nblocks = batch * tiles_per_leaf;
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  if (tile == 128)
    hipLaunchKernelGGL((k_gemm_f32<128, 128>), dim3((unsigned)nblocks), dim3(256), 0, stream, S, T, P,
                       (int)m, (int)n, (int)k, tiles_n, tiles_per_leaf, nblocks);
  else
    hipLaunchKernelGGL((k_gemm_f32<64, 64>), dim3((unsigned)nblocks), dim3(256), 0, stream, S, T, P,
                       (int)m, (int)n, (int)k, tiles_n, tiles_per_leaf, nblocks);
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
