// Measured ceilings for the rooflines: a streaming copy (HBM bandwidth) and
// register-only loops of matrix-core instructions per data type (MFMA peak),
// launched on the caller's stream and timed by the caller.  They read no
// operands from memory: every wavefront keeps CH independent accumulators busy
// and writes one value per lane at the end, so that nothing is optimised away.
#include <hip/hip_runtime.h>

#include "devptr.hpp"
#include "kernels.hpp"

namespace rbc {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef int i8v __attribute__((ext_vector_type(8)));

constexpr int CH = 8;  // independent accumulation chains per wavefront

// Four 16-byte streaming (non-temporal) loads in flight per thread, then their
// streaming stores, as the combination kernels move their data.
__global__ __launch_bounds__(256) void k_copy(const f4* __restrict__ src, f4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const f4 a = __builtin_nontemporal_load(src + i), b = __builtin_nontemporal_load(src + i + stride);
    const f4 c = __builtin_nontemporal_load(src + i + 2 * stride), d = __builtin_nontemporal_load(src + i + 3 * stride);
    __builtin_nontemporal_store(a, dst + i);
    __builtin_nontemporal_store(b, dst + i + stride);
    __builtin_nontemporal_store(c, dst + i + 2 * stride);
    __builtin_nontemporal_store(d, dst + i + 3 * stride);
  }
  for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

template <int KIND>
__global__ __launch_bounds__(256) void k_mfma(int iters, float seed, float* __restrict__ sink) {
  const float x = seed * (float)(threadIdx.x + 1);
  float out = 0.f;
  if constexpr (KIND == RBC_PEAK_F32) {
    f4 acc[CH] = {};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, x, acc[c], 0, 0, 0);
#pragma unroll
    for (int c = 0; c < CH; ++c) out += acc[c][0];
  } else if constexpr (KIND == RBC_PEAK_F64) {
    d4 acc[CH] = {};
    const double y = x;
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(y, y, acc[c], 0, 0, 0);
#pragma unroll
    for (int c = 0; c < CH; ++c) out += (float)acc[c][0];
  } else if constexpr (KIND == RBC_PEAK_F32_32 || KIND == RBC_PEAK_F16_32 || KIND == RBC_PEAK_BF16_32) {
    f16v acc[CH / 2] = {};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < CH / 2; ++c) {
        if constexpr (KIND == RBC_PEAK_F32_32) {
          acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(x, x, acc[c], 0, 0, 0);
        } else if constexpr (KIND == RBC_PEAK_F16_32) {
          const h8 a = (h8)(_Float16)x;
          acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, a, acc[c], 0, 0, 0);
        } else {
          const b8 a = (b8)(__bf16)x;
          acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, a, acc[c], 0, 0, 0);
        }
      }
#pragma unroll
    for (int c = 0; c < CH / 2; ++c) out += acc[c][0];
  } else if constexpr (KIND == RBC_PEAK_F16 || KIND == RBC_PEAK_BF16) {
    f4 acc[CH] = {};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        if constexpr (KIND == RBC_PEAK_F16) {
          const h8 a = (h8)(_Float16)x;
          acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, a, acc[c], 0, 0, 0);
        } else {
          const b8 a = (b8)(__bf16)x;
          acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, a, acc[c], 0, 0, 0);
        }
      }
#pragma unroll
    for (int c = 0; c < CH; ++c) out += acc[c][0];
  } else {  // RBC_PEAK_FP8: 32x32x64 e4m3 at unit scale
    f16v acc[CH / 2] = {};
    // bytes 0x38 ^ (8 * (lane % 8)): finite e4m3 values in [0, 1]
    const i8v a = (i8v)(int)(0x38383838u ^ ((threadIdx.x & 7u) << 3));
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < CH / 2; ++c)
        acc[c] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, a, acc[c], 0, 0, 0, 127, 0, 127);
#pragma unroll
    for (int c = 0; c < CH / 2; ++c) out += acc[c][0];
  }
  global_ptr(sink)[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = out;
}

}  // namespace

extern "C" {

rbc_status rbc_peak_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (!src || !dst) return fail(RBC_EINVAL, "null buffer");
  if (bytes % 16 || reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
    return fail(RBC_EINVAL, "copy of %zu bytes: size and both pointers must be multiples of 16", bytes);
  const int64_t n = (int64_t)(bytes / 16);
  if (n == 0) return RBC_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     static_cast<const f4*>(src), static_cast<f4*>(dst), n);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? RBC_OK : fail(RBC_EHIP, "copy launch: %s", hipGetErrorString(e));
}

rbc_status rbc_peak_mfma(int kind, int blocks, int iters, float* sink, double* flops, void* stream) {
  if (!sink || blocks < 1 || iters < 1) return fail(RBC_EINVAL, "null sink or empty launch");
  const dim3 g((unsigned)blocks), b(256);
  const hipStream_t s = (hipStream_t)stream;
  double per;  // flops of one instruction
  switch (kind) {
    case RBC_PEAK_F32: hipLaunchKernelGGL(k_mfma<RBC_PEAK_F32>, g, b, 0, s, iters, 1.0f, sink); per = 2.0 * 16 * 16 * 4; break;
    case RBC_PEAK_F64: hipLaunchKernelGGL(k_mfma<RBC_PEAK_F64>, g, b, 0, s, iters, 1.0f, sink); per = 2.0 * 16 * 16 * 4; break;
    case RBC_PEAK_F16: hipLaunchKernelGGL(k_mfma<RBC_PEAK_F16>, g, b, 0, s, iters, 1.0f, sink); per = 2.0 * 16 * 16 * 32; break;
    case RBC_PEAK_BF16: hipLaunchKernelGGL(k_mfma<RBC_PEAK_BF16>, g, b, 0, s, iters, 1.0f, sink); per = 2.0 * 16 * 16 * 32; break;
    case RBC_PEAK_FP8: hipLaunchKernelGGL(k_mfma<RBC_PEAK_FP8>, g, b, 0, s, iters, 1.0f, sink); per = 2.0 * 32 * 32 * 64; break;
    case RBC_PEAK_F32_32: hipLaunchKernelGGL(k_mfma<RBC_PEAK_F32_32>, g, b, 0, s, iters, 1.0f, sink); per = 2.0 * 32 * 32 * 2; break;
    case RBC_PEAK_F16_32: hipLaunchKernelGGL(k_mfma<RBC_PEAK_F16_32>, g, b, 0, s, iters, 1.0f, sink); per = 2.0 * 32 * 32 * 16; break;
    case RBC_PEAK_BF16_32: hipLaunchKernelGGL(k_mfma<RBC_PEAK_BF16_32>, g, b, 0, s, iters, 1.0f, sink); per = 2.0 * 32 * 32 * 16; break;
    default: return fail(RBC_EINVAL, "unknown matrix-core kind %d", kind);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RBC_EHIP, "matrix-core loop launch: %s", hipGetErrorString(e));
  const double waves = (double)blocks * 4, chains = (kind == RBC_PEAK_F32 || kind == RBC_PEAK_F64 || kind == RBC_PEAK_F16 ||
                                                    kind == RBC_PEAK_BF16) ? CH : CH / 2;
  if (flops) *flops = waves * iters * chains * per;
  return RBC_OK;
}

}  // extern "C"
}  // namespace rbc
