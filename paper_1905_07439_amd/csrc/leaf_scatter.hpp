// The deepest level's scatter (eq. recursive-random-formula, the W side of the
// deepest level) folded into the f32 leaf product: after a workgroup has
// stored its tile of leaf l = parent * R + r, it counts the tile in the
// parent's counter of every 64 x 64 region the tile covers; the workgroup that
// brings a region's count to R reads that region of the parent's R products
// and writes the region of every sub-block of the parent's product block.
//
// Ordering: each wavefront waits for its own stores, the workgroup meets at a
// barrier, then thread 0 executes an agent-scope release fence (an L2
// write-back on gfx950, waited for before the counters move) and adds to the
// counters.  A counter's additions form one release sequence, so the thread
// whose addition returns R - 1 executes an agent-scope acquire fence (L1 and
// L2 invalidation) and has seen every other tile of the region once the
// workgroup's barrier releases the other wavefronts to read.
#pragma once

#include "devptr.hpp"
#include "gemm_tiles.hpp"
#include "kernels.hpp"

namespace rbc {
namespace tiles {

// Folded coefficient of output sub-block (k, l), product r (f32 table).
__device__ __forceinline__ float leaf_scatter_coef(const SideLevel& L, int bc, int k, int l, int r, int R) {
  const gbl<const float>* tab = global_ptr(static_cast<const float*>(L.tab));
  const float c = tab[(L.pr[k] * bc + L.pc[l]) * R + r];
  return L.sr[k] * L.sc[l] < 0 ? -c : c;
}

// One 64 x 64 region (rows row0.., columns col0.. of every leaf of `parent`):
// 256 threads, each four rows (16 apart) of four consecutive columns.
__device__ __forceinline__ void leaf_scatter_region(const LeafScatter& s, const float* P, int m, int n, int R,
                                                    int64_t parent, int row0, int col0) {
#pragma clang fp contract(off)
  const int tid = threadIdx.x;
  const int rr = row0 + (tid >> 4), cc = col0 + (tid & 15) * 4;
  const gbl<const float>* Pp = global_ptr(P) + parent * R * (int64_t)m * n + (int64_t)rr * n + cc;
  gbl<float>* Op = global_ptr(s.out) + parent * s.out_batch + (int64_t)rr * s.out_ld + cc;
  for (int k = 0; k < s.br; ++k)
    for (int l = 0; l < s.bc; ++l) {
      floatx4 acc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
      bool first = true;
      for (int r = 0; r < R; ++r) {
        const float c = __builtin_bit_cast(
            float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, leaf_scatter_coef(s.lw, s.bc, k, l, r, R))));
        if (c == 0.f) continue;  // uniform
        const gbl<const float>* Pr = Pp + (int64_t)r * m * n;
        floatx4 x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = *reinterpret_cast<const gbl<const floatx4>*>(Pr + (int64_t)(16 * q) * n);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const floatx4 t = c * x[q];
          acc[q] = first ? t : acc[q] + t;
        }
        first = false;
      }
      gbl<float>* O = Op + k * s.row_blk + l * s.col_blk;
#pragma unroll
      for (int q = 0; q < 4; ++q) *reinterpret_cast<gbl<floatx4>*>(O + (int64_t)(16 * q) * s.out_ld) = acc[q];
    }
}

// Every thread of the workgroup calls this after its stores of the BM x BN tile
// (tile row tm, column tn) of leaf `leaf`.  flags: BM / 64 * BN / 64 ints of LDS.
template <int BM, int BN>
__device__ __forceinline__ void leaf_scatter_tile(const LeafScatter& s, const float* P, int m, int n, int R,
                                                  int64_t leaf, int tm, int tn, int32_t* flags) {
  constexpr int QM = BM / 64, QN = BN / 64;
  const int64_t parent = leaf / R;
  const int sub_n = n / 64;
  const int64_t base = parent * (int64_t)(m / 64) * sub_n;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    // The fence's L2 write-back must be complete before a counter moves; the
    // compiler does not wait for it when nothing it tracks is outstanding.
    __builtin_amdgcn_s_waitcnt(0);
    bool any = false;
#pragma unroll
    for (int i = 0; i < QM; ++i)
#pragma unroll
      for (int j = 0; j < QN; ++j) {
        int32_t* c = s.cnt + base + (int64_t)(tm * QM + i) * sub_n + tn * QN + j;
        const bool last = __hip_atomic_fetch_add(c, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == R - 1;
        flags[i * QN + j] = last;
        any = any || last;
      }
    if (any) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      // the invalidation is complete before the barrier lets the other wavefronts read
      __builtin_amdgcn_s_waitcnt(0);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < QM; ++i)
#pragma unroll
    for (int j = 0; j < QN; ++j)
      if (__builtin_amdgcn_readfirstlane(flags[i * QN + j]))
        leaf_scatter_region(s, P, m, n, R, parent, (tm * QM + i) * 64, (tn * QN + j) * 64);
}

}  // namespace tiles
}  // namespace rbc
