// Level-synchronous execution of a batch's task table: the tasks are grouped
// by their depth in the dependency graph and by task type; every group runs as
// one grid in which each workgroup executes one piece of one task, through the
// same device functions as the stand-alone kernels (so every product keeps its
// bits).  Kernel boundaries order the levels: no waits, no fences, and each
// kernel has the register budget of its own task type only.
#pragma once
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "combine.hpp"
#include "tile_f32.hpp"
#include "tile_fp8.hpp"
#include "tile_lowp.hpp"
#include "scale.hpp"

namespace rbc {
namespace batch {

// One workgroup's work: piece `piece` of task `task` (index into the task table).
struct PieceRef {
  int32_t task;
  int32_t piece;
};

struct GroupArgs {
  const Task* tasks;
  const PieceRef* pieces;  // this group's entries, one per workgroup
  const GatherParams* gather;
  const ScatterParams* scatter;
  const LeafDesc* leaf;
  const ScaleDesc* scale;
};

__device__ __forceinline__ const Task& group_task(const GroupArgs& a, int32_t* piece) {
  const PieceRef r = a.pieces[blockIdx.x];
  const int32_t t = __builtin_amdgcn_readfirstlane(r.task);
  *piece = __builtin_amdgcn_readfirstlane(r.piece);
  return a.tasks[t];
}

template <int I>
__global__ __launch_bounds__(256) void k_group_gather(GroupArgs a) {
  constexpr CombVariant G = kGathers[I];
  int32_t piece;
  const Task& task = group_task(a, &piece);
  const GatherParams& p = a.gather[task.param];
  __shared__ float ct[comb::gather_coef_entries<float, G.out, G.nl, G.br, G.bc, G.R>()];
  comb::stage_gather_coefs<float, G.out, G.nl, G.br, G.bc, G.R>(p.lev, ct);
  if constexpr (G.out == OUT_F16S || G.out == OUT_FP8X2) {
    __shared__ int32_t exps[comb::group_outputs<G.nl, G.R>()];
    comb::load_exponents<G.nl, G.R>(p, task.sub, exps);
    comb::gather_block<float, G.out, G.vec, G.nl, G.br, G.bc, G.R>(p, ct, piece, task.sub, exps);
  } else {
    comb::gather_block<float, G.out, G.vec, G.nl, G.br, G.bc, G.R>(p, ct, piece, task.sub, nullptr);
  }
}

template <int I>
__global__ __launch_bounds__(256) void k_group_scatter(GroupArgs a) {
  constexpr CombVariant S = kScatters[I];
  int32_t piece;
  const Task& task = group_task(a, &piece);
  const ScatterParams& p = a.scatter[task.param];
  __shared__ float ct[comb::scatter_coef_entries<float, S.nl, S.br, S.bc, S.R>()];
  comb::stage_scatter_coefs<float, S.nl, S.br, S.bc, S.R>(p.lev, ct);
  comb::scatter_block<float, float, float, S.vec, S.nl, S.br, S.bc, S.R>(p, ct, piece, task.sub);
}

template <int I>
__global__ __launch_bounds__(256) void k_group_leaf(GroupArgs a) {
  constexpr LeafVariant L = kLeaves[I];
  int32_t piece;
  const Task& task = group_task(a, &piece);
  const LeafDesc& d = a.leaf[task.param];
  if constexpr (L.prec == RBC_PREC_F32) {
    __shared__ __attribute__((aligned(16))) float smem[tiles::F32Tile<L.tile, L.tile, L.bk>::SMEM];
    tiles::gemm_f32_tile<L.tile, L.tile, L.bk>(static_cast<const float*>(d.S), static_cast<const float*>(d.T), d.P,
                                               d.m, d.n, d.k, d.tiles_n, d.tiles_per_leaf, piece, smem);
  } else if constexpr (L.prec == RBC_PREC_F16S) {
    __shared__ __attribute__((aligned(16))) uint16_t smem[tiles::LowpTile<tiles::LOWP_F16S, L.tile, L.tile>::SMEM_HALVES];
    tiles::gemm_lowp_tile<tiles::LOWP_F16S, L.tile, L.tile>(
        static_cast<const uint16_t*>(d.S), static_cast<const uint16_t*>(d.T), d.P, d.m, d.n, d.k, d.plane_s,
        d.plane_t, d.eS, d.eT, d.tiles_n, d.tiles_per_leaf, piece, smem);
  } else {
    __shared__ __attribute__((aligned(16))) uint8_t smem[tiles::Fp8Tile<L.tile, L.tile>::SMEM_BYTES];
    tiles::gemm_fp8c_tile<L.tile, L.tile>(static_cast<const uint8_t*>(d.S), static_cast<const uint8_t*>(d.T), d.P,
                                          d.m, d.n, d.k, d.plane_s, d.plane_t, d.eS, d.eT, d.tiles_n,
                                          d.tiles_per_leaf, piece, smem);
  }
}

// Scale tasks: a max|X| piece is a run of level_rows rows of its task (the
// last one shorter); the exponent task is one piece.
static __global__ __launch_bounds__(256) void k_group_maxabs(GroupArgs a) {
  int32_t piece;
  const Task& task = group_task(a, &piece);
  const ScaleDesc& d = a.scale[task.param];
  const int64_t end = task.first + task.count;
  const int64_t nr = end - piece < d.level_rows ? end - piece : d.level_rows;
  scale::maxabs_fold(scale::maxabs_rows(d.X, d.ld, d.cols, piece, nr), d.maxbits);
}

static __global__ __launch_bounds__(256) void k_group_exponents(GroupArgs a) {
  int32_t piece;
  const Task& task = group_task(a, &piece);
  const ScaleDesc& d = a.scale[task.param];
  const float mx = __uint_as_float(*global_ptr(d.maxbits));
  const gbl<const float>* G = global_ptr(d.G);
  gbl<int32_t>* e = global_ptr(d.e);
  for (int64_t l = threadIdx.x; l < d.n_leaves; l += 256) e[l] = scale::leaf_exponent(mx, G[l], d.target);
}

// Launch of one group: kind and variant select the kernel, `pieces` entries.
template <int PREC, int I>
hipError_t launch_gather_variant(int v, const GroupArgs& a, unsigned grid, hipStream_t s) {
  if constexpr (I < kNumGathers) {
    constexpr CombVariant G = kGathers[I];
    constexpr bool in = G.out == OUT_SAME || (PREC == RBC_PREC_F16S && G.out == OUT_F16S) ||
                        (PREC == RBC_PREC_FP8C && G.out == OUT_FP8X2);
    if constexpr (in) {
      if (v == I) {
        hipLaunchKernelGGL(k_group_gather<I>, dim3(grid), dim3(256), 0, s, a);
        return hipGetLastError();
      }
    }
    return launch_gather_variant<PREC, I + 1>(v, a, grid, s);
  }
  return hipErrorInvalidValue;
}

template <int I>
hipError_t launch_scatter_variant(int v, const GroupArgs& a, unsigned grid, hipStream_t s) {
  if constexpr (I < kNumScatters) {
    if (v == I) {
      hipLaunchKernelGGL(k_group_scatter<I>, dim3(grid), dim3(256), 0, s, a);
      return hipGetLastError();
    }
    return launch_scatter_variant<I + 1>(v, a, grid, s);
  }
  return hipErrorInvalidValue;
}

template <int PREC, int I>
hipError_t launch_leaf_variant(int v, const GroupArgs& a, unsigned grid, hipStream_t s) {
  if constexpr (I < kNumLeaves) {
    if constexpr (kLeaves[I].prec == PREC) {
      if (v == I) {
        hipLaunchKernelGGL(k_group_leaf<I>, dim3(grid), dim3(256), 0, s, a);
        return hipGetLastError();
      }
    }
    return launch_leaf_variant<PREC, I + 1>(v, a, grid, s);
  }
  return hipErrorInvalidValue;
}

template <int PREC>
hipError_t launch_group_prec(int kind, int variant, const GroupArgs& a, int64_t grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  const unsigned g = (unsigned)grid;
  switch (kind) {
    case TK_GATHER: return launch_gather_variant<PREC, 0>(variant, a, g, s);
    case TK_SCATTER: return launch_scatter_variant<0>(variant, a, g, s);
    case TK_LEAF: return launch_leaf_variant<PREC, 0>(variant, a, g, s);
    case TK_MAXABS:
      hipLaunchKernelGGL(k_group_maxabs, dim3(g), dim3(256), 0, s, a);
      return hipGetLastError();
    case TK_EXPONENTS:
      hipLaunchKernelGGL(k_group_exponents, dim3(g), dim3(256), 0, s, a);
      return hipGetLastError();
    default: return hipSuccess;  // gates: ordering only
  }
}

}  // namespace batch
}  // namespace rbc
