// The persistent batch kernel (see batch.hpp for the task model).
//
// Synchronisation: after a task, every wavefront waits until its own memory
// operations have completed (s_waitcnt 0: the stores have reached the L2; the
// workgroup barrier alone does not wait for global stores), then a barrier,
// then thread 0's agent-scope release fence and the atomic add of the task's
// piece count to its completion counter.  A waiting task's thread 0 polls its counters with
// agent-scope atomic loads (sleeping between polls) and then takes an
// agent-scope acquire fence before the barrier that releases the other
// wavefronts.  On this hardware those fences act on caches that the whole
// workgroup shares: the release writes back the XCD's L2 (which holds every
// wavefront's completed stores), the acquire invalidates the CU's L1 and the
// XCD's L2 before any wavefront of the workgroup loads task data.  So one
// fence per task and direction is enough, and producers and consumers may run
// on different XCDs.
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

template <int PREC>
struct Smem {
  // the fp8 leaves the engine runs (96, 64, 32) have two LDS layouts
  static constexpr size_t fp8_bytes =
      tiles::Fp8Tile<96, 96>::SMEM_BYTES > tiles::Fp8Tile<64, 64>::SMEM_BYTES ? tiles::Fp8Tile<96, 96>::SMEM_BYTES
                                                                             : tiles::Fp8Tile<64, 64>::SMEM_BYTES;
  static constexpr size_t bytes =
      PREC == RBC_PREC_F32    ? sizeof(float) * tiles::F32Tile<64, 64, 32>::SMEM
      : PREC == RBC_PREC_F16S ? sizeof(uint16_t) * tiles::LowpTile<tiles::LOWP_F16S, 128, 128>::SMEM_HALVES
                              : fp8_bytes;
};

// Most outputs per top block among the compiled gathers (f16s exponents in LDS).
constexpr int max_gather_outputs() {
  int m = 0;
  for (const CombVariant& v : kGathers) {
    int o = 1;
    for (int l = 0; l < v.nl; ++l) o *= v.R;
    m = o > m ? o : m;
  }
  return m;
}
constexpr int kMaxGatherOutputs = max_gather_outputs();

// Most staged coefficients among the compiled gathers and scatters.
template <int I>
constexpr int max_coef_entries() {
  if constexpr (I < kNumGathers + kNumScatters) {
    constexpr bool g = I < kNumGathers;
    constexpr CombVariant v = g ? kGathers[I] : kScatters[I - kNumGathers];
    constexpr int e = g ? comb::gather_coef_entries<float, v.out, v.nl, v.br, v.bc, v.R>()
                        : comb::scatter_coef_entries<float, v.nl, v.br, v.bc, v.R>();
    constexpr int rest = max_coef_entries<I + 1>();
    return e > rest ? e : rest;
  } else {
    return 1;
  }
}
constexpr int kMaxCoefEntries = max_coef_entries<0>();

template <int PREC>
constexpr bool gather_in(const CombVariant& v) {
  return v.out == OUT_SAME || (PREC == RBC_PREC_F16S && v.out == OUT_F16S) ||
         (PREC == RBC_PREC_FP8C && v.out == OUT_FP8X2);
}

template <int OUTF, int V, int NL, int BR, int BC, int R>
__device__ __forceinline__ void gather_task(const GatherParams& p, int64_t first, int count, int64_t in,
                                            int32_t* exps, float* ct) {
  static_assert(comb::gather_coef_entries<float, OUTF, NL, BR, BC, R>() <= kMaxCoefEntries, "staging too small");
  comb::stage_gather_coefs<float, OUTF, NL, BR, BC, R>(p.lev, ct);
  if constexpr (OUTF == OUT_F16S || OUTF == OUT_FP8X2) comb::load_exponents<NL, R>(p, in, exps);
  // the walk specialized to Strassen's pattern for every variant: its registers spill here
  // (70 VGPRs), yet the 512-product batch went from 123.8 to 113.8 ms
  for (int c = 0; c < count; ++c) comb::gather_block<float, OUTF, V, NL, BR, BC, R, true>(p, ct, first + c, in, exps);
}

template <int V, int NL, int BR, int BC, int R>
__device__ __forceinline__ void scatter_task(const ScatterParams& p, int64_t first, int count, int64_t o,
                                             float* ct) {
  static_assert(comb::scatter_coef_entries<float, NL, BR, BC, R>() <= kMaxCoefEntries, "staging too small");
  comb::stage_scatter_coefs<float, NL, BR, BC, R>(p.lev, ct);
  for (int c = 0; c < count; ++c)
    comb::scatter_block<float, float, float, V, NL, BR, BC, R>(p, ct, first + c, o);
}

template <int PREC, int TILE, int BK>
__device__ __forceinline__ void leaf_task(const LeafDesc& d, int64_t first, int count, void* smem) {
  for (int c = 0; c < count; ++c) {
    if (c) __syncthreads();  // the previous tile's LDS reads are done
    if constexpr (PREC == RBC_PREC_F32)
      tiles::gemm_f32_tile<TILE, TILE, BK>(static_cast<const float*>(d.S), static_cast<const float*>(d.T),
                                           d.P, d.m, d.n, d.k, d.tiles_n, d.tiles_per_leaf, first + c,
                                           static_cast<float*>(smem));
    else if constexpr (PREC == RBC_PREC_FP8C)
      tiles::gemm_fp8c_tile<TILE, TILE>(static_cast<const uint8_t*>(d.S), static_cast<const uint8_t*>(d.T), d.P,
                                        d.m, d.n, d.k, d.plane_s, d.plane_t, d.eS, d.eT, d.tiles_n,
                                        d.tiles_per_leaf, first + c, static_cast<uint8_t*>(smem));
    else
      tiles::gemm_lowp_tile<tiles::LOWP_F16S, TILE, TILE>(
          static_cast<const uint16_t*>(d.S), static_cast<const uint16_t*>(d.T), d.P, d.m, d.n, d.k,
          d.plane_s, d.plane_t, d.eS, d.eT, d.tiles_n, d.tiles_per_leaf, first + c,
          static_cast<uint16_t*>(smem));
  }
}

template <int PREC, int I>
__device__ __forceinline__ void run_gather(int v, const GatherParams& p, int64_t first, int count,
                                           int64_t in, int32_t* exps, float* ct) {
  if constexpr (I < kNumGathers) {
    constexpr CombVariant G = kGathers[I];
    if constexpr (gather_in<PREC>(G)) {
      if (v == I) return gather_task<G.out, G.vec, G.nl, G.br, G.bc, G.R>(p, first, count, in, exps, ct);
    }
    run_gather<PREC, I + 1>(v, p, first, count, in, exps, ct);
  }
}

template <int I>
__device__ __forceinline__ void run_scatter(int v, const ScatterParams& p, int64_t first, int count,
                                            int64_t o, float* ct) {
  if constexpr (I < kNumScatters) {
    constexpr CombVariant S = kScatters[I];
    if (v == I) return scatter_task<S.vec, S.nl, S.br, S.bc, S.R>(p, first, count, o, ct);
    run_scatter<I + 1>(v, p, first, count, o, ct);
  }
}

template <int PREC, int I>
__device__ __forceinline__ void run_leaf(int v, const LeafDesc& d, int64_t first, int count, void* smem) {
  if constexpr (I < kNumLeaves) {
    constexpr LeafVariant L = kLeaves[I];
    if constexpr (L.prec == PREC) {
      if (v == I) return leaf_task<PREC, L.tile, L.bk>(d, first, count, smem);
    }
    run_leaf<PREC, I + 1>(v, d, first, count, smem);
  }
}

__device__ __forceinline__ int32_t load_relaxed(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 only.  True once counter c reaches need; false on abort or time-out
// (the time-out raises the abort flag and records the task).
__device__ __forceinline__ bool wait_for(const int32_t* c, int32_t need, int32_t* ctl, int64_t task,
                                         int64_t timeout) {
  if (load_relaxed(c) >= need) return true;
  const uint64_t t0 = wall_clock64();
  for (uint32_t spins = 0;; ++spins) {
    __builtin_amdgcn_s_sleep(2);
    if (load_relaxed(c) >= need) return true;
    if (load_relaxed(ctl + CTL_ABORT)) return false;
    // wall-clock limit, with a poll-count backstop (each poll sleeps at least 128 cycles)
    if ((int64_t)(wall_clock64() - t0) > timeout || spins >= (1u << 22)) {
      atomicCAS(ctl + CTL_STUCK_TASK, 0, (int32_t)(task + 1));
      __hip_atomic_store(ctl + CTL_ABORT, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
}

// Leader steps of the task loop (thread 0 acts, the others return at once).
// They are kept out of line on purpose: with them inlined, the compiler may
// merge the leader block that ends one iteration with the one that starts
// the next into a single divergent region across the loop's back edge and
// restructure the loop so that the other lanes reach the next barrier without
// the leader, re-reading the previous task.  Called by every thread, the
// functions leave the kernel's loop without any divergent branch.
// With a trace buffer, thread 0 records per task: the wall clock when the
// task was taken, when its dependencies were met, when it was signalled, and
// the workgroup that ran it.
__device__ __noinline__ void leader_pop(int32_t* ctl, int64_t n_tasks, int32_t* slot) {
  if (threadIdx.x == 0) {
    int32_t t = atomicAdd(ctl + CTL_HEAD, 1);
    if (load_relaxed(ctl + CTL_ABORT)) t = (int32_t)n_tasks;
    *slot = t;
  }
}

__device__ __noinline__ void leader_wait(const Task* task, int32_t* ctl, int32_t t, int64_t timeout,
                                         int32_t* slot, uint64_t* trace) {
  if (threadIdx.x == 0) {
    const uint64_t t0 = trace ? wall_clock64() : 0;
    int32_t* cnt = ctl + CTL_WORDS;
    bool ok = true;
    if (task->wait[0] >= 0) ok = wait_for(cnt + task->wait[0], task->need[0], ctl, t, timeout);
    if (ok && task->wait[1] >= 0) ok = wait_for(cnt + task->wait[1], task->need[1], ctl, t, timeout);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *slot = ok;
    if (trace) {
      trace[(int64_t)t * 4 + 0] = t0;
      trace[(int64_t)t * 4 + 1] = wall_clock64();
      trace[(int64_t)t * 4 + 3] = blockIdx.x;
    }
  }
}

__device__ __noinline__ void leader_signal(int32_t* ctl, int32_t t, int32_t signal, int32_t count,
                                           uint64_t* trace) {
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    // The fence writes the L2 back (buffer_wbl2), and the counter may only
    // move once that write-back is done.  The compiler drops the wait that
    // the fence needs after the write-back when no memory operation it
    // tracks is outstanding (the caller has already waited for all of its
    // own), so the wait is spelled out: without it a workgroup on another
    // XCD can see the counter, invalidate its caches and still read the old
    // bytes from memory.
    __builtin_amdgcn_s_waitcnt(0);
    // The update itself is a release operation at agent scope as well, so that
    // the ordering does not rest on the fence and the wait alone.
    if (signal >= 0)
      __hip_atomic_fetch_add(ctl + CTL_WORDS + signal, count, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (trace) trace[(int64_t)t * 4 + 2] = wall_clock64();
  }
}

template <int PREC>
__global__ __launch_bounds__(256, 2) void k_batch(const Task* __restrict__ tasks, int64_t n_tasks,
                                                  const GatherParams* __restrict__ gather,
                                                  const ScatterParams* __restrict__ scatter,
                                                  const LeafDesc* __restrict__ leaf,
                                                  const ScaleDesc* __restrict__ scale_d, int32_t* ctl,
                                                  int64_t timeout_ticks, uint64_t* trace) {
  __shared__ __attribute__((aligned(16))) char smem[Smem<PREC>::bytes];
  __shared__ int32_t s_task;
  __shared__ int32_t s_ok;
  __shared__ int32_t s_exps[kMaxGatherOutputs];
  __shared__ float s_coef[kMaxCoefEntries];
  for (;;) {
    leader_pop(ctl, n_tasks, &s_task);
    __syncthreads();
    // Every thread reads the same value; saying so keeps the task and its
    // parameters in scalar registers.
    const int32_t t = __builtin_amdgcn_readfirstlane(s_task);
    if (t >= n_tasks) break;
    const Task& task = tasks[t];
    leader_wait(&task, ctl, t, timeout_ticks, &s_ok, trace);
    __syncthreads();
    if (!__builtin_amdgcn_readfirstlane(s_ok)) break;
    switch (task.kind) {
      case TK_MAXABS: {
        const ScaleDesc& d = scale_d[task.param];
        scale::maxabs_fold(scale::maxabs_rows(d.X, d.ld, d.cols, task.first, task.count), d.maxbits);
        break;
      }
      case TK_EXPONENTS: {
        const ScaleDesc& d = scale_d[task.param];
        const float mx = __uint_as_float(__hip_atomic_load(d.maxbits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        const gbl<const float>* G = global_ptr(d.G);
        gbl<int32_t>* e = global_ptr(d.e);
        for (int64_t l = threadIdx.x; l < d.n_leaves; l += 256) e[l] = scale::leaf_exponent(mx, G[l], d.target);
        break;
      }
      case TK_GATHER:
        run_gather<PREC, 0>(task.variant, gather[task.param], task.first, task.count, task.sub, s_exps, s_coef);
        break;
      case TK_LEAF:
        run_leaf<PREC, 0>(task.variant, leaf[task.param], task.first, task.count, smem);
        break;
      case TK_SCATTER:
        run_scatter<0>(task.variant, scatter[task.param], task.first, task.count, task.sub, s_coef);
        break;
      default:
        break;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    leader_signal(ctl, t, task.signal, task.count, trace);
  }
}
static __global__ void k_zero_words(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

template <int PREC>
hipError_t occupancy(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch<PREC>, 256, 0);
}

template <int PREC>
hipError_t launch(const KernelArgs& a, int grid, hipStream_t s) {
  int64_t zb = (a.n_ctl + 255) / 256;
  if (zb > 1024) zb = 1024;
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)zb), dim3(256), 0, s, a.ctl, a.n_ctl);
  hipLaunchKernelGGL(k_batch<PREC>, dim3((unsigned)grid), dim3(256), 0, s, a.tasks, a.n_tasks, a.gather,
                     a.scatter, a.leaf, a.scale, a.ctl, a.timeout_ticks, a.trace);
  return hipGetLastError();
}

}  // namespace batch
}  // namespace rbc
