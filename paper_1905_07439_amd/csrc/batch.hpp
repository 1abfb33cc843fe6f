// Batch engine: many independent products in one persistent kernel.
//
// The host turns every product of a batch into a list of tasks (a task is a
// few workgroup-sized pieces of one gather, leaf or scatter launch of that
// product, exactly as the single-product path would launch them) and sorts
// them so that every task comes after the tasks it depends on.  The
// persistent kernel's workgroups take tasks in that order from an atomic
// queue head, wait until the dependency counters of the task are complete,
// run it with the same device functions as the stand-alone kernels, and add
// the number of pieces done to the task's completion counter.  Because every
// task's dependencies precede it in the queue, the smallest unfinished task
// that has been taken can always run, so the kernel cannot deadlock; waits
// are additionally bounded by a wall-clock limit that, when exceeded, sets an
// abort flag that makes every workgroup leave.
//
// This header is shared by the host builder (batch.cpp) and the kernel
// (batch.hip): it holds the task layout and the tables of compiled variants.
#pragma once

#include <cstdint>

#include "kernels.hpp"

namespace rbc {
namespace batch {

// TK_GATE does no work: it waits for a product that used the same workspace
// region earlier in the queue and then counts towards the entry of the next.
enum TaskKind : int16_t {
  TK_MAXABS = 0, TK_EXPONENTS = 1, TK_GATHER = 2, TK_LEAF = 3, TK_SCATTER = 4, TK_GATE = 5
};

struct Task {
  int16_t kind;
  int16_t variant;   // index into the variant table of the kind
  int32_t param;     // index into the parameter array of the kind
  int32_t wait[2];   // counter indices (-1: none)
  int32_t need[2];   // value each counter must reach
  int32_t signal;    // counter that receives `count` on completion (-1: none)
  int32_t count;     // pieces (workgroup-sized blocks) this task covers
  int64_t first;     // first piece
  int64_t sub;       // gather: top block index; scatter: output block index
};
static_assert(sizeof(Task) == 48, "task layout");

// Leaf product of one item: pieces are the output tiles of the batched
// leaf GEMM (leaf-major), as in the stand-alone launch without block remap.
struct LeafDesc {
  const void* S;
  const void* T;
  float* P;
  int32_t m, n, k, tiles_n, tiles_per_leaf, pad_;
  int64_t plane_s, plane_t;
  const int32_t* eS;
  const int32_t* eT;
};

// f16s / fp8c operand scale of one item side: a maxabs piece is one row of the
// operand (pieces = rows); the exponent task writes every leaf's exponent.
struct ScaleDesc {
  const float* X;
  int64_t ld, rows, cols;
  uint32_t* maxbits;
  const float* G;
  int32_t* e;
  int64_t n_leaves;
  int64_t pieces;
  float target;        // bound of the scaled operand (2^15 for f16, 448 for e4m3)
  int32_t level_rows;  // rows per workgroup in the level-synchronous mode
};

struct CombVariant {
  int out, vec, nl, br, bc, R;
};
struct LeafVariant {
  int prec, tile, bk;
};

// Compiled gather variants (float elements).  Positions per thread are 4 or
// 1; a launch whose alignment allows only 2 runs with 1, which computes the
// same values (every output element's sum is independent of the others).
constexpr CombVariant kGathers[] = {
    {OUT_SAME, 4, 1, 3, 3, 23}, {OUT_SAME, 1, 1, 3, 3, 23}, {OUT_SAME, 4, 1, 2, 2, 7},
    {OUT_SAME, 1, 1, 2, 2, 7},  {OUT_SAME, 4, 2, 2, 2, 7},  {OUT_SAME, 1, 2, 2, 2, 7},
    {OUT_F16S, 4, 1, 3, 3, 23}, {OUT_F16S, 1, 1, 3, 3, 23}, {OUT_F16S, 4, 1, 2, 2, 7},
    {OUT_F16S, 1, 1, 2, 2, 7},  {OUT_F16S, 4, 2, 2, 2, 7},  {OUT_F16S, 1, 2, 2, 2, 7},
    {OUT_FP8X2, 4, 1, 3, 3, 23}, {OUT_FP8X2, 1, 1, 3, 3, 23}, {OUT_FP8X2, 4, 1, 2, 2, 7},
    {OUT_FP8X2, 1, 1, 2, 2, 7},  {OUT_FP8X2, 4, 2, 2, 2, 7},  {OUT_FP8X2, 1, 2, 2, 2, 7},
};
// Compiled scatter variants (float products, accumulation and output).  Two
// fused levels keep 16 accumulators per position, so they run with at most
// 2 positions per thread to bound the kernel's register budget.
constexpr CombVariant kScatters[] = {
    {OUT_SAME, 4, 1, 3, 3, 23}, {OUT_SAME, 1, 1, 3, 3, 23}, {OUT_SAME, 4, 1, 2, 2, 7},
    {OUT_SAME, 1, 1, 2, 2, 7},  {OUT_SAME, 2, 2, 2, 2, 7},  {OUT_SAME, 1, 2, 2, 2, 7},
};
// Compiled leaf variants: (precision, square tile, K slab).  The tile edge
// does not change any output element's summation order (that is fixed by the
// K slab), so f32 leaves run with 64 x 64 tiles and fp8c leaves of a 128-tile
// plan with 64 x 64 tiles in the batch kernel, which keeps its register budget.
constexpr LeafVariant kLeaves[] = {
    {RBC_PREC_F32, 64, 32}, {RBC_PREC_F32, 64, 16},
    {RBC_PREC_F16S, 128, 32}, {RBC_PREC_F16S, 96, 32}, {RBC_PREC_F16S, 64, 32}, {RBC_PREC_F16S, 32, 32},
    {RBC_PREC_FP8C, 96, 64},  {RBC_PREC_FP8C, 64, 64}, {RBC_PREC_FP8C, 32, 64},
};
constexpr int kNumGathers = sizeof(kGathers) / sizeof(kGathers[0]);
constexpr int kNumScatters = sizeof(kScatters) / sizeof(kScatters[0]);
constexpr int kNumLeaves = sizeof(kLeaves) / sizeof(kLeaves[0]);

// Control words at the start of the counter array.
enum Control { CTL_HEAD = 0, CTL_ABORT = 1, CTL_STUCK_TASK = 2, CTL_WORDS = 4 };

struct KernelArgs {
  const Task* tasks;
  int64_t n_tasks;
  const GatherParams* gather;
  const ScatterParams* scatter;
  const LeafDesc* leaf;
  const ScaleDesc* scale;
  int32_t* ctl;            // CTL_WORDS control words, then the counters
  int64_t n_ctl;           // words zeroed before every run (control + counters)
  int64_t timeout_ticks;   // wall-clock limit of one dependency wait
  uint64_t* trace;         // null, or 4 words per task (taken, ready, done, workgroup)
};

// Host side of the kernel (batch_*.hip).  prec selects the kernel instance:
// RBC_PREC_F32, RBC_PREC_F16S or RBC_PREC_FP8C.
hipError_t batch_occupancy(int prec, int* blocks_per_cu);
hipError_t launch_batch(int prec, const KernelArgs& a, int grid, hipStream_t stream);
// Level-synchronous groups (batch_group.hpp): one workgroup per entry.
struct PieceRef;
struct GroupArgs;
hipError_t launch_group(int prec, int kind, int variant, const Task* tasks, const void* pieces,
                        const GatherParams* gather, const ScatterParams* scatter, const LeafDesc* leaf,
                        const ScaleDesc* scale, int64_t grid, hipStream_t stream);
// Zero n control words (the counters, and the f16s/fp8c max|X| words).
hipError_t launch_zero_words(int32_t* p, int64_t n, hipStream_t stream);

}  // namespace batch
}  // namespace rbc
