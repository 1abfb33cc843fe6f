// Kernel parameter blocks and launchers shared by the HIP translation units
// and the C ABI.  Parameters travel by value as kernel arguments, so a launch
// copies nothing to the device besides them.
#pragma once

#include <hip/hip_runtime_api.h>

#include "core.hpp"

namespace rbc {

constexpr int kMaxGroupLevels = 3;

// Output formats of a gather.
enum GatherOut { OUT_SAME = 0, OUT_BF16X2 = 1, OUT_F16S = 2, OUT_FP8X2 = 3 };

// Gather of one group: every top block (n_in of them) becomes Rg bottom blocks,
// S = sum over (k, l) of the folded coefficient times block (k, l), level by
// level inside the group.  Element types: double (f64) or float.
struct GatherParams {
  const void* src;
  int64_t ld_src;      // row stride of a top block
  int64_t src_batch;   // elements between consecutive top blocks (0: a single user matrix)
  int64_t src_rows, src_cols;  // readable part of a top block; zero beyond (virtual padding)
  void* dst;
  int64_t rows_bot, cols_bot;  // bottom block size
  int64_t dst_batch;   // elements between consecutive bottom blocks
  int64_t plane;       // bf16x2 / fp8x2 output: elements between the hi and lo planes
  int32_t* scale_exp;   // f16s / fp8 output: power-of-two exponent per bottom block
  // Stand-alone path: the gather derives those exponents itself from the
  // partial maxima of |X| and the per-leaf path norms (writing them to
  // scale_exp for the leaf product); null when scale_exp is filled beforehand.
  const float* scale_partial;
  const float* scale_G;
  int32_t scale_nparts;
  float scale_target;
  int64_t n_in;
  // Streaming (non-temporal) stores, for a group whose output only the next
  // gather group reads.  The leaf operands are written with ordinary stores, so
  // that they stay in the caches for the leaf kernel: against streaming stores,
  // f32 Strassen F-hat^(3) at N = 4096 went from 0.986 to 0.982 ms per product,
  // f16s at Q = 2 from 0.303 to 0.294 ms and the rank-10 APA on bf16 hi+lo
  // leaves at N = 3072 from 0.272 to 0.252 ms (its leaf 0.192 -> 0.176 ms);
  // fp8c at Q = 4, whose first group feeds the second, was 1.4% slower with
  // ordinary stores there.
  int32_t nt_store;
  int32_t side;        // 0: A (U tables), 1: B (V tables)
  SideLevel lev[kMaxGroupLevels];
};

// One gather launch: side a alone (sides = 1), or the A and B sides of a
// level group together (sides = 2; same element type, output, shape and vec).
struct GatherPair {
  GatherParams a, b;
  int sides;
};

// Scatter of one group: Rg bottom blocks per top block are combined through W.
struct ScatterParams {
  const void* src;
  int64_t src_batch;   // elements between consecutive bottom blocks (= rows_bot * cols_bot)
  void* dst;
  int64_t ld_dst;
  int64_t dst_batch;   // elements between consecutive top blocks (0: the user's C)
  int64_t dst_rows, dst_cols;  // writable part of a top block (crop)
  int64_t rows_bot, cols_bot;
  int64_t n_out;
  SideLevel lev[kMaxGroupLevels];
};

// f32 leaf products whose operands are formed while they are loaded: leaf l
// is product r = l % R of parent block l / R of the level above, and its S
// (T) is the sum, over the parent's sub-blocks (k, l) in row-major order, of
// the folded coefficient times the sub-block, as the deepest level's gather
// would have written it (one rounding per multiply and per add).  At most two
// coefficients of any product may be nonzero on either side.
struct LeafGather {
  const float* A;                  // A-side parents: a_batch elements apart, row stride a_ld
  const float* B;
  int64_t a_batch, a_ld, b_batch, b_ld;
  int64_t a_row_blk, a_col_blk;    // element offset of sub-block (1, 0) and of (0, 1) in a parent
  int64_t b_row_blk, b_col_blk;
  SideLevel la, lb;                // the deepest level's A and B sides (f32 tables)
  int32_t bra, bca, brb, bcb, R;
};

// The deepest level's scatter folded into the same launch (leaf scatter): the
// R leaf products of a parent (leaves parent * R + r) are combined through the
// deepest level's folded W into the parent's product block, sub-block (k, l)
// = the sum over r, in order, of the folded coefficient times P_r (one
// rounding per multiply and per add, products with a zero coefficient
// skipped), as that level's scatter would.  A per-parent counter for every
// 64 x 64 region of a leaf counts the leaf tiles stored there; the workgroup
// whose tile brings a region's count to R combines that region.
struct LeafScatter {
  float* out;                // parents' product blocks: out_batch elements apart, row stride out_ld
  int32_t* cnt;              // (m / 64) (n / 64) counters per parent, zero before the launch
  int64_t out_batch, out_ld;
  int64_t row_blk, col_blk;  // element offset of sub-block (1, 0) and of (0, 1) in an out block
  SideLevel lw;              // the deepest level's C side (f32 table)
  int32_t br, bc;            // sub-blocks of an out block (b1 x b3)
};

// Element-type codes for launchers.
enum Elt { ELT_F32 = 0, ELT_F64 = 1 };

// vec: element positions per thread (1, 2 or 4); every pointer, leading
// dimension and block stride of the launch must be a multiple of it.
hipError_t launch_gather(Elt elt, GatherOut out, int vec, int nl, int br, int bc, int R,
                         const GatherParams& p, hipStream_t stream);
// The same for two gathers of one shape in one launch (pb: the second side).
hipError_t launch_gather2(Elt elt, GatherOut out, int vec, int nl, int br, int bc, int R,
                          const GatherParams& pa, const GatherParams& pb, hipStream_t stream);
// tp: product element type, ta: accumulation type, to: output element type
hipError_t launch_scatter(Elt tp, Elt ta, Elt to, int vec, int nl, int br, int bc, int R,
                          const ScatterParams& p, hipStream_t stream);

// Batched leaf products P_l = S_l T_l, l < batch; S: m x k, T: k x n, P: m x n,
// each row-major and contiguous, consecutive leaves back to back.
hipError_t launch_gemm_f32(const float* S, const float* T, float* P, int64_t m, int64_t n, int64_t k,
                           int64_t batch, int tile, hipStream_t stream);
// P (batch leaves of m x n) from operands gathered on the fly (LeafGather);
// with ls, also the parents' product blocks (LeafScatter; its counters are
// cleared by this call, on the stream, before the product).
hipError_t launch_gemm_f32_gathered(const LeafGather& g, float* P, int64_t m, int64_t n, int64_t k,
                                    int64_t batch, int tile, hipStream_t stream,
                                    const LeafScatter* ls = nullptr);
hipError_t launch_gemm_f64(const double* S, const double* T, double* P, int64_t m, int64_t n,
                           int64_t k, int64_t batch, hipStream_t stream);
// Leaves of any size m x k by k x n (no tile padding), f32 or f64 (exact-block plans).
hipError_t launch_gemm_f32_masked(const float* S, const float* T, float* P, int64_t m, int64_t n, int64_t k,
                                  int64_t batch, hipStream_t stream);
hipError_t launch_gemm_f64_masked(const double* S, const double* T, double* P, int64_t m, int64_t n, int64_t k,
                                  int64_t batch, hipStream_t stream);
// bf16x3: S and T hold hi planes followed (plane elements later) by lo planes.
hipError_t launch_gemm_bf16x3(const uint16_t* S, const uint16_t* T, float* P, int64_t m, int64_t n,
                              int64_t k, int64_t batch, int tile, hipStream_t stream);
// f16s: S and T hold f16 leaf operands scaled by 2^eS[l], 2^eT[l]; P is unscaled.
hipError_t launch_gemm_f16s(const uint16_t* S, const uint16_t* T, float* P, int64_t m, int64_t n,
                            int64_t k, int64_t batch, int tile, const int32_t* eS, const int32_t* eT,
                            hipStream_t stream);
// fp8c: S and T hold e4m3 hi planes followed (plane bytes later) by lo planes,
// scaled by 2^eS[l], 2^eT[l]; P = 2^-(eS+eT) (hi hi + (hi lo + lo hi) / 16).
hipError_t launch_gemm_fp8c(const uint8_t* S, const uint8_t* T, float* P, int64_t m, int64_t n, int64_t k,
                            int64_t batch, int tile, const int32_t* eS, const int32_t* eT, hipStream_t stream);
// acc (rows x cols, contiguous f64) = (first ? 0 : acc) + x (row stride ldx), elementwise.
hipError_t launch_accumulate(double* acc, const void* x, Elt elt, int64_t rows, int64_t cols, int64_t ldx,
                             int first, hipStream_t s, double weight = 1.0);
hipError_t launch_scale_f64(double* acc, int64_t n, double scale, hipStream_t s);
// Partial maxima of |X|: maxabs_blocks(rows, cols) floats at `partial`
// (overwritten), at most kScalePartials.  The gather of the leaf operands
// reduces them and derives the per-leaf exponents.
constexpr int kScalePartials = 1024;
inline int maxabs_blocks(int64_t rows, int64_t cols) {
  // at least 32 KB of X per workgroup, at most kScalePartials workgroups
  int64_t b = (rows * cols + 8191) / 8192;
  if (b > kScalePartials) b = kScalePartials;
  if (b > rows) b = rows;
  return (int)(b < 1 ? 1 : b);
}
hipError_t launch_maxabs(const float* X, int64_t ld, int64_t rows, int64_t cols, float* partial, hipStream_t s);
// The same for two matrices in one launch.
hipError_t launch_maxabs2(const float* XA, int64_t lda, int64_t ra, int64_t ca, float* pa, const float* XB,
                          int64_t ldb, int64_t rb, int64_t cb, float* pb, hipStream_t s);

}  // namespace rbc
