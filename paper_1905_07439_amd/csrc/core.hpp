// Host core of librbc: schemes, draws, fold and plans.  Plain C++17: no HIP
// types appear here, so the planner and the validator build and run on any
// host.  The device side (kernels.hpp) consumes the descriptors defined here.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rbc.h"

namespace rbc {

constexpr int kMaxB = 4;     // block partition per level and dimension
constexpr int kMaxR = 64;    // products per level
constexpr int kMaxLevels = RBC_MAX_LEVELS;

// ---- errors ---------------------------------------------------------------
rbc_status fail(rbc_status st, const char* fmt, ...);
void clear_error();

// ---- schemes (Section 1, Definition 1, eq. epsilon-def) -------------------
struct Scheme {
  int b1 = 0, b2 = 0, b3 = 0, R = 0;
  std::vector<double> U, V, W;  // [b1][b2][R], [b2][b3][R], [b1][b3][R]
  bool integral = false;        // every entry an integer (exact validation)
  double tau = 0, kappa = 0, ynorm = 0, q = 0;
  double kappa_total = 0;       // sum_{i,l,j} (1 - sum_r u v w); kappa = total / (b1 b2 b3)
};

// Fill tau, kappa, ynorm, q by brute force over the index 6-tuples.
void analyse(Scheme& s);
rbc_status make_scheme(int b1, int b2, int b3, int R, const double* U, const double* V,
                       const double* W, double residual_tol, Scheme& out);
rbc_status builtin_scheme(const char* name, double lambda, uint64_t aux_seed, Scheme& out);

// ---- draws (Section 2.1) ----------------------------------------------------
void philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
// signs and perms receive b1 + b2 + b3 entries each.
void draw_level(uint64_t seed, int depth, int b1, int b2, int b3, rbc_mode mode, int32_t* signs,
                int32_t* perms);
bool valid_draw(int b1, int b2, int b3, const int32_t* signs, const int32_t* perms);

// (1 - kappa)^-1 exactly as 1.0 / (1.0 - kappa) in double.
double kappa_factor(const Scheme& s);
void fold(const Scheme& s, const int32_t* signs, const int32_t* perms, bool kappa_scale,
          double* Uh, double* Vh, double* Wh);

// ---- plans (Section 2.1.1) --------------------------------------------------
// One side (A, B or C) of one level as the kernels see it: block-row and
// block-column signs and permutations and the product count.  The folded
// coefficient of block (k, l), product r, is
//   tab[(pr[k] * BC + pc[l]) * R + r] * sr[k] * sc[l].
struct SideLevel {
  int8_t pr[kMaxB], pc[kMaxB];
  int8_t sr[kMaxB], sc[kMaxB];
  int32_t R;
  int32_t strassen;  // the table's nonzero entries are Strassen's: kStrassenUNz (A side), kStrassenVNz (B), kStrassenWNz (C)
  const void* tab;  // device table of this side (f64 or f32, see Plan)
};

// Nonzero products of each 2 x 2 output block (11, 12, 21, 22) in Strassen's W,
// the form of Golub & Van Loan: C11 = P1 + P4 - P5 + P7, C12 = P3 + P5,
// C21 = P2 + P4, C22 = P1 - P2 + P3 + P6 (0-based, padded with -1).  Scatters
// over tables with exactly this pattern skip the zero terms at compile time.
constexpr int kStrassenWNz[4][4] = {{0, 3, 4, 6}, {2, 4, -1, -1}, {1, 3, -1, -1}, {0, 1, 2, 5}};
constexpr int kStrassenWNzCount[4] = {4, 2, 2, 4};
// Nonzero blocks (11, 12, 21, 22) of each product in the same form's U and V:
// P1 = (A11 + A22)(B11 + B22), P2 = (A21 + A22) B11, P3 = A11 (B12 - B22),
// P4 = A22 (B21 - B11), P5 = (A11 + A12) B22, P6 = (A21 - A11)(B11 + B12),
// P7 = (A12 - A22)(B21 + B22); at most two, padded with -1.
constexpr int kStrassenUNz[7][2] = {{0, 3}, {2, 3}, {0, -1}, {3, -1}, {0, 1}, {0, 2}, {1, 3}};
constexpr int kStrassenVNz[7][2] = {{0, 3}, {0, -1}, {1, 3}, {0, 2}, {3, -1}, {0, 1}, {2, 3}};

// Consecutive levels that one kernel pass fuses.  All levels of a group share
// the block shape <b1, b2, b3>.  "top" blocks enter the group from above (the
// user's A/B/C for group 0), "bot" blocks are the group's leaves (the leaf
// operands and products for the last group).
struct Group {
  int d0 = 0, d1 = 0;             // levels [d0, d1)
  int b1 = 0, b2 = 0, b3 = 0;
  int64_t n_in = 1;               // subproblems entering the group = prod_{d < d0} R_d
  int64_t Rg = 1;                 // prod_{d0 <= d < d1} R_d
  int64_t a_rows_top = 0, a_cols_top = 0, a_rows_bot = 0, a_cols_bot = 0;
  int64_t b_rows_top = 0, b_cols_top = 0, b_rows_bot = 0, b_cols_bot = 0;
  int64_t c_rows_top = 0, c_cols_top = 0, c_rows_bot = 0, c_cols_bot = 0;
  // Workspace byte offsets of the bottom-side buffers: gathered A side,
  // gathered B side, and the products the scatter of this group reads.
  size_t off_a_bot = 0, off_b_bot = 0, off_c_bot = 0;
};

struct LevelTables {  // host copies, uploaded once per device
  std::vector<double> U, V, W, Wk;  // Wk = (1 - kappa)^-1 * W (double product)
  std::vector<float> Uf, Vf, Wf, Wkf;
};

// Byte offset of the per-leaf exponents in the auxiliary workspace: after
// 1024 partial maxima for each of A and B.
constexpr size_t kAuxExpOffset = 2 * 1024 * sizeof(float);

struct Plan {
  int64_t M = 0, K = 0, N = 0, Mp = 0, Kp = 0, Np = 0, mM = 0, mK = 0, mN = 0;
  int64_t n_leaves = 1;
  int Q = 0;
  rbc_prec prec = RBC_PREC_F32;
  int tile_m = 0, tile_n = 0, tile_k = 0;
  // Exact blocks (leaf_tile = -1): the recursion's blocks are those of the
  // unpadded problem (padding only to a multiple of the block counts), and the
  // leaves, of any size, run through the masked leaf kernels.
  bool exact_blocks = false;
  std::vector<Scheme> levels;
  std::vector<LevelTables> tables;
  std::vector<Group> groups;
  size_t ws_bytes = 0, off_S = 0, off_T = 0, off_P = 0, bytes_S = 0, bytes_T = 0, bytes_P = 0;
  // f16s, fp8c: auxiliary workspace (partial maxima of |A| and |B|, then the
  // per-leaf exponents at kAuxExpOffset) and the per-leaf path norms G of the A
  // and B sides (product over levels of coefficient 1-norms)
  size_t off_aux = 0, bytes_aux = 0;
  std::vector<float> gA, gB;
  size_t g_off[2] = {0, 0};
  // element sizes: combination precision (gather side), recombination (scatter side)
  int comb_bytes = 4, recomb_bytes = 4;
  // Leaf gather: an f32 plan of two or more levels whose deepest scheme has at
  // most two nonzero coefficients per product in U and in V can form its leaf
  // operands inside the leaf product, from the blocks of the level above.
  // fgroups then gather levels [0, Q - 1) (the last one's bottom blocks, the
  // parents of the leaves, at off_S and off_T when they fit there); the stage
  // calls and the batch engine keep the separate gather of every level.
  // Scatter passes of rbc_matmul and the stage calls: as `groups`, but up to
  // three Strassen-shaped levels per pass (k_scatter3, one pass where two
  // would write and re-read the blocks between them).  The gathers and the
  // batch engine keep `groups`.  Boundary buffers are those of `groups` where
  // a boundary coincides, else unused ones of `groups` or new ones.
  std::vector<Group> sgroups;
  bool fuse_max = false;         // fuse levels regardless of the pass's parallel work
  bool leaf_gather_ok = false;   // the plan qualifies
  bool leaf_gather = false;      // rbc_matmul takes that path
  std::vector<Group> fgroups;
  // Leaf scatter (with the leaf gather): the leaf product also combines the
  // deepest level's products into the parents' product blocks (off_pc), and
  // the scatter passes run over fgroups.  Counters at off_cnt, n_cnt of them.
  // Those regions are laid out (off_cnt != 0) when it is first turned on.
  bool leaf_scatter_ok = false;
  bool leaf_scatter = false;
  size_t off_pc = 0, off_cnt = 0;
  int64_t n_cnt = 0;

  // device state, created on first use (see device.cpp)
  int device = -1;
  void* dev_tables = nullptr;  // one allocation holding every level's tables
  std::vector<size_t> tab_off;   // per level: offsets of U, V, W, Wk (double) then Uf, Vf, Wf, Wkf
  // timing
  bool timing = false;
  std::vector<void*> events;     // hipEvent_t, 5 per recorded call
  int64_t recorded = 0;
};

// The leaf scatter's workspace regions (appended to the plan's workspace on first use).
void layout_leaf_scatter(Plan& p);

// Is a fused group of `nl` levels of shape <b1,b2,b3> with R products compiled?
bool fused_supported(int b1, int b2, int b3, int R, int nl);

// fuse_max: fuse up to the most levels per pass even where a pass has little
// parallel work (for batches, where many products share the GPU).
rbc_status make_plan(int64_t M, int64_t K, int64_t N, const std::vector<Scheme>& levels,
                     rbc_prec prec, int leaf_tile, Plan& out, bool fuse_max = false);

// Table index helpers into Plan::tab_off (per level, 8 entries).
enum TabKind { TAB_U = 0, TAB_V = 1, TAB_W = 2, TAB_WK = 3 };

}  // namespace rbc
