/*
 * rbc.h -- C ABI of librbc: matrix multiplication by randomized (approximate)
 * bilinear computation on AMD MI355X (gfx950).
 *
 * Method: Malik & Becker, "Randomization of Approximate Bilinear Computation
 * for Matrix Multiplication".  A bilinear computation (BC) with tensors
 * (U, V, W) computes C = A B blockwise (Section 1, eqs. bilinear-computation
 * and bilinear-computation-block); it is randomized by signed block
 * permutations (Definition 2, eq. f-hat-def) and applied recursively, one
 * draw per level, with a standard product at the leaves
 * (Section 2.1.1, eq. recursive-random-formula).  The library evaluates the
 * folded form of eq. randomized-algorithm (proof of Proposition 10): the
 * signs and permutations are folded into the coefficients, so randomization
 * moves no data.
 *
 * Conventions shared by every call:
 *   - Every function returns rbc_status; no C++ exception crosses the ABI.
 *     On error, rbc_last_error() returns a thread-local message.
 *   - Scheme tensors are row-major doubles: U[b1][b2][R] (U[k][l][r] weights
 *     block A_kl in product r), V[b2][b3][R], W[b1][b3][R].
 *   - Matrices are row-major.  A is M x K with leading dimension lda >= K,
 *     B is K x N (ldb >= N), C is M x N (ldc >= N).  A, B, C and the
 *     workspace are DEVICE pointers owned by the caller; they must not alias.
 *   - Element type: double for RBC_PREC_F64, float for every other precision.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is enqueued asynchronously on it; argument and plan errors
 *     are reported synchronously; device faults surface at the next
 *     synchronizing call as RBC_EHIP.
 *   - Draw arrays: for a plan with Q levels, `signs` and `perms` hold, per
 *     level from the top, b1 + b2 + b3 entries: s1[0..b1) s2[0..b2) s3[0..b3)
 *     (+1/-1) and pi1 pi2 pi3 (0-based permutations).
 *   - Determinism: the same (plan, inputs, draws) give bitwise identical C.
 */
#ifndef RBC_H
#define RBC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RBC_ABI_VERSION 2
#define RBC_MAX_LEVELS 8

typedef enum {
  RBC_OK = 0,
  RBC_EINVAL = 1,       /* bad argument, shape or pointer */
  RBC_ESCHEME = 2,      /* scheme residual above tolerance, or |1 - kappa| too small */
  RBC_ENOMEM = 3,       /* workspace too small, or host allocation failed */
  RBC_EHIP = 4,         /* a HIP runtime call failed (message in rbc_last_error) */
  RBC_EUNSUPPORTED = 5, /* valid request this build does not implement */
  RBC_EBUSY = 6         /* a shared resource is in use by another host thread; retry later */
} rbc_status;

/* Randomization modes (Section 3.2: fully randomized, random sign, random
 * permutation; "none" is the deterministic F^(Q) of Section 3). */
typedef enum {
  RBC_MODE_FULL = 0,
  RBC_MODE_SIGNS = 1,
  RBC_MODE_PERMS = 2,
  RBC_MODE_NONE = 3
} rbc_mode;

/* Leaf precision.  The block combinations (S_r, T_r, and the W-recombination)
 * run in the element type's precision, except where noted. */
typedef enum {
  RBC_PREC_F64 = 0,    /* f64 everywhere; leaves on v_mfma_f64 */
  RBC_PREC_F32 = 1,    /* f32 everywhere; leaves on v_mfma_f32 */
  RBC_PREC_BF16X3 = 2, /* f32 combinations; leaf operands split hi+lo in bf16,
                          3 bf16 MFMA products with f32 accumulation; the
                          W-recombination in f64, C rounded to f32 */
  RBC_PREC_F16S = 3,   /* f32 combinations; each leaf operand scaled by a power
                          of two (from max|A| or max|B| and the coefficient
                          1-norms along its path, so that |2^e S| <= 2^15) and
                          rounded to f16; f16 MFMA with f32 accumulation, the
                          product unscaled exactly; f32 W-recombination */
  RBC_PREC_FP8C = 4    /* f32 combinations; each leaf operand scaled as for
                          f16s but to |2^e S| <= 448, then split into OCP e4m3
                          hi = rn(2^e S) and lo = rn(16 (2^e S - hi)); fp8 MFMA
                          with f32 accumulation of hi*hi and, in one correction
                          pass, hi*lo + lo*hi (weighted 1/16); the product
                          unscaled exactly; f32 W-recombination */
} rbc_prec;

typedef struct rbc_scheme_s* rbc_scheme;
typedef struct rbc_plan_s* rbc_plan;
typedef struct rbc_batch_s* rbc_batch;

/* Plan geometry, see rbc_plan_get_info. */
typedef struct {
  int64_t M, K, N;          /* problem size */
  int64_t Mp, Kp, Np;       /* zero-padded size (end of Section 2.1.1) */
  int64_t mM, mK, mN;       /* leaf block: S is mM x mK, T is mK x mN */
  int64_t n_leaves;         /* prod_d R_d */
  int32_t levels;           /* Q */
  int32_t n_groups;         /* fused level groups of the gathers (and of the batch engine's scatters) */
  int32_t prec;             /* rbc_prec */
  int32_t tile_m, tile_n, tile_k;  /* leaf GEMM tile */
  size_t workspace_bytes;   /* minimum workspace for rbc_matmul */
  size_t off_S, off_T, off_P;      /* byte offsets of the leaf operands and products */
  size_t bytes_S, bytes_T, bytes_P;
  size_t off_aux, bytes_aux;       /* RBC_PREC_F16S, RBC_PREC_FP8C: partial maxima of |A| and of
                                      |B| (1024 f32 each, scratch), then at off_aux + 8192 the
                                      per-leaf exponents of S and of T (n_leaves int32 each) */
  int32_t n_scatter_groups; /* scatter passes of rbc_matmul and rbc_stage_scatter: up to three
                               2x2x2, rank-7 levels share one where the pass has enough work */
} rbc_plan_info;

const char* rbc_status_str(rbc_status s);
/* Thread-local text of the last error on this thread ("" if none). */
const char* rbc_last_error(void);
int rbc_abi_version(void);

/* ---- schemes (Section 1; Definition 1; eq. epsilon-def) ---------------- */

/* Copy (U, V, W) into a new immutable scheme and validate it: the Brent
 * residual tau = ||Y - X||_F is computed by brute force over every index
 * 6-tuple (eq. requirement; exactly, in 64-bit integers, when every entry is
 * an integer).  Fails with RBC_ESCHEME when tau > residual_tol or when
 * |1 - kappa| < 1e-12 (Definition 2 needs kappa != 1).  Pass
 * residual_tol = INFINITY to accept approximate schemes (ABCs).
 * Limits: 1 <= b1, b2, b3 <= 4, 1 <= R <= 64. */
rbc_status rbc_scheme_create(int b1, int b2, int b3, int R, const double* U, const double* V,
                             const double* W, double residual_tol, rbc_scheme* out);
/* Builtin schemes, by family name; `lambda` and `aux_seed` parameterise the
 * approximate families and must both be 0 for the exact ones.
 *   Exact (Brent residual 0, validated in integers):
 *     "strassen"  rank 7, <2,2,2> (Strassen 1969 in the form of Golub & Van Loan);
 *     "laderman"  rank 23, <3,3,3> (Laderman 1976);
 *     "naive:b1,b2,b3"  the standard algorithm as a BC, R = b1 b2 b3.
 *   Approximate, APA family (Section 1, eq. APA-y: the residual is O(lambda)
 *   with no constant term and W holds 1/lambda coefficients), 0 < lambda <= 1:
 *     "apa322"  rank 10 for <3,2,2> (two five-product formulas for a 2x2
 *               problem missing one block of A, after Bini et al. 1979);
 *     "apa223", "apa232"  its cyclic rotations (<2,2,3>, <2,3,2>).  The three
 *               as consecutive levels form one step of a rank-1000 approximate
 *               scheme for 12x12 blocks.  Rounding errors of the leaf products
 *               grow like 1/lambda per APA level.
 *   Approximate, perturbed exact schemes (Section 3.1), 0 <= lambda <= 1:
 *     "perturbed_strassen", "perturbed_laderman": each of U, V, W gets i.i.d.
 *     N(0, sigma^2) noise, sigma = lambda, on every entry equal to +1 and on 5
 *     entries equal to 0 drawn uniformly without replacement.  The random
 *     numbers are a fixed function of aux_seed: Philox4x64-10 with key
 *     (aux_seed, 1), blocks at counters (1,0,0,0), (2,0,0,0), ..., words in
 *     order; per tensor (U, V, W): one normal per +1 entry in row-major order,
 *     then 5 picks among the zero entries (row-major list, partial Fisher-Yates:
 *     for i = 0..4, j = i + floor(word (nz - i) / 2^64), swap entries i and j
 *     of the list), then one normal per pick in pick order.  A word gives
 *     u = (floor(word / 2^12) + 1/2) 2^-52; a normal is the Box-Muller value
 *     sqrt(-2 ln u1) cos(2 pi u2) of two consecutive words (libm log, cos,
 *     sqrt); an entry x becomes fl(x + fl(sigma z)).
 * Errors: RBC_EINVAL for an unknown name or a lambda / aux_seed out of range. */
rbc_status rbc_scheme_builtin(const char* name, double lambda, uint64_t aux_seed, rbc_scheme* out);
/* dims = {b1, b2, b3, R}; tau (Definition 1), kappa (eq. epsilon-def),
 * ||Y||_F (eq. def-y), q = sqrt(sum_r ||U_r||^2 ||V_r||^2 ||W_r||^2)
 * (eq. square-root-of-sum).  Any output pointer may be NULL. */
rbc_status rbc_scheme_info(rbc_scheme s, int dims[4], double* tau, double* kappa, double* ynorm,
                           double* q);
/* Copy the tensors out (buffers sized b1*b2*R, b2*b3*R, b1*b3*R). */
rbc_status rbc_scheme_tensors(rbc_scheme s, double* U, double* V, double* W);
void rbc_scheme_destroy(rbc_scheme s);

/* ---- draws and fold (Section 2.1; Definition 2; Prop. 10) --------------- */

/* The draw of level `depth` (0 = outermost) for `seed`: Philox4x64-10 (Salmon
 * et al. 2011) with key (seed, 0) and counters (j+1, depth, 0, 0), j = 0, 1,
 * ...; one 64-bit word per sign (s = +1 iff the top bit is 0) for
 * s1, s2, s3, then Fisher-Yates from the identity for pi1, pi2, pi3
 * (i = b-1..1: j = floor(word (i+1) / 2^64), swap p[i], p[j]).  Mode SIGNS
 * sets pi = id, PERMS sets s = 1, NONE both; all words are consumed in every
 * mode.  signs and perms receive b1 + b2 + b3 entries each. */
rbc_status rbc_draw(uint64_t seed, int depth, int b1, int b2, int b3, rbc_mode mode, int32_t* signs,
                    int32_t* perms);
/* Folded tensors of eq. randomized-algorithm for one draw:
 *   Uh[k][l][r] = U[pi1(k)][pi2(l)][r] s1(k) s2(l)
 *   Vh[k][l][r] = V[pi2(k)][pi3(l)][r] s2(k) s3(l)
 *   Wh[i][j][r] = c s1(i) s3(j) W[pi1(i)][pi3(j)][r],  c = (1 - kappa)^-1 if
 *   kappa_scale, else 1. */
rbc_status rbc_fold(rbc_scheme s, const int32_t* signs, const int32_t* perms, int kappa_scale,
                    double* Uh, double* Vh, double* Wh);

/* ---- plans (Section 2.1.1) ----------------------------------------------- */

/* Plan C = F-hat^(Q)(A, B) for an M x K by K x N product with `levels`
 * schemes, top level first (the scheme objects may be destroyed after the
 * call).  The leaf block sizes are the padded sizes divided by
 * prod b1, prod b2, prod b3, rounded up to the leaf GEMM tile; A and B are
 * zero padded virtually (never copied).  leaf_tile = 0 picks the tile
 * automatically; otherwise it is the square tile edge (f32, bf16x3: 64 or
 * 128; f16s, fp8c: 32, 64, 96 or 128; f64: 16).  levels may be 0 (plain product by the leaf kernel).
 * leaf_tile = -1 (f32 and f64 only; RBC_EUNSUPPORTED otherwise) asks for exact blocks: the
 * padding is only to a multiple of prod b1, prod b2, prod b3, so the recursion splits
 * the matrices exactly as the unpadded problem (an N = 320 product with five Strassen
 * levels has leaves of 10 x 10), and the leaves, of any size, run on a kernel that
 * masks the edges of its 16 x 16 tiles (small leaves; no leaf gather). */
rbc_status rbc_plan_create(int64_t M, int64_t K, int64_t N, int levels, const rbc_scheme* schemes,
                           rbc_prec prec, int leaf_tile, rbc_plan* out);
rbc_status rbc_plan_get_info(rbc_plan p, rbc_plan_info* info);
/* Algorithmic HBM bytes of one rbc_matmul, per stage: bytes[0] gathers of A,
 * bytes[1] gathers of B (with the max|X| pass of f16s), bytes[2] leaf
 * products (S and T read once, P written once; with the leaf gather on, the
 * parent blocks read once instead of S and T), bytes[3] scatters.  Every
 * stage counts each element it must read and write once: the readable part
 * of a top block (virtual padding is never read), every bottom block, and the
 * writable part of C. */
rbc_status rbc_plan_traffic(rbc_plan p, double bytes[4]);
/* Leaf gather (eq. recursive-random-formula, deepest level).  For an
 * RBC_PREC_F32 plan of two or more levels whose deepest scheme has at most two
 * nonzero coefficients per product in U and in V (Strassen), rbc_matmul can
 * form the leaf operands S and T inside the leaf product: each leaf tile
 * loads the (at most two) sub-blocks of its parent block that its folded
 * coefficients select and combines them as the deepest level's gather would,
 * in the same order with one rounding per multiply and add, so C is the same
 * to the bit.  The leaf operands are then never written to or read from HBM;
 * the workspace size and the stage calls are the same either way (the stage
 * calls always gather every level).  By default it is on where a cost
 * model predicts a gain (the gathers' saved HBM bytes at 5 TB/s against a 9%
 * slower leaf product: on for N = 4096 with three or four Strassen levels,
 * off with two); RBC_LEAF_GATHER=1 (=0) in the environment turns it on (off)
 * for every new plan that qualifies.
 * set: on = 0 returns to separate gathers; on != 0 fails with
 * RBC_EUNSUPPORTED for a plan that does not qualify.  get: whether it is on
 * and whether the plan qualifies (either pointer may be NULL). */
rbc_status rbc_plan_set_leaf_gather(rbc_plan p, int on);
/* Level fusion (how the recursion's levels are grouped into combination passes).
 * By default (fuse_max = 0) two levels share a pass only when that pass has at
 * least 2^18 elements of parallel work (top blocks entering it x elements of a
 * bottom block); smaller products take one pass per level, which is faster for
 * them alone.  fuse_max = 1 fuses wherever the shapes allow (for batches: many
 * products share the GPU, and fewer, larger tasks pay).  Changing it re-lays
 * out the workspace (query rbc_plan_get_info again) and resets the leaf
 * gather and the leaf scatter to their defaults; the results are the same either
 * way. */
rbc_status rbc_plan_set_fusion(rbc_plan p, int fuse_max);
rbc_status rbc_plan_get_leaf_gather(rbc_plan p, int* on, int* available);
/* Leaf scatter (eq. recursive-random-formula, the W side of the deepest level).
 * With the leaf gather on, rbc_matmul can also fold the deepest level's scatter
 * into the leaf product's launch: the workgroup that stores the last of a
 * parent's R leaf tiles over a 64 x 64 region combines that region of the R
 * products through the deepest level's folded W (in order over r, one rounding
 * per multiply and add, zero coefficients skipped) into the parent's product
 * block, and the scatter passes then start one level up.  C is the same to the
 * bit.  The plan qualifies with the leaf gather (leaf sides multiples of 64).
 * Turning it on the first time appends to the plan's workspace the parents'
 * product blocks and one int32 counter per parent and 64 x 64 region (query
 * rbc_plan_get_info's ws_bytes again; it stays that size).  Each
 * leaf tile then ends with an agent-scope release (an L2 write-back on gfx950),
 * which with the combinations costs more than the scatter pass it saves, so it
 * is off by default; RBC_LEAF_SCATTER=1 in the environment turns it on for
 * every new plan that takes the leaf gather.
 * set: on != 0 fails with RBC_EUNSUPPORTED unless the plan qualifies and its
 * leaf gather is on; turning the leaf gather off turns it off.  get: whether it
 * is on and whether the plan qualifies (either pointer may be NULL). */
rbc_status rbc_plan_set_leaf_scatter(rbc_plan p, int on);
rbc_status rbc_plan_get_leaf_scatter(rbc_plan p, int* on, int* available);
void rbc_plan_destroy(rbc_plan p);

/* ---- products ------------------------------------------------------------ */

/* C = F-hat^(Q)(A, B) with the draws of (seed, mode) for every level.
 * kappa_scale: multiply by (1 - kappa)^-1 at every level (eq.
 * recursive-random-formula); exact schemes have kappa = 0.
 * workspace: device buffer of at least info.workspace_bytes, 256-byte
 * aligned, used for the leaf operands and products; it must not be used by
 * another call until this one has completed on the stream. */
rbc_status rbc_matmul(rbc_plan p, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                      int64_t ldc, uint64_t seed, rbc_mode mode, int kappa_scale, void* workspace,
                      size_t ws_bytes, void* stream);
/* Same, with explicit draws (host arrays, layout above). */
rbc_status rbc_matmul_draws(rbc_plan p, const void* A, int64_t lda, const void* B, int64_t ldb,
                            void* C, int64_t ldc, const int32_t* signs, const int32_t* perms,
                            int kappa_scale, void* workspace, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): rbc_matmul with the
 * workspace taken from a fixed device array of RBC_NOALLOC_MAX_WORKSPACE bytes
 * inside the library, instead of a caller's buffer.  Same kernels, so C is
 * bitwise that of rbc_matmul with the same arguments.  Nothing is allocated:
 * every device that runs the library holds one copy of the array until the
 * process ends.  Calls on one device share that copy: calls that overlap on
 * one device (two streams, two host threads) race and give wrong results;
 * serialize them (one stream).  Every call writes each workspace byte it
 * reads, so what an earlier call left there does not matter.
 * Errors (nothing launched): RBC_EINVAL for a plan whose workspace_bytes
 * exceed RBC_NOALLOC_MAX_WORKSPACE, a plan whose coefficient tables are not
 * on the current device yet (a plan's first rbc_matmul on a device uploads
 * them, allocating once: run it once before), a plan with stage timing on,
 * a bad mode or the argument errors of rbc_matmul. */
#define RBC_NOALLOC_MAX_WORKSPACE ((size_t)64 << 20)
rbc_status rbc_matmul_noalloc(rbc_plan p, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                              int64_t ldc, uint64_t seed, rbc_mode mode, int kappa_scale, void* stream);

/* ---- averages of several products (Section 3, error of average) -----------
 * Cavg = (1/K) sum_k F-hat_k(A, B), F-hat_k with the draws of (seeds[k], mode),
 * accumulated elementwise in f64 in the order k = 0, 1, ..., K-1 (Cavg: device,
 * M x N contiguous f64; seeds: host array of K).  The workspace holds the plan's
 * workspace and one product (rbc_average_workspace bytes). */
rbc_status rbc_average_workspace(rbc_plan p, size_t* bytes);
rbc_status rbc_matmul_average(rbc_plan p, const void* A, int64_t lda, const void* B, int64_t ldb, double* Cavg,
                              const uint64_t* seeds, int64_t K, rbc_mode mode, int kappa_scale, void* workspace,
                              size_t ws_bytes, void* stream);
/* acc (rows x cols, contiguous f64, device) = (first ? 0 : acc) + X elementwise;
 * X is f64 (x_is_f64) or f32 with row stride ldx.  Building block for averages
 * over explicit draws. */
rbc_status rbc_accumulate(double* acc, const void* X, int x_is_f64, int64_t rows, int64_t cols, int64_t ldx,
                          int first, void* stream);
/* acc = (first ? 0 : acc) + weight * X elementwise, otherwise as rbc_accumulate
 * (rbc_accumulate is weight = 1).  Error: RBC_EINVAL for a null pointer, a bad
 * shape or a weight that is not finite. */
rbc_status rbc_accumulate_weighted(double* acc, const void* X, int x_is_f64, int64_t rows, int64_t cols,
                                   int64_t ldx, double weight, int first, void* stream);

/* ---- exact product from an approximate scheme (Section 1, eq. APA-to-EBC) --
 * An approximate scheme's product Y(eps) differs from A B by a polynomial in eps
 * with zero constant term; with d + 1 distinct values the weighted sum
 * sum_i alpha_i Y(eps_i) is exact when that degree is at most d.
 *
 * rbc_apa_ebc_weights: alpha[0..n-1] (host) for eps[0..n-1] (host, distinct,
 * nonzero, finite, 1 <= n <= RBC_EBC_MAX_VALUES): the solution of
 * sum_i alpha_i = 1, sum_i alpha_i eps_i^k = 0 for k = 1..n-1.
 *
 * rbc_matmul_apa_ebc: C (device, M x N contiguous f64) = sum_i alpha_i F-hat_i(A, B),
 * F-hat_i from plans[i] (host array of n plans), whose schemes are the
 * approximate scheme at eps[i]: all plans share M, K, N, precision and the block
 * shapes of their levels, and every product uses the draws of (seed, mode) as
 * rbc_matmul.  The identity sum_i alpha_i Y(eps_i) = X holds for the unscaled
 * products, so kappa_scale must be 0 unless every level of every plan has
 * kappa = 0 (then it changes nothing); otherwise RBC_EINVAL.  A, B as rbc_matmul.  Products are computed one at a
 * time into the workspace (at least the largest rbc_average_workspace of the
 * plans) and added in the order i = 0..n-1 with the f64 accumulator.  Errors:
 * RBC_EINVAL for null pointers, bad eps, plans that differ, or a short
 * workspace; nothing is launched then. */
#define RBC_EBC_MAX_VALUES 32
rbc_status rbc_apa_ebc_weights(const double* eps, int64_t n, double* alpha);
rbc_status rbc_matmul_apa_ebc(const rbc_plan* plans, const double* eps, int64_t n, const void* A, int64_t lda,
                              const void* B, int64_t ldb, double* C, uint64_t seed, rbc_mode mode,
                              int kappa_scale, void* workspace, size_t ws_bytes, void* stream);

/* x[i] *= s for i < n (device f64). */
rbc_status rbc_scale_f64(double* x, int64_t n, double s, void* stream);

/* ---- stages of rbc_matmul, for composition and testing --------------------
 * gather:  which = 0 forms every leaf S (from A), which = 1 every leaf T
 *          (from B), into the workspace at info.off_S / info.off_T, as
 *          n_leaves row-major blocks in leaf order (r_0 slowest).  For
 *          RBC_PREC_BF16X3 the region holds the hi plane then the lo plane;
 *          for RBC_PREC_F16S it holds f16 values and the gather also writes
 *          the operand's per-leaf exponents in the auxiliary region; for
 *          RBC_PREC_FP8C it holds the e4m3 hi plane then the lo plane (one
 *          byte per element each), with exponents as for f16s.
 * leaf:    P_l = S_l T_l for every leaf l into info.off_P.
 * scatter: C from the P blocks through the folded W of every level.
 * The block combinations sum in a fixed order: S_r over (k, l) row-major and
 * C_ij over ascending r, skipping zero coefficients, one rounding per
 * multiply and per add (no fused multiply-add). */
rbc_status rbc_stage_gather(rbc_plan p, int which, const void* X, int64_t ldx,
                            const int32_t* signs, const int32_t* perms, void* workspace,
                            size_t ws_bytes, void* stream);
rbc_status rbc_stage_leaf(rbc_plan p, void* workspace, size_t ws_bytes, void* stream);
rbc_status rbc_stage_scatter(rbc_plan p, const int32_t* signs, const int32_t* perms, int kappa_scale,
                             void* C, int64_t ldc, void* workspace, size_t ws_bytes, void* stream);

/* ---- timing ---------------------------------------------------------------
 * With timing on, every rbc_matmul / rbc_matmul_draws records HIP events on
 * its stream around each stage.  rbc_plan_timing_collect waits for the
 * recorded events and returns, per stage (0 gather A, 1 gather B, 2 leaf,
 * 3 scatter), the summed milliseconds and the number of calls, then clears
 * them.  At most 4096 calls may be recorded between collects (RBC_ENOMEM). */
rbc_status rbc_plan_set_timing(rbc_plan p, int on);
rbc_status rbc_plan_timing_collect(rbc_plan p, double ms[4], int64_t* calls);


/* ---- measured ceilings (for the rooflines) ----------------------------------
 * rbc_peak_copy: dst = src, bytes a multiple of 16 and both 16-byte aligned
 * (device pointers), on `stream`; the caller times it (HBM bytes moved:
 * 2 x bytes).  rbc_peak_mfma: `blocks` workgroups of 256 threads each run
 * `iters` rounds of independent matrix-core instructions of one type on
 * register operands (f32: 16x16x4, f64: 16x16x4, f16 and bf16: 16x16x32, fp8
 * e4m3: 32x32x64 at unit scale; the _32 kinds: f32 32x32x2, f16 and bf16
 * 32x32x16); `sink` (device, blocks x 256 floats) receives one value per lane;
 * *flops the floating-point operations launched.  Both return RBC_EINVAL for
 * bad arguments and RBC_EHIP when the launch fails. */
enum {
  RBC_PEAK_F32 = 0, RBC_PEAK_F64 = 1, RBC_PEAK_F16 = 2, RBC_PEAK_BF16 = 3, RBC_PEAK_FP8 = 4,
  RBC_PEAK_F32_32 = 5, RBC_PEAK_F16_32 = 6, RBC_PEAK_BF16_32 = 7
};
rbc_status rbc_peak_copy(const void* src, void* dst, size_t bytes, void* stream);
rbc_status rbc_peak_mfma(int kind, int blocks, int iters, float* sink, double* flops, void* stream);

/* ---- batches: many independent products in one persistent launch ---------
 * A batch holds products C_i = F-hat^(Q_i)(A_i, B_i), each with its own plan,
 * operands, seed and mode, all of one precision (RBC_PREC_F32,
 * RBC_PREC_F16S or RBC_PREC_FP8C; every level shape must be Strassen-shaped <2,2,2> with 7
 * products or Laderman-shaped <3,3,3> with 23).  The library turns every
 * product into tasks (pieces of its gather, leaf and scatter stages), orders
 * them so that dependencies come first, and runs them all in one persistent
 * kernel whose workgroups take tasks from a queue and wait on per-subproblem
 * completion counters.  Each product's result is bitwise identical to
 * rbc_matmul with the same plan, operands, seed and mode: the tasks run the
 * same arithmetic in the same order.
 *
 * Ownership: the batch keeps pointers to the plans and operand buffers given
 * to rbc_batch_add; they must stay valid until the batch is destroyed.  The
 * caller owns the workspace (rbc_batch_workspace bytes, 256-byte aligned),
 * which holds the task table, the counters and every product's stage buffers.
 *
 * Waits inside the kernel are bounded by timeout_ms of wall-clock time; a
 * wait that exceeds it stops the whole kernel and rbc_batch_check reports
 * RBC_EHIP (the results are then incomplete). */
typedef struct {
  int32_t window;      /* products whose tasks are interleaved in the queue (0: 32) */
  int32_t grid;        /* workgroups of the persistent kernel (0: resident maximum) */
  int32_t timeout_ms;  /* limit of one dependency wait (0: 5000) */
  int32_t trace;       /* nonzero: record per-task timestamps (rbc_batch_trace) */
  int64_t task_bytes;  /* HBM bytes one task aims to move (0: 4 MiB) */
  int64_t item_budget; /* bytes for the products' stage buffers (0: one region per product).
                        * With a budget the regions form a ring: a product reuses the
                        * bytes of earlier ones and its first tasks wait until those
                        * have finished.  Must hold the largest product's buffers. */
  int32_t mode;        /* RBC_BATCH_PERSISTENT (0) or RBC_BATCH_LEVELS (1), below */
  int32_t order;       /* persistent queue order: RBC_ORDER_PRODUCTS (0) or RBC_ORDER_DEPTH (1) */
} rbc_batch_options;

/* Execution modes of a batch.  PERSISTENT: one persistent kernel takes the tasks
 * from a queue and waits on dependency counters.  LEVELS: the tasks are grouped by
 * their depth in the dependency graph and by type, and every group runs as one
 * grid of one-piece workgroups (a few tens of launches per batch, ordered by the
 * stream); timeout_ms, trace and grid do not apply.  Both give every product the
 * same bits. */
enum { RBC_BATCH_PERSISTENT = 0, RBC_BATCH_LEVELS = 1 };

/* Queue order of the persistent kernel.  PRODUCTS: each product's tasks depth
 * first (a gather of one top block, the subtree below it, its scatter),
 * products interleaved in chunks over `window`.  DEPTH: the same tasks sorted by
 * their depth in the dependency graph (every stage of every product before the
 * next stage).  Both orders are topological; results are the same bits. */
enum { RBC_ORDER_PRODUCTS = 0, RBC_ORDER_DEPTH = 1 };

typedef struct {
  int64_t n_items, n_tasks, n_counters;
  int64_t scale_tasks, gather_tasks, leaf_tasks, scatter_tasks, gate_tasks;
  int64_t levels, launches;  /* RBC_BATCH_LEVELS: dependency depths and grouped launches */
  size_t workspace_bytes; /* total, as rbc_batch_workspace */
  size_t control_bytes;   /* task table, parameters and counters (the rest is stage buffers) */
  int32_t grid, prec;
} rbc_batch_info;

/* One task of the persistent kernel, as rbc_batch_task_table returns them
 * (queue order).  kind: 0 max|X| of an f16s operand, 1 its per-leaf
 * exponents, 2 gather, 3 leaf products, 4 scatter, 5 gate (no work: waits
 * for an earlier product that used the same workspace bytes).  The task covers pieces
 * [first, first + count) of its stage (pieces are workgroup-sized: 256
 * threads' positions of a combination, one output tile of the leaf
 * product), for top block `sub` of a gather or output block `sub` of a
 * scatter.  It waits until counter wait[i] reaches need[i] (wait[i] < 0: no
 * wait) and adds count to counter `signal` when done. */
typedef struct {
  int16_t kind, variant;
  int32_t param;
  int32_t wait[2], need[2];
  int32_t signal, count;
  int64_t first, sub;
} rbc_batch_task;

/* opt may be NULL (defaults). */
rbc_status rbc_batch_create(const rbc_batch_options* opt, rbc_batch* out);
/* Append a product; *index (may be NULL) receives its position. */
rbc_status rbc_batch_add(rbc_batch b, rbc_plan p, const void* A, int64_t lda, const void* B, int64_t ldb,
                         void* C, int64_t ldc, uint64_t seed, rbc_mode mode, int kappa_scale,
                         int64_t* index);
rbc_status rbc_batch_workspace(rbc_batch b, size_t* bytes);
/* Build the task table for this workspace and upload it (asynchronously on
 * stream; the batch keeps its host copy unchanged until the upload is done).
 * Call again after adding products or to use another workspace. */
rbc_status rbc_batch_prepare(rbc_batch b, void* workspace, size_t ws_bytes, void* stream);
/* Enqueue one run on stream: a counter reset and the persistent kernel (or the
 * grouped launches of RBC_BATCH_LEVELS).
 * use_graph != 0 captures both into a HIP graph on first use (stream must
 * not be the default stream) and replays it afterwards. */
rbc_status rbc_batch_launch(rbc_batch b, void* stream, int use_graph);
/* Wait for stream, then report RBC_EHIP if a dependency wait timed out. */
rbc_status rbc_batch_check(rbc_batch b, void* stream);
rbc_status rbc_batch_get_info(rbc_batch b, rbc_batch_info* info);
/* Workgroups of the persistent kernel for later launches (0: the resident
 * maximum; larger values are clamped to it).  A smaller grid leaves room for
 * kernels on other streams, e.g. other batches of a serving loop. */
rbc_status rbc_batch_set_grid(rbc_batch b, int grid);
/* Where a product's stage buffers live in the workspace (byte offset and
 * size), the queue index of its first task, and its two counters: the one
 * its first tasks wait on (previous users of its bytes) and the one its last
 * stage fills. */
typedef struct {
  size_t region_offset, region_bytes;
  int64_t first_task;
  int32_t gate_counter, done_counter;
} rbc_batch_item;
rbc_status rbc_batch_get_item(rbc_batch b, int64_t index, rbc_batch_item* out);
/* With options.trace: after a run has completed, copy up to cap records of
 * 4 words per task (queue order): device wall-clock ticks when the task was
 * taken, when its dependencies were met and when it was signalled, then the
 * workgroup that ran it.  *n receives the task count, *ticks_per_us (may be
 * NULL) the clock rate. */
rbc_status rbc_batch_trace(rbc_batch b, uint64_t* out, int64_t cap, int64_t* n, double* ticks_per_us);
/* Copy up to cap tasks of the last built table into out (host memory; out may
 * be NULL with cap 0) and the table's length into *n. */
rbc_status rbc_batch_task_table(rbc_batch b, rbc_batch_task* out, int64_t cap, int64_t* n);
void rbc_batch_destroy(rbc_batch b);

#ifdef __cplusplus
}
#endif

#endif /* RBC_H */
