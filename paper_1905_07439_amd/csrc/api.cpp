// C ABI of librbc (include/rbc.h): argument checking, device tables, stage
// sequencing and timing.  Every entry point catches C++ exceptions and turns
// them into status codes.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <new>
#include <vector>

#include "core.hpp"
#include "kernels.hpp"
#include "handles.hpp"
#include "launches.hpp"

namespace rbc {
const char* last_error_text();
}

using namespace rbc;


#define RBC_GUARD_BEGIN try {
#define RBC_GUARD_END                                                  \
  }                                                                    \
  catch (const std::bad_alloc&) {                                      \
    return fail(RBC_ENOMEM, "host allocation failed");                 \
  }                                                                    \
  catch (...) {                                                        \
    return fail(RBC_EINVAL, "unexpected C++ exception");               \
  }

#define HIP_CHECK(expr)                                                             \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return fail(RBC_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

extern "C" {

const char* rbc_status_str(rbc_status s) {
  switch (s) {
    case RBC_OK: return "ok";
    case RBC_EINVAL: return "invalid argument";
    case RBC_ESCHEME: return "invalid scheme";
    case RBC_ENOMEM: return "out of memory";
    case RBC_EHIP: return "HIP error";
    case RBC_EUNSUPPORTED: return "unsupported";
    case RBC_EBUSY: return "busy";
  }
  return "unknown status";
}

const char* rbc_last_error(void) { return last_error_text(); }

int rbc_abi_version(void) { return RBC_ABI_VERSION; }

rbc_status rbc_scheme_create(int b1, int b2, int b3, int R, const double* U, const double* V,
                             const double* W, double residual_tol, rbc_scheme* out) {
  RBC_GUARD_BEGIN
  if (!out) return fail(RBC_EINVAL, "null output handle");
  *out = nullptr;
  Scheme s;
  rbc_status st = make_scheme(b1, b2, b3, R, U, V, W, residual_tol, s);
  if (st != RBC_OK) return st;
  *out = new rbc_scheme_s{std::move(s)};
  return RBC_OK;
  RBC_GUARD_END
}

rbc_status rbc_scheme_builtin(const char* name, double lambda, uint64_t aux_seed, rbc_scheme* out) {
  RBC_GUARD_BEGIN
  if (!out) return fail(RBC_EINVAL, "null output handle");
  *out = nullptr;
  Scheme s;
  rbc_status st = builtin_scheme(name, lambda, aux_seed, s);
  if (st != RBC_OK) return st;
  *out = new rbc_scheme_s{std::move(s)};
  return RBC_OK;
  RBC_GUARD_END
}

rbc_status rbc_scheme_info(rbc_scheme h, int dims[4], double* tau, double* kappa, double* ynorm,
                           double* q) {
  if (!h) return fail(RBC_EINVAL, "null scheme");
  const Scheme& s = h->s;
  if (dims) dims[0] = s.b1, dims[1] = s.b2, dims[2] = s.b3, dims[3] = s.R;
  if (tau) *tau = s.tau;
  if (kappa) *kappa = s.kappa;
  if (ynorm) *ynorm = s.ynorm;
  if (q) *q = s.q;
  return RBC_OK;
}

rbc_status rbc_scheme_tensors(rbc_scheme h, double* U, double* V, double* W) {
  if (!h || !U || !V || !W) return fail(RBC_EINVAL, "null argument");
  std::memcpy(U, h->s.U.data(), h->s.U.size() * sizeof(double));
  std::memcpy(V, h->s.V.data(), h->s.V.size() * sizeof(double));
  std::memcpy(W, h->s.W.data(), h->s.W.size() * sizeof(double));
  return RBC_OK;
}

void rbc_scheme_destroy(rbc_scheme h) { delete h; }

rbc_status rbc_draw(uint64_t seed, int depth, int b1, int b2, int b3, rbc_mode mode, int32_t* signs,
                    int32_t* perms) {
  if (!signs || !perms) return fail(RBC_EINVAL, "null output");
  if (b1 < 1 || b2 < 1 || b3 < 1 || b1 > kMaxB || b2 > kMaxB || b3 > kMaxB)
    return fail(RBC_EINVAL, "block partition out of range");
  if (depth < 0) return fail(RBC_EINVAL, "negative depth");
  if (mode < RBC_MODE_FULL || mode > RBC_MODE_NONE) return fail(RBC_EINVAL, "bad mode %d", (int)mode);
  draw_level(seed, depth, b1, b2, b3, mode, signs, perms);
  return RBC_OK;
}

rbc_status rbc_fold(rbc_scheme h, const int32_t* signs, const int32_t* perms, int kappa_scale,
                    double* Uh, double* Vh, double* Wh) {
  if (!h || !signs || !perms || !Uh || !Vh || !Wh) return fail(RBC_EINVAL, "null argument");
  const Scheme& s = h->s;
  if (!valid_draw(s.b1, s.b2, s.b3, signs, perms)) return fail(RBC_EINVAL, "invalid draw");
  fold(s, signs, perms, kappa_scale != 0, Uh, Vh, Wh);
  return RBC_OK;
}

rbc_status rbc_plan_create(int64_t M, int64_t K, int64_t N, int levels, const rbc_scheme* schemes,
                           rbc_prec prec, int leaf_tile, rbc_plan* out) {
  RBC_GUARD_BEGIN
  if (!out) return fail(RBC_EINVAL, "null output handle");
  *out = nullptr;
  if (levels < 0 || levels > RBC_MAX_LEVELS) return fail(RBC_EINVAL, "levels = %d", levels);
  if (levels > 0 && !schemes) return fail(RBC_EINVAL, "null scheme array");
  std::vector<Scheme> lv;
  for (int d = 0; d < levels; ++d) {
    if (!schemes[d]) return fail(RBC_EINVAL, "null scheme at level %d", d);
    lv.push_back(schemes[d]->s);
  }
  Plan p;
  rbc_status st = make_plan(M, K, N, lv, prec, leaf_tile, p);
  if (st != RBC_OK) return st;
  *out = new rbc_plan_s{std::move(p)};
  return RBC_OK;
  RBC_GUARD_END
}

rbc_status rbc_plan_get_info(rbc_plan h, rbc_plan_info* info) {
  if (!h || !info) return fail(RBC_EINVAL, "null argument");
  const Plan& p = h->p;
  info->M = p.M, info->K = p.K, info->N = p.N;
  info->Mp = p.Mp, info->Kp = p.Kp, info->Np = p.Np;
  info->mM = p.mM, info->mK = p.mK, info->mN = p.mN;
  info->n_leaves = p.n_leaves;
  info->levels = p.Q;
  info->n_groups = (int32_t)p.groups.size();
  info->prec = (int32_t)p.prec;
  info->tile_m = p.tile_m, info->tile_n = p.tile_n, info->tile_k = p.tile_k;
  info->workspace_bytes = p.ws_bytes;
  info->off_S = p.off_S, info->off_T = p.off_T, info->off_P = p.off_P;
  info->bytes_S = p.bytes_S, info->bytes_T = p.bytes_T, info->bytes_P = p.bytes_P;
  info->off_aux = p.off_aux, info->bytes_aux = p.bytes_aux;
  info->n_scatter_groups = (int32_t)p.sgroups.size();
  return RBC_OK;
}

rbc_status rbc_plan_traffic(rbc_plan h, double bytes[4]) {
  if (!h || !bytes) return fail(RBC_EINVAL, "null argument");
  const Plan& p = h->p;
  const double e = p.prec == RBC_PREC_F64 ? 8 : 4;              // combination element
  const double e_leaf =
      p.prec == RBC_PREC_F64 ? 8 : ((p.prec == RBC_PREC_F16S || p.prec == RBC_PREC_FP8C) ? 2 : 4);  // leaf operand
  const double e_prod = p.prec == RBC_PREC_F64 ? 8 : 4;         // leaf product
  const double e_mid = (p.prec == RBC_PREC_F64 || p.prec == RBC_PREC_BF16X3) ? 8 : 4;  // recombination
  const double e_out = p.prec == RBC_PREC_F64 ? 8 : 4;          // C
  for (int i = 0; i < 4; ++i) bytes[i] = 0;
  // gathers: the readable part of every top block once, every bottom block once
  const std::vector<Group>& gg = p.leaf_gather ? p.fgroups : p.groups;
  for (size_t gi = 0; gi < gg.size(); ++gi) {
    const Group& g = gg[gi];
    const bool last = gi + 1 == gg.size() && !p.leaf_gather;
    const double n_out = (double)g.n_in * g.Rg;
    const double rdA = gi == 0 ? (double)p.M * p.K : (double)g.n_in * g.a_rows_top * g.a_cols_top;
    const double rdB = gi == 0 ? (double)p.K * p.N : (double)g.n_in * g.b_rows_top * g.b_cols_top;
    const double wo = last ? e_leaf : e;
    bytes[0] += rdA * e + n_out * g.a_rows_bot * g.a_cols_bot * wo;
    bytes[1] += rdB * e + n_out * g.b_rows_bot * g.b_cols_bot * wo;
  }
  const bool ls = p.leaf_gather && p.leaf_scatter;
  const std::vector<Group>& sg = ls ? p.fgroups : p.sgroups;
  const size_t ng = sg.size();
  for (size_t gi = 0; gi < ng; ++gi) {
    const Group& g = sg[gi];
    const bool last = gi + 1 == ng && !ls;
    const double n_out = (double)g.n_in * g.Rg;
    // scatter: every bottom block once, the writable part of every top block once
    const double rp = last ? e_prod : e_mid;
    const double wc = gi == 0 ? (double)p.M * p.N * e_out : (double)g.n_in * g.c_rows_top * g.c_cols_top * e_mid;
    bytes[3] += n_out * g.c_rows_bot * g.c_cols_bot * rp + wc;
  }
  if (p.prec == RBC_PREC_F16S || p.prec == RBC_PREC_FP8C)
    bytes[0] += (double)p.M * p.K * 4, bytes[1] += (double)p.K * p.N * 4;  // max|X|
  bytes[2] = (double)p.n_leaves * ((double)p.mM * p.mK * e_leaf + (double)p.mK * p.mN * e_leaf +
                                   (double)p.mM * p.mN * e_prod);
  if (p.leaf_gather) {  // every parent block once instead of the leaf operands
    const Group& g = p.fgroups.back();
    const double n_par = (double)g.n_in * g.Rg;
    bytes[2] = n_par * ((double)g.a_rows_bot * g.a_cols_bot + (double)g.b_rows_bot * g.b_cols_bot) * e +
               (double)p.n_leaves * p.mM * p.mN * e_prod;
    // leaf scatter: the products read back once, the parents' product blocks written once
    if (ls) bytes[2] += (double)p.n_leaves * p.mM * p.mN * e_prod + n_par * (double)g.c_rows_bot * g.c_cols_bot * e_mid;
  }
  return RBC_OK;
}

void rbc_plan_destroy(rbc_plan h) {
  if (!h) return;
  Plan& p = h->p;
  if (p.dev_tables) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p.device);
    (void)hipFree(p.dev_tables);
    for (void* e : p.events) (void)hipEventDestroy((hipEvent_t)e);
    if (cur >= 0) (void)hipSetDevice(cur);
  } else {
    for (void* e : p.events) (void)hipEventDestroy((hipEvent_t)e);
  }
  delete h;
}

}  // extern "C"

namespace {

struct Ctx {
  Plan& p;
  char* ws;
  hipStream_t stream;
  Draws dr;
};

rbc_status run_gather(Ctx& c, int which, const void* X, int64_t ldx, bool leaf_gather = false) {
  std::vector<ScaleLaunch> scale;
  std::vector<GatherLaunch> gl;
  build_gather(c.p, c.dr, which, X, ldx, c.ws, scale, gl, leaf_gather);
  for (const ScaleLaunch& l : scale) {
    hipError_t e = launch(l, c.stream);
    if (e != hipSuccess) return fail(RBC_EHIP, "scale launch: %s", hipGetErrorString(e));
  }
  for (const GatherLaunch& l : gl) {
    hipError_t e = launch(l, c.stream);
    if (e != hipSuccess) return fail(RBC_EHIP, "gather launch: %s", hipGetErrorString(e));
  }
  return RBC_OK;
}

// The gathers of A and B, each level group's two sides in one launch (the
// per-side order of the groups is kept; the sides are independent).
rbc_status run_gathers(Ctx& c, const void* A, int64_t lda, const void* B, int64_t ldb, bool leaf_gather) {
  std::vector<ScaleLaunch> sa, sb;
  std::vector<GatherLaunch> ga, gb;
  build_gather(c.p, c.dr, 0, A, lda, c.ws, sa, ga, leaf_gather);
  build_gather(c.p, c.dr, 1, B, ldb, c.ws, sb, gb, leaf_gather);
  if (sa.size() == 1 && sb.size() == 1) {
    hipError_t e = launch(sa[0], sb[0], c.stream);
    if (e != hipSuccess) return fail(RBC_EHIP, "scale launch: %s", hipGetErrorString(e));
  } else {
    for (const std::vector<ScaleLaunch>* v : {&sa, &sb})
      for (const ScaleLaunch& l : *v) {
        hipError_t e = launch(l, c.stream);
        if (e != hipSuccess) return fail(RBC_EHIP, "scale launch: %s", hipGetErrorString(e));
      }
  }
  for (size_t i = 0; i < ga.size() || i < gb.size(); ++i) {
    hipError_t e = hipSuccess;
    if (i < ga.size() && i < gb.size()) e = launch(ga[i], gb[i], c.stream);
    else e = launch(i < ga.size() ? ga[i] : gb[i], c.stream);
    if (e != hipSuccess) return fail(RBC_EHIP, "gather launch: %s", hipGetErrorString(e));
  }
  return RBC_OK;
}

rbc_status run_leaf(Ctx& c, bool leaf_gather = false, bool leaf_scatter = false, bool kappa_scale = false) {
  hipError_t e = leaf_gather ? launch(build_leaf_gather(c.p, c.dr, c.ws, leaf_scatter, kappa_scale), c.stream)
                             : launch(build_leaf(c.p, c.ws), c.stream);
  if (e != hipSuccess) return fail(RBC_EHIP, "leaf launch: %s", hipGetErrorString(e));
  return RBC_OK;
}

rbc_status run_scatter(Ctx& c, bool kappa_scale, void* C, int64_t ldc, bool leaf_scatter = false) {
  std::vector<ScatterLaunch> sl;
  build_scatter(c.p, c.dr, kappa_scale, C, ldc, c.ws, sl, leaf_scatter ? c.p.fgroups : c.p.sgroups, leaf_scatter);
  for (const ScatterLaunch& l : sl) {
    hipError_t e = launch(l, c.stream);
    if (e != hipSuccess) return fail(RBC_EHIP, "scatter launch: %s", hipGetErrorString(e));
  }
  return RBC_OK;
}

rbc_status record(Plan& p, hipStream_t s, int slot) {
  if (!p.timing) return RBC_OK;
  const size_t idx = (size_t)p.recorded * 5 + slot;
  while (p.events.size() <= idx) {
    hipEvent_t e;
    HIP_CHECK(hipEventCreate(&e));
    p.events.push_back(e);
  }
  HIP_CHECK(hipEventRecord((hipEvent_t)p.events[idx], s));
  return RBC_OK;
}

}  // namespace

rbc_status rbc::matmul_impl(Plan& p, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                            int64_t ldc, const int32_t* signs, const int32_t* perms, int kappa_scale,
                            void* ws, size_t ws_bytes, void* stream) {
  if (!A || !B || !C) return fail(RBC_EINVAL, "null matrix pointer");
  if (lda < p.K || ldb < p.N || ldc < p.N) return fail(RBC_EINVAL, "leading dimension too small");
  rbc_status st = check_ws(p, ws, ws_bytes);
  if (st != RBC_OK) return st;
  Ctx c{p, static_cast<char*>(ws), (hipStream_t)stream, {}};
  if ((st = check_draws(p, signs, perms, c.dr)) != RBC_OK) return st;
  if ((st = ensure_device(p)) != RBC_OK) return st;
  if (p.timing && p.recorded >= 4096) return fail(RBC_ENOMEM, "timing buffer full; collect first");
  const bool lg = p.leaf_gather;
  if ((st = record(p, c.stream, 0)) != RBC_OK) return st;
  if (p.timing) {  // separate launches, so that the events time A and B apart
    if ((st = run_gather(c, 0, A, lda, lg)) != RBC_OK) return st;
    if ((st = record(p, c.stream, 1)) != RBC_OK) return st;
    if ((st = run_gather(c, 1, B, ldb, lg)) != RBC_OK) return st;
  } else if ((st = run_gathers(c, A, lda, B, ldb, lg)) != RBC_OK) {
    return st;
  }
  if ((st = record(p, c.stream, 2)) != RBC_OK) return st;
  const bool ls = lg && p.leaf_scatter;
  if ((st = run_leaf(c, lg, ls, kappa_scale != 0)) != RBC_OK) return st;
  if ((st = record(p, c.stream, 3)) != RBC_OK) return st;
  if ((st = run_scatter(c, kappa_scale != 0, C, ldc, ls)) != RBC_OK) return st;
  if ((st = record(p, c.stream, 4)) != RBC_OK) return st;
  if (p.timing) ++p.recorded;
  return RBC_OK;
}

extern "C" {

rbc_status rbc_matmul(rbc_plan h, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                      int64_t ldc, uint64_t seed, rbc_mode mode, int kappa_scale, void* workspace,
                      size_t ws_bytes, void* stream) {
  RBC_GUARD_BEGIN
  if (!h) return fail(RBC_EINVAL, "null plan");
  if (mode < RBC_MODE_FULL || mode > RBC_MODE_NONE) return fail(RBC_EINVAL, "bad mode %d", (int)mode);
  std::vector<int32_t> s, pm;
  seeded_draws(h->p, seed, mode, s, pm);
  return matmul_impl(h->p, A, lda, B, ldb, C, ldc, s.data(), pm.data(), kappa_scale, workspace,
                     ws_bytes, stream);
  RBC_GUARD_END
}

rbc_status rbc_matmul_draws(rbc_plan h, const void* A, int64_t lda, const void* B, int64_t ldb,
                            void* C, int64_t ldc, const int32_t* signs, const int32_t* perms,
                            int kappa_scale, void* workspace, size_t ws_bytes, void* stream) {
  RBC_GUARD_BEGIN
  if (!h) return fail(RBC_EINVAL, "null plan");
  return matmul_impl(h->p, A, lda, B, ldb, C, ldc, signs, perms, kappa_scale, workspace, ws_bytes,
                     stream);
  RBC_GUARD_END
}

rbc_status rbc_accumulate(double* acc, const void* X, int x_is_f64, int64_t rows, int64_t cols, int64_t ldx,
                          int first, void* stream) {
  if (!acc || !X) return fail(RBC_EINVAL, "null pointer");
  if (rows < 0 || cols < 0 || ldx < cols) return fail(RBC_EINVAL, "bad shape");
  HIP_CHECK(launch_accumulate(acc, X, x_is_f64 ? ELT_F64 : ELT_F32, rows, cols, ldx, first != 0,
                              (hipStream_t)stream));
  return RBC_OK;
}

rbc_status rbc_scale_f64(double* x, int64_t n, double s, void* stream) {
  if (!x || n < 0) return fail(RBC_EINVAL, "bad argument");
  HIP_CHECK(launch_scale_f64(x, n, s, (hipStream_t)stream));
  return RBC_OK;
}

rbc_status rbc_average_workspace(rbc_plan h, size_t* bytes) {
  if (!h || !bytes) return fail(RBC_EINVAL, "null argument");
  const Plan& p = h->p;
  const size_t elt = p.prec == RBC_PREC_F64 ? 8 : 4;
  *bytes = (p.ws_bytes + 255) / 256 * 256 + (size_t)p.M * p.N * elt;
  return RBC_OK;
}

rbc_status rbc_matmul_average(rbc_plan h, const void* A, int64_t lda, const void* B, int64_t ldb, double* Cavg,
                              const uint64_t* seeds, int64_t K, rbc_mode mode, int kappa_scale, void* workspace,
                              size_t ws_bytes, void* stream) {
  RBC_GUARD_BEGIN
  if (!h || !Cavg || !seeds) return fail(RBC_EINVAL, "null argument");
  if (K < 1) return fail(RBC_EINVAL, "K must be at least 1");
  if (mode < RBC_MODE_FULL || mode > RBC_MODE_NONE) return fail(RBC_EINVAL, "bad mode %d", (int)mode);
  Plan& p = h->p;
  size_t need = 0;
  rbc_status st = rbc_average_workspace(h, &need);
  if (st != RBC_OK) return st;
  if (!workspace || ws_bytes < need) return fail(RBC_EINVAL, "workspace of %zu bytes < %zu needed", ws_bytes, need);
  const size_t plan_ws = (p.ws_bytes + 255) / 256 * 256;
  void* prod = static_cast<char*>(workspace) + plan_ws;
  const Elt elt = p.prec == RBC_PREC_F64 ? ELT_F64 : ELT_F32;
  std::vector<int32_t> s, pm;
  for (int64_t k = 0; k < K; ++k) {
    seeded_draws(p, seeds[k], mode, s, pm);
    st = matmul_impl(p, A, lda, B, ldb, prod, p.N, s.data(), pm.data(), kappa_scale, workspace, plan_ws, stream);
    if (st != RBC_OK) return st;
    HIP_CHECK(launch_accumulate(Cavg, prod, elt, p.M, p.N, p.N, k == 0, (hipStream_t)stream));
  }
  HIP_CHECK(launch_scale_f64(Cavg, p.M * p.N, 1.0 / (double)K, (hipStream_t)stream));
  return RBC_OK;
  RBC_GUARD_END
}

rbc_status rbc_accumulate_weighted(double* acc, const void* X, int x_is_f64, int64_t rows, int64_t cols,
                                   int64_t ldx, double weight, int first, void* stream) {
  if (!acc || !X) return fail(RBC_EINVAL, "null pointer");
  if (rows < 0 || cols < 0 || ldx < cols) return fail(RBC_EINVAL, "bad shape");
  if (!std::isfinite(weight)) return fail(RBC_EINVAL, "weight is not finite");
  HIP_CHECK(launch_accumulate(acc, X, x_is_f64 ? ELT_F64 : ELT_F32, rows, cols, ldx, first != 0,
                              (hipStream_t)stream, weight));
  return RBC_OK;
}

rbc_status rbc_apa_ebc_weights(const double* eps, int64_t n, double* alpha) {
  if (!eps || !alpha) return fail(RBC_EINVAL, "null argument");
  if (n < 1 || n > RBC_EBC_MAX_VALUES) return fail(RBC_EINVAL, "n = %lld outside [1, %d]", (long long)n,
                                                   RBC_EBC_MAX_VALUES);
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(eps[i]) || eps[i] == 0.0) return fail(RBC_EINVAL, "eps[%lld] is zero or not finite",
                                                             (long long)i);
    for (int64_t j = 0; j < i; ++j)
      if (eps[j] == eps[i]) return fail(RBC_EINVAL, "eps[%lld] repeats eps[%lld]", (long long)i, (long long)j);
  }
  // The combination must reproduce the value at eps = 0 of every polynomial of
  // degree < n through the n points: the Lagrange basis evaluated at zero.
  for (int64_t i = 0; i < n; ++i) {
    double a = 1.0;
    for (int64_t j = 0; j < n; ++j)
      if (j != i) a *= eps[j] / (eps[j] - eps[i]);
    alpha[i] = a;
  }
  return RBC_OK;
}

rbc_status rbc_matmul_apa_ebc(const rbc_plan* plans, const double* eps, int64_t n, const void* A, int64_t lda,
                              const void* B, int64_t ldb, double* C, uint64_t seed, rbc_mode mode,
                              int kappa_scale, void* workspace, size_t ws_bytes, void* stream) {
  RBC_GUARD_BEGIN
  if (!plans || !eps || !C) return fail(RBC_EINVAL, "null argument");
  if (mode < RBC_MODE_FULL || mode > RBC_MODE_NONE) return fail(RBC_EINVAL, "bad mode %d", (int)mode);
  double alpha[RBC_EBC_MAX_VALUES];
  rbc_status st = rbc_apa_ebc_weights(eps, n, alpha);
  if (st != RBC_OK) return st;
  for (int64_t i = 0; i < n; ++i)
    if (!plans[i]) return fail(RBC_EINVAL, "plans[%lld] is null", (long long)i);
  const Plan& p0 = plans[0]->p;
  std::vector<int32_t> s0, pm0, s, pm;
  seeded_draws(p0, seed, mode, s0, pm0);
  size_t need = 0;
  for (int64_t i = 0; i < n; ++i) {
    const Plan& p = plans[i]->p;
    if (p.M != p0.M || p.K != p0.K || p.N != p0.N || p.prec != p0.prec)
      return fail(RBC_EINVAL, "plans[%lld] differs from plans[0] in shape or precision", (long long)i);
    seeded_draws(p, seed, mode, s, pm);
    if (s != s0 || pm != pm0) return fail(RBC_EINVAL, "plans[%lld] differs from plans[0] in its levels' block shapes",
                                          (long long)i);
    // The weights make sum_i alpha_i Y(eps_i) = X for the unscaled Y; a level with
    // kappa != 0 scaled by (1 - kappa)^-1 would break that identity.
    if (kappa_scale)
      for (int d = 0; d < p.Q; ++d)
        if (p.levels[d].kappa != 0.0)
          return fail(RBC_EINVAL, "kappa_scale with plans[%lld] level %d: kappa = %.17g != 0 (the combination "
                      "is exact only for the unscaled products)", (long long)i, d, p.levels[d].kappa);
    size_t b = 0;
    if ((st = rbc_average_workspace(plans[i], &b)) != RBC_OK) return st;
    need = b > need ? b : need;
  }
  if (!workspace || ws_bytes < need) return fail(RBC_EINVAL, "workspace of %zu bytes < %zu needed", ws_bytes, need);
  const Elt elt = p0.prec == RBC_PREC_F64 ? ELT_F64 : ELT_F32;
  for (int64_t i = 0; i < n; ++i) {
    Plan& p = plans[i]->p;
    const size_t plan_ws = (p.ws_bytes + 255) / 256 * 256;
    void* prod = static_cast<char*>(workspace) + plan_ws;
    st = matmul_impl(p, A, lda, B, ldb, prod, p.N, s0.data(), pm0.data(), kappa_scale, workspace, plan_ws, stream);
    if (st != RBC_OK) return st;
    HIP_CHECK(launch_accumulate(C, prod, elt, p.M, p.N, p.N, i == 0, (hipStream_t)stream, alpha[i]));
  }
  return RBC_OK;
  RBC_GUARD_END
}

rbc_status rbc_stage_gather(rbc_plan h, int which, const void* X, int64_t ldx, const int32_t* signs,
                            const int32_t* perms, void* workspace, size_t ws_bytes, void* stream) {
  RBC_GUARD_BEGIN
  if (!h) return fail(RBC_EINVAL, "null plan");
  Plan& p = h->p;
  if (which != 0 && which != 1) return fail(RBC_EINVAL, "which must be 0 (A) or 1 (B)");
  if (!X) return fail(RBC_EINVAL, "null matrix pointer");
  if (ldx < (which == 0 ? p.K : p.N)) return fail(RBC_EINVAL, "leading dimension too small");
  rbc_status st = check_ws(p, workspace, ws_bytes);
  if (st != RBC_OK) return st;
  Ctx c{p, static_cast<char*>(workspace), (hipStream_t)stream, {}};
  if ((st = check_draws(p, signs, perms, c.dr)) != RBC_OK) return st;
  if ((st = ensure_device(p)) != RBC_OK) return st;
  return run_gather(c, which, X, ldx);
  RBC_GUARD_END
}

rbc_status rbc_stage_leaf(rbc_plan h, void* workspace, size_t ws_bytes, void* stream) {
  RBC_GUARD_BEGIN
  if (!h) return fail(RBC_EINVAL, "null plan");
  Plan& p = h->p;
  rbc_status st = check_ws(p, workspace, ws_bytes);
  if (st != RBC_OK) return st;
  Ctx c{p, static_cast<char*>(workspace), (hipStream_t)stream, {}};
  return run_leaf(c);
  RBC_GUARD_END
}

rbc_status rbc_stage_scatter(rbc_plan h, const int32_t* signs, const int32_t* perms, int kappa_scale,
                             void* C, int64_t ldc, void* workspace, size_t ws_bytes, void* stream) {
  RBC_GUARD_BEGIN
  if (!h) return fail(RBC_EINVAL, "null plan");
  Plan& p = h->p;
  if (!C) return fail(RBC_EINVAL, "null matrix pointer");
  if (ldc < p.N) return fail(RBC_EINVAL, "leading dimension too small");
  rbc_status st = check_ws(p, workspace, ws_bytes);
  if (st != RBC_OK) return st;
  Ctx c{p, static_cast<char*>(workspace), (hipStream_t)stream, {}};
  if ((st = check_draws(p, signs, perms, c.dr)) != RBC_OK) return st;
  if ((st = ensure_device(p)) != RBC_OK) return st;
  return run_scatter(c, kappa_scale != 0, C, ldc);
  RBC_GUARD_END
}

rbc_status rbc_plan_set_timing(rbc_plan h, int on) {
  if (!h) return fail(RBC_EINVAL, "null plan");
  h->p.timing = on != 0;
  return RBC_OK;
}

rbc_status rbc_plan_set_fusion(rbc_plan h, int fuse_max) {
  RBC_GUARD_BEGIN
  if (!h) return fail(RBC_EINVAL, "null plan");
  Plan& p = h->p;
  if (p.fuse_max == (fuse_max != 0)) return RBC_OK;
  Plan q;
  rbc_status st = make_plan(p.M, p.K, p.N, p.levels, p.prec, p.tile_m, q, fuse_max != 0);
  if (st != RBC_OK) return st;
  // the device tables and events do not depend on the grouping
  q.device = p.device, q.dev_tables = p.dev_tables, q.tab_off = p.tab_off;
  q.timing = p.timing, q.events = std::move(p.events), q.recorded = p.recorded;
  p.dev_tables = nullptr;
  p = std::move(q);
  return RBC_OK;
  RBC_GUARD_END
}

rbc_status rbc_plan_set_leaf_gather(rbc_plan h, int on) {
  if (!h) return fail(RBC_EINVAL, "null plan");
  if (on && !h->p.leaf_gather_ok)
    return fail(RBC_EUNSUPPORTED, "leaf gather needs f32, two or more levels and at most two terms per product");
  h->p.leaf_gather = on != 0;
  if (!on) h->p.leaf_scatter = false;
  return RBC_OK;
}

rbc_status rbc_plan_set_leaf_scatter(rbc_plan h, int on) {
  if (!h) return fail(RBC_EINVAL, "null plan");
  if (on && !(h->p.leaf_scatter_ok && h->p.leaf_gather))
    return fail(RBC_EUNSUPPORTED, "leaf scatter needs the leaf gather on");
  if (on) layout_leaf_scatter(h->p);
  h->p.leaf_scatter = on != 0;
  return RBC_OK;
}

rbc_status rbc_plan_get_leaf_scatter(rbc_plan h, int* on, int* available) {
  if (!h) return fail(RBC_EINVAL, "null plan");
  if (on) *on = h->p.leaf_scatter ? 1 : 0;
  if (available) *available = h->p.leaf_scatter_ok ? 1 : 0;
  return RBC_OK;
}

rbc_status rbc_plan_get_leaf_gather(rbc_plan h, int* on, int* available) {
  if (!h) return fail(RBC_EINVAL, "null plan");
  if (on) *on = h->p.leaf_gather ? 1 : 0;
  if (available) *available = h->p.leaf_gather_ok ? 1 : 0;
  return RBC_OK;
}

rbc_status rbc_plan_timing_collect(rbc_plan h, double ms[4], int64_t* calls) {
  RBC_GUARD_BEGIN
  if (!h || !ms) return fail(RBC_EINVAL, "null argument");
  Plan& p = h->p;
  for (int i = 0; i < 4; ++i) ms[i] = 0;
  for (int64_t c = 0; c < p.recorded; ++c) {
    HIP_CHECK(hipEventSynchronize((hipEvent_t)p.events[c * 5 + 4]));
    for (int i = 0; i < 4; ++i) {
      float t = 0;
      HIP_CHECK(hipEventElapsedTime(&t, (hipEvent_t)p.events[c * 5 + i], (hipEvent_t)p.events[c * 5 + i + 1]));
      ms[i] += t;
    }
  }
  if (calls) *calls = p.recorded;
  p.recorded = 0;
  return RBC_OK;
  RBC_GUARD_END
}

}  // extern "C"
