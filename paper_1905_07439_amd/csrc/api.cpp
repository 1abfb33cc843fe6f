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

namespace rbc {
const char* last_error_text();
}

using namespace rbc;

struct rbc_scheme_s {
  Scheme s;
};
struct rbc_plan_s {
  Plan p;
};

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

rbc_status rbc_scheme_builtin(const char* name, rbc_scheme* out) {
  RBC_GUARD_BEGIN
  if (!out) return fail(RBC_EINVAL, "null output handle");
  *out = nullptr;
  Scheme s;
  rbc_status st = builtin_scheme(name, s);
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

// Upload the coefficient tables of every level on first use on a device.
rbc_status ensure_device(Plan& p) {
  int dev = -1;
  HIP_CHECK(hipGetDevice(&dev));
  if (p.dev_tables) {
    if (dev != p.device) return fail(RBC_EINVAL, "plan was first used on device %d, now %d", p.device, dev);
    return RBC_OK;
  }
  std::vector<char> blob;
  p.tab_off.clear();
  auto put = [&](const void* src, size_t bytes) {
    const size_t off = (blob.size() + 255) & ~size_t(255);
    blob.resize(off + bytes);
    std::memcpy(blob.data() + off, src, bytes);
    p.tab_off.push_back(off);
  };
  for (const LevelTables& t : p.tables) {
    put(t.U.data(), t.U.size() * 8);
    put(t.V.data(), t.V.size() * 8);
    put(t.W.data(), t.W.size() * 8);
    put(t.Wk.data(), t.Wk.size() * 8);
    put(t.Uf.data(), t.Uf.size() * 4);
    put(t.Vf.data(), t.Vf.size() * 4);
    put(t.Wf.data(), t.Wf.size() * 4);
    put(t.Wkf.data(), t.Wkf.size() * 4);
  }
  if (!p.gA.empty()) {
    put(p.gA.data(), p.gA.size() * 4);
    p.g_off[0] = p.tab_off.back();
    put(p.gB.data(), p.gB.size() * 4);
    p.g_off[1] = p.tab_off.back();
  }
  if (blob.empty()) blob.resize(256);
  void* d = nullptr;
  HIP_CHECK(hipMalloc(&d, blob.size()));
  hipError_t e = hipMemcpy(d, blob.data(), blob.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return fail(RBC_EHIP, "table upload: %s", hipGetErrorString(e));
  }
  p.dev_tables = d;
  p.device = dev;
  return RBC_OK;
}

const void* table(const Plan& p, int level, TabKind kind, bool f64) {
  const size_t idx = (size_t)level * 8 + (f64 ? 0 : 4) + (size_t)kind;
  return static_cast<const char*>(p.dev_tables) + p.tab_off[idx];
}

// Per-level draw pointers into the concatenated arrays.
struct Draws {
  std::vector<int32_t> s, pm;
  std::vector<size_t> off;
};

rbc_status check_draws(const Plan& p, const int32_t* signs, const int32_t* perms, Draws& d) {
  if (p.Q > 0 && (!signs || !perms)) return fail(RBC_EINVAL, "null draw arrays");
  size_t o = 0;
  d.off.clear();
  for (int l = 0; l < p.Q; ++l) {
    const Scheme& s = p.levels[l];
    if (!valid_draw(s.b1, s.b2, s.b3, signs + o, perms + o))
      return fail(RBC_EINVAL, "invalid draw at level %d", l);
    d.off.push_back(o);
    o += s.b1 + s.b2 + s.b3;
  }
  d.s.assign(signs, signs + o);
  d.pm.assign(perms, perms + o);
  return RBC_OK;
}

enum Side { SIDE_A, SIDE_B, SIDE_C };

// Positions per thread for a combination launch: the widest of 4, 2, 1 that
// divides the block width, every leading dimension and block stride, and the
// element alignment of every pointer.  8-byte accumulators use at most 2, and
// 1 in two-level groups (register budget).
// RBC_COMBINE_VEC (1, 2 or 4) lowers the cap for tuning.
int max_vec_override() {
  static const int v = [] {
    const char* e = std::getenv("RBC_COMBINE_VEC");
    const int x = e ? std::atoi(e) : 4;
    return (x == 1 || x == 2 || x == 4) ? x : 4;
  }();
  return v;
}

int pick_vec(int elt_bytes, int64_t cols, std::initializer_list<int64_t> strides,
             std::initializer_list<const void*> ptrs, bool wide_acc, int nl) {
  const int cap = std::min(wide_acc ? (nl >= 2 ? 1 : 2) : 4, max_vec_override());
  for (int v = cap; v > 1; v /= 2) {
    bool ok = cols % v == 0;
    for (int64_t s : strides) ok = ok && s % v == 0;
    for (const void* q : ptrs) ok = ok && reinterpret_cast<uintptr_t>(q) % (size_t)(v * elt_bytes) == 0;
    if (ok) return v;
  }
  return 1;
}

void fill_side(const Plan& p, const Draws& dr, int level, Side side, bool f64, bool kappa_scale,
               SideLevel& L) {
  const Scheme& s = p.levels[level];
  const int32_t* sg = dr.s.data() + dr.off[level];
  const int32_t* pm = dr.pm.data() + dr.off[level];
  const int32_t *s1 = sg, *s2 = sg + s.b1, *s3 = sg + s.b1 + s.b2;
  const int32_t *p1 = pm, *p2 = pm + s.b1, *p3 = pm + s.b1 + s.b2;
  const int32_t *sr, *sc, *pr, *pc;
  int nr, nc;
  TabKind kind;
  if (side == SIDE_A) sr = s1, sc = s2, pr = p1, pc = p2, nr = s.b1, nc = s.b2, kind = TAB_U;
  else if (side == SIDE_B) sr = s2, sc = s3, pr = p2, pc = p3, nr = s.b2, nc = s.b3, kind = TAB_V;
  else sr = s1, sc = s3, pr = p1, pc = p3, nr = s.b1, nc = s.b3, kind = kappa_scale ? TAB_WK : TAB_W;
  std::memset(&L, 0, sizeof L);
  for (int i = 0; i < nr; ++i) L.pr[i] = (int8_t)pr[i], L.sr[i] = (int8_t)sr[i];
  for (int j = 0; j < nc; ++j) L.pc[j] = (int8_t)pc[j], L.sc[j] = (int8_t)sc[j];
  L.R = s.R;
  L.tab = table(p, level, kind, f64);
}

struct Ctx {
  Plan& p;
  char* ws;
  hipStream_t stream;
  Draws dr;
};

rbc_status check_ws(const Plan& p, void* ws, size_t bytes) {
  if (!ws) return fail(RBC_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(RBC_EINVAL, "workspace not 256-byte aligned");
  if (bytes < p.ws_bytes)
    return fail(RBC_ENOMEM, "workspace of %zu bytes, plan needs %zu", bytes, p.ws_bytes);
  return RBC_OK;
}

rbc_status run_gather(Ctx& c, int which, const void* X, int64_t ldx) {
  Plan& p = c.p;
  const bool f64 = p.prec == RBC_PREC_F64;
  const bool f16s = p.prec == RBC_PREC_F16S;
  int32_t* exps = nullptr;
  if (f16s) {
    uint32_t* maxbits = reinterpret_cast<uint32_t*>(c.ws + p.off_aux) + which;
    exps = reinterpret_cast<int32_t*>(c.ws + p.off_aux + 256) + (size_t)which * p.n_leaves;
    const float* G = reinterpret_cast<const float*>(static_cast<const char*>(p.dev_tables) + p.g_off[which]);
    hipError_t e = launch_leaf_scales(static_cast<const float*>(X), ldx, which == 0 ? p.M : p.K,
                                      which == 0 ? p.K : p.N, maxbits, G, exps, p.n_leaves, c.stream);
    if (e != hipSuccess) return fail(RBC_EHIP, "scale launch: %s", hipGetErrorString(e));
  }
  for (size_t gi = 0; gi < p.groups.size(); ++gi) {
    const Group& g = p.groups[gi];
    const bool last = gi + 1 == p.groups.size();
    GatherParams gp;
    std::memset(&gp, 0, sizeof gp);
    const int64_t rows_top = which == 0 ? g.a_rows_top : g.b_rows_top;
    const int64_t cols_top = which == 0 ? g.a_cols_top : g.b_cols_top;
    if (gi == 0) {
      gp.src = X, gp.ld_src = ldx, gp.src_batch = 0;
      gp.src_rows = which == 0 ? p.M : p.K;
      gp.src_cols = which == 0 ? p.K : p.N;
    } else {
      const Group& up = p.groups[gi - 1];
      gp.src = c.ws + (which == 0 ? up.off_a_bot : up.off_b_bot);
      gp.ld_src = cols_top, gp.src_batch = rows_top * cols_top;
      gp.src_rows = rows_top, gp.src_cols = cols_top;
    }
    gp.rows_bot = which == 0 ? g.a_rows_bot : g.b_rows_bot;
    gp.cols_bot = which == 0 ? g.a_cols_bot : g.b_cols_bot;
    gp.dst = c.ws + (which == 0 ? g.off_a_bot : g.off_b_bot);
    gp.dst_batch = gp.rows_bot * gp.cols_bot;
    gp.n_in = g.n_in;
    const bool bf16_out = last && p.prec == RBC_PREC_BF16X3;
    const bool f16_out = last && f16s;
    gp.plane = bf16_out ? (int64_t)p.n_leaves * gp.rows_bot * gp.cols_bot : 0;
    gp.scale_exp = f16_out ? exps : nullptr;
    for (int d = g.d0; d < g.d1; ++d)
      fill_side(p, c.dr, d, which == 0 ? SIDE_A : SIDE_B, f64, false, gp.lev[d - g.d0]);
    const int br = which == 0 ? g.b1 : g.b2, bc = which == 0 ? g.b2 : g.b3;
    const int R = p.Q ? p.levels[g.d0].R : 1;
    const int vec = pick_vec(f64 ? 8 : 4, gp.cols_bot, {gp.ld_src, gp.src_batch, gp.dst_batch, gp.plane},
                             {gp.src, gp.dst}, f64, g.d1 - g.d0);
    hipError_t e = launch_gather(f64 ? ELT_F64 : ELT_F32, bf16_out ? OUT_BF16X2 : (f16_out ? OUT_F16S : OUT_SAME), vec,
                                 g.d1 - g.d0, br, bc, R, gp, c.stream);
    if (e != hipSuccess) return fail(RBC_EHIP, "gather launch: %s", hipGetErrorString(e));
  }
  return RBC_OK;
}

rbc_status run_leaf(Ctx& c) {
  Plan& p = c.p;
  hipError_t e;
  if (p.prec == RBC_PREC_F64)
    e = launch_gemm_f64(reinterpret_cast<const double*>(c.ws + p.off_S),
                        reinterpret_cast<const double*>(c.ws + p.off_T),
                        reinterpret_cast<double*>(c.ws + p.off_P), p.mM, p.mN, p.mK, p.n_leaves,
                        c.stream);
  else if (p.prec == RBC_PREC_F32)
    e = launch_gemm_f32(reinterpret_cast<const float*>(c.ws + p.off_S),
                        reinterpret_cast<const float*>(c.ws + p.off_T),
                        reinterpret_cast<float*>(c.ws + p.off_P), p.mM, p.mN, p.mK, p.n_leaves,
                        p.tile_m, c.stream);
  else if (p.prec == RBC_PREC_F16S)
    e = launch_gemm_f16s(reinterpret_cast<const uint16_t*>(c.ws + p.off_S),
                         reinterpret_cast<const uint16_t*>(c.ws + p.off_T),
                         reinterpret_cast<float*>(c.ws + p.off_P), p.mM, p.mN, p.mK, p.n_leaves, p.tile_m,
                         reinterpret_cast<const int32_t*>(c.ws + p.off_aux + 256),
                         reinterpret_cast<const int32_t*>(c.ws + p.off_aux + 256) + p.n_leaves, c.stream);
  else
    e = launch_gemm_bf16x3(reinterpret_cast<const uint16_t*>(c.ws + p.off_S),
                           reinterpret_cast<const uint16_t*>(c.ws + p.off_T),
                           reinterpret_cast<float*>(c.ws + p.off_P), p.mM, p.mN, p.mK, p.n_leaves,
                           p.tile_m, c.stream);
  if (e != hipSuccess) return fail(RBC_EHIP, "leaf launch: %s", hipGetErrorString(e));
  return RBC_OK;
}

rbc_status run_scatter(Ctx& c, bool kappa_scale, void* C, int64_t ldc) {
  Plan& p = c.p;
  const bool f64_tabs = p.prec == RBC_PREC_F64 || p.prec == RBC_PREC_BF16X3;
  for (size_t gi = p.groups.size(); gi-- > 0;) {
    const Group& g = p.groups[gi];
    const bool last = gi + 1 == p.groups.size();
    ScatterParams sp;
    std::memset(&sp, 0, sizeof sp);
    sp.src = c.ws + g.off_c_bot;
    sp.rows_bot = g.c_rows_bot, sp.cols_bot = g.c_cols_bot;
    sp.src_batch = sp.rows_bot * sp.cols_bot;
    if (gi == 0) {
      sp.dst = C, sp.ld_dst = ldc, sp.dst_batch = 0, sp.dst_rows = p.M, sp.dst_cols = p.N;
    } else {
      const Group& up = p.groups[gi - 1];
      sp.dst = c.ws + up.off_c_bot;
      sp.ld_dst = g.c_cols_top, sp.dst_batch = g.c_rows_top * g.c_cols_top;
      sp.dst_rows = g.c_rows_top, sp.dst_cols = g.c_cols_top;
    }
    sp.n_out = g.n_in;
    for (int d = g.d0; d < g.d1; ++d) fill_side(p, c.dr, d, SIDE_C, f64_tabs, kappa_scale, sp.lev[d - g.d0]);
    Elt tp, ta, to;
    if (p.prec == RBC_PREC_F64) tp = ta = to = ELT_F64;
    else if (p.prec == RBC_PREC_F32 || p.prec == RBC_PREC_F16S) tp = ta = to = ELT_F32;
    else tp = last ? ELT_F32 : ELT_F64, ta = ELT_F64, to = gi == 0 ? ELT_F32 : ELT_F64;
    const int R = p.Q ? p.levels[g.d0].R : 1;
    const int vec = pick_vec(to == ELT_F64 ? 8 : 4, sp.cols_bot, {sp.ld_dst, sp.dst_batch, sp.src_batch},
                             {sp.src, sp.dst}, ta == ELT_F64, g.d1 - g.d0);
    hipError_t e = launch_scatter(tp, ta, to, vec, g.d1 - g.d0, g.b1, g.b3, R, sp, c.stream);
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

rbc_status matmul_impl(Plan& p, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
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
  if ((st = record(p, c.stream, 0)) != RBC_OK) return st;
  if ((st = run_gather(c, 0, A, lda)) != RBC_OK) return st;
  if ((st = record(p, c.stream, 1)) != RBC_OK) return st;
  if ((st = run_gather(c, 1, B, ldb)) != RBC_OK) return st;
  if ((st = record(p, c.stream, 2)) != RBC_OK) return st;
  if ((st = run_leaf(c)) != RBC_OK) return st;
  if ((st = record(p, c.stream, 3)) != RBC_OK) return st;
  if ((st = run_scatter(c, kappa_scale != 0, C, ldc)) != RBC_OK) return st;
  if ((st = record(p, c.stream, 4)) != RBC_OK) return st;
  if (p.timing) ++p.recorded;
  return RBC_OK;
}

void seeded_draws(const Plan& p, uint64_t seed, rbc_mode mode, std::vector<int32_t>& s,
                  std::vector<int32_t>& pm) {
  s.clear(), pm.clear();
  for (int d = 0; d < p.Q; ++d) {
    const Scheme& sc = p.levels[d];
    const int n = sc.b1 + sc.b2 + sc.b3;
    const size_t o = s.size();
    s.resize(o + n), pm.resize(o + n);
    draw_level(seed, d, sc.b1, sc.b2, sc.b3, mode, s.data() + o, pm.data() + o);
  }
}

}  // namespace

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
