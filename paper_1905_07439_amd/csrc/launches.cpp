// Host-side construction of kernel launches (see launches.hpp).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <initializer_list>

#include "launches.hpp"

#define HIP_CHECK(expr)                                                             \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return fail(RBC_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

namespace rbc {

static_assert(kAuxExpOffset == 2 * kScalePartials * sizeof(float), "aux layout");


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

namespace {

// Device address of a level's table (null before the tables are uploaded,
// when launch descriptions are built only to size a batch).
const void* table(const Plan& p, int level, TabKind kind, bool f64) {
  const size_t idx = (size_t)level * 8 + (f64 ? 0 : 4) + (size_t)kind;
  if (!p.dev_tables || idx >= p.tab_off.size()) return nullptr;
  return static_cast<const char*>(p.dev_tables) + p.tab_off[idx];
}

enum Side { SIDE_A, SIDE_B, SIDE_C };

// Positions per thread for a combination launch: the widest of 4, 2, 1 that
// divides the block width, every leading dimension and block stride, and the
// element alignment of every pointer.  8-byte accumulators use at most 2, and
// 1 in two-level groups (register budget).  Scatters of two or more levels use
// at most 2: with 4, each thread's R^2 operand loads run in R dependent rounds
// and the launch has too few wavefronts to hide them (measured: the bottom
// scatter of three Strassen levels at N = 4096 in f32 takes 176 us with 4
// positions per thread, 135 us with 2).
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
             std::initializer_list<const void*> ptrs, bool wide_acc, int nl, bool scatter) {
  const int cap = std::min({wide_acc ? (nl >= 2 ? 1 : 2) : 4, scatter && nl >= 2 ? 2 : 4, max_vec_override()});
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
  if (s.b1 == 2 && s.b2 == 2 && s.b3 == 2 && s.R == 7) {
    // the table the kernels read, in their precision, against Strassen's pattern
    const LevelTables& t = p.tables[level];
    bool same = true;
    for (int b = 0; b < 4 && same; ++b)
      for (int r = 0; r < 7 && same; ++r) {
        bool listed = false;
        if (side == SIDE_C) {
          for (int n = 0; n < kStrassenWNzCount[b]; ++n) listed = listed || kStrassenWNz[b][n] == r;
        } else {
          const int* nz = side == SIDE_A ? kStrassenUNz[r] : kStrassenVNz[r];
          listed = nz[0] == b || nz[1] == b;
        }
        const size_t i = (size_t)b * 7 + r;
        double v;
        if (side == SIDE_A) v = f64 ? t.U[i] : (double)t.Uf[i];
        else if (side == SIDE_B) v = f64 ? t.V[i] : (double)t.Vf[i];
        else v = f64 ? (kappa_scale ? t.Wk[i] : t.W[i]) : (double)(kappa_scale ? t.Wkf[i] : t.Wf[i]);
        same = (v != 0.0) == listed;
      }
    L.strassen = same ? 1 : 0;
  }
}

}  // namespace

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

rbc_status check_ws(const Plan& p, void* ws, size_t bytes) {
  if (!ws) return fail(RBC_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(RBC_EINVAL, "workspace not 256-byte aligned");
  if (bytes < p.ws_bytes)
    return fail(RBC_ENOMEM, "workspace of %zu bytes, plan needs %zu", bytes, p.ws_bytes);
  return RBC_OK;
}

void build_gather(const Plan& p, const Draws& dr, int which, const void* X, int64_t ldx, char* ws,
                  std::vector<ScaleLaunch>& scale, std::vector<GatherLaunch>& out, bool leaf_gather) {
  scale.clear(), out.clear();
  const std::vector<Group>& groups = leaf_gather ? p.fgroups : p.groups;
  const bool f64 = p.prec == RBC_PREC_F64;
  const bool scaled = p.prec == RBC_PREC_F16S || p.prec == RBC_PREC_FP8C;
  int32_t* exps = nullptr;
  if (scaled) {
    ScaleLaunch sl;
    sl.X = static_cast<const float*>(X), sl.ld = ldx;
    sl.rows = which == 0 ? p.M : p.K, sl.cols = which == 0 ? p.K : p.N;
    sl.partial = reinterpret_cast<float*>(ws + p.off_aux) + (size_t)which * kScalePartials;
    exps = reinterpret_cast<int32_t*>(ws + p.off_aux + kAuxExpOffset) + (size_t)which * p.n_leaves;
    sl.G = reinterpret_cast<const float*>(static_cast<const char*>(p.dev_tables) + p.g_off[which]);
    sl.e = exps, sl.n_leaves = p.n_leaves;
    sl.target = p.prec == RBC_PREC_FP8C ? 448.0f : 32768.0f;
    scale.push_back(sl);
  }
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Group& g = groups[gi];
    const bool last = gi + 1 == groups.size() && !leaf_gather;  // writes the leaf operands
    GatherLaunch L;
    GatherParams& gp = L.p;
    std::memset(&gp, 0, sizeof gp);
    const int64_t rows_top = which == 0 ? g.a_rows_top : g.b_rows_top;
    const int64_t cols_top = which == 0 ? g.a_cols_top : g.b_cols_top;
    if (gi == 0) {
      gp.src = X, gp.ld_src = ldx, gp.src_batch = 0;
      gp.src_rows = which == 0 ? p.M : p.K;
      gp.src_cols = which == 0 ? p.K : p.N;
    } else {
      const Group& up = groups[gi - 1];
      gp.src = ws + (which == 0 ? up.off_a_bot : up.off_b_bot);
      gp.ld_src = cols_top, gp.src_batch = rows_top * cols_top;
      gp.src_rows = rows_top, gp.src_cols = cols_top;
    }
    gp.rows_bot = which == 0 ? g.a_rows_bot : g.b_rows_bot;
    gp.cols_bot = which == 0 ? g.a_cols_bot : g.b_cols_bot;
    gp.dst = ws + (which == 0 ? g.off_a_bot : g.off_b_bot);
    gp.dst_batch = gp.rows_bot * gp.cols_bot;
    gp.n_in = g.n_in;
    gp.nt_store = gi + 1 < groups.size() ? 1 : 0;
    gp.side = which;
    const bool bf16_out = last && p.prec == RBC_PREC_BF16X3;
    const bool f16_out = last && p.prec == RBC_PREC_F16S;
    const bool fp8_out = last && p.prec == RBC_PREC_FP8C;
    gp.plane = (bf16_out || fp8_out) ? (int64_t)p.n_leaves * gp.rows_bot * gp.cols_bot : 0;
    gp.scale_exp = (f16_out || fp8_out) ? exps : nullptr;
    gp.scale_partial = nullptr, gp.scale_G = nullptr, gp.scale_nparts = 0, gp.scale_target = 0.f;
    if (f16_out || fp8_out) {  // the exponents are derived by this gather (load_exponents)
      const ScaleLaunch& sl = scale[0];
      gp.scale_partial = sl.partial, gp.scale_G = sl.G, gp.scale_target = sl.target;
      gp.scale_nparts = maxabs_blocks(sl.rows, sl.cols);
    }
    for (int d = g.d0; d < g.d1; ++d)
      fill_side(p, dr, d, which == 0 ? SIDE_A : SIDE_B, f64, false, gp.lev[d - g.d0]);
    L.br = which == 0 ? g.b1 : g.b2, L.bc = which == 0 ? g.b2 : g.b3;
    L.R = p.Q ? p.levels[g.d0].R : 1;
    L.nl = g.d1 - g.d0;
    L.vec = pick_vec(f64 ? 8 : 4, gp.cols_bot, {gp.ld_src, gp.src_batch, gp.dst_batch, gp.plane},
                     {gp.src, gp.dst}, f64, L.nl, false);
    L.elt = f64 ? ELT_F64 : ELT_F32;
    L.out = bf16_out ? OUT_BF16X2 : (f16_out ? OUT_F16S : (fp8_out ? OUT_FP8X2 : OUT_SAME));
    out.push_back(L);
  }
}

LeafLaunch build_leaf(const Plan& p, char* ws) {
  LeafLaunch L;
  L.prec = p.prec;
  L.S = ws + p.off_S, L.T = ws + p.off_T, L.P = ws + p.off_P;
  L.m = p.mM, L.n = p.mN, L.k = p.mK, L.batch = p.n_leaves, L.tile = p.tile_m;
  L.masked = p.exact_blocks;
  L.eS = L.eT = nullptr;
  if (p.prec == RBC_PREC_F16S || p.prec == RBC_PREC_FP8C) {
    L.eS = reinterpret_cast<const int32_t*>(ws + p.off_aux + kAuxExpOffset);
    L.eT = L.eS + p.n_leaves;
  }
  return L;
}

LeafGatherLaunch build_leaf_gather(const Plan& p, const Draws& dr, char* ws, bool leaf_scatter,
                                   bool kappa_scale) {
  LeafGatherLaunch L;
  std::memset(&L.g, 0, sizeof L.g);
  std::memset(&L.ls, 0, sizeof L.ls);
  const Group& up = p.fgroups.back();
  const Scheme& s = p.levels[p.Q - 1];
  LeafGather& g = L.g;
  g.A = reinterpret_cast<const float*>(ws + up.off_a_bot);
  g.B = reinterpret_cast<const float*>(ws + up.off_b_bot);
  g.a_ld = up.a_cols_bot, g.a_batch = up.a_rows_bot * up.a_cols_bot;
  g.b_ld = up.b_cols_bot, g.b_batch = up.b_rows_bot * up.b_cols_bot;
  g.a_row_blk = p.mM * g.a_ld, g.a_col_blk = p.mK;
  g.b_row_blk = p.mK * g.b_ld, g.b_col_blk = p.mN;
  fill_side(p, dr, p.Q - 1, SIDE_A, false, false, g.la);
  fill_side(p, dr, p.Q - 1, SIDE_B, false, false, g.lb);
  g.bra = s.b1, g.bca = s.b2, g.brb = s.b2, g.bcb = s.b3, g.R = s.R;
  L.P = reinterpret_cast<float*>(ws + p.off_P);
  L.m = p.mM, L.n = p.mN, L.k = p.mK, L.batch = p.n_leaves, L.tile = p.tile_m;
  L.scatter = leaf_scatter;
  if (leaf_scatter) {
    LeafScatter& ls = L.ls;
    ls.out = reinterpret_cast<float*>(ws + p.off_pc);
    ls.cnt = reinterpret_cast<int32_t*>(ws + p.off_cnt);
    ls.out_ld = up.c_cols_bot, ls.out_batch = up.c_rows_bot * up.c_cols_bot;
    ls.row_blk = p.mM * ls.out_ld, ls.col_blk = p.mN;
    fill_side(p, dr, p.Q - 1, SIDE_C, false, kappa_scale, ls.lw);
    ls.br = s.b1, ls.bc = s.b3;
  }
  return L;
}

void build_scatter(const Plan& p, const Draws& dr, bool kappa_scale, void* C, int64_t ldc, char* ws,
                   std::vector<ScatterLaunch>& out, const std::vector<Group>& groups, bool from_parents) {
  out.clear();
  const bool f64_tabs = p.prec == RBC_PREC_F64 || p.prec == RBC_PREC_BF16X3;
  for (size_t gi = groups.size(); gi-- > 0;) {
    const Group& g = groups[gi];
    const bool last = gi + 1 == groups.size() && !from_parents;
    ScatterLaunch L;
    ScatterParams& sp = L.p;
    std::memset(&sp, 0, sizeof sp);
    sp.src = ws + g.off_c_bot;
    sp.rows_bot = g.c_rows_bot, sp.cols_bot = g.c_cols_bot;
    sp.src_batch = sp.rows_bot * sp.cols_bot;
    if (gi == 0) {
      sp.dst = C, sp.ld_dst = ldc, sp.dst_batch = 0, sp.dst_rows = p.M, sp.dst_cols = p.N;
    } else {
      const Group& up = groups[gi - 1];
      sp.dst = ws + up.off_c_bot;
      sp.ld_dst = g.c_cols_top, sp.dst_batch = g.c_rows_top * g.c_cols_top;
      sp.dst_rows = g.c_rows_top, sp.dst_cols = g.c_cols_top;
    }
    sp.n_out = g.n_in;
    for (int d = g.d0; d < g.d1; ++d) fill_side(p, dr, d, SIDE_C, f64_tabs, kappa_scale, sp.lev[d - g.d0]);
    if (p.prec == RBC_PREC_F64) L.tp = L.ta = L.to = ELT_F64;
    else if (p.prec == RBC_PREC_F32 || p.prec == RBC_PREC_F16S || p.prec == RBC_PREC_FP8C)
      L.tp = L.ta = L.to = ELT_F32;
    else L.tp = last ? ELT_F32 : ELT_F64, L.ta = ELT_F64, L.to = gi == 0 ? ELT_F32 : ELT_F64;
    L.R = p.Q ? p.levels[g.d0].R : 1;
    L.nl = g.d1 - g.d0;
    L.br = g.b1, L.bc = g.b3;
    L.vec = pick_vec(L.to == ELT_F64 ? 8 : 4, sp.cols_bot, {sp.ld_dst, sp.dst_batch, sp.src_batch},
                     {sp.src, sp.dst}, L.ta == ELT_F64, L.nl, true);
    out.push_back(L);
  }
}

hipError_t launch(const ScaleLaunch& l, hipStream_t s) {
  return launch_maxabs(l.X, l.ld, l.rows, l.cols, l.partial, s);
}

hipError_t launch(const ScaleLaunch& a, const ScaleLaunch& b, hipStream_t s) {
  return launch_maxabs2(a.X, a.ld, a.rows, a.cols, a.partial, b.X, b.ld, b.rows, b.cols, b.partial, s);
}

hipError_t launch(const GatherLaunch& l, hipStream_t s) {
  return launch_gather(l.elt, l.out, l.vec, l.nl, l.br, l.bc, l.R, l.p, s);
}

hipError_t launch(const GatherLaunch& a, const GatherLaunch& b, hipStream_t s) {
  if (a.elt != b.elt || a.out != b.out || a.nl != b.nl || a.br != b.br || a.bc != b.bc || a.R != b.R) {
    hipError_t e = launch(a, s);
    return e != hipSuccess ? e : launch(b, s);
  }
  // any narrower vec than the host picked for a side is valid for it
  const int vec = a.vec < b.vec ? a.vec : b.vec;
  return launch_gather2(a.elt, a.out, vec, a.nl, a.br, a.bc, a.R, a.p, b.p, s);
}

hipError_t launch(const LeafLaunch& l, hipStream_t s) {
  if (l.masked) {
    if (l.prec == RBC_PREC_F64)
      return launch_gemm_f64_masked(static_cast<const double*>(l.S), static_cast<const double*>(l.T),
                                    static_cast<double*>(l.P), l.m, l.n, l.k, l.batch, s);
    if (l.prec == RBC_PREC_F32)
      return launch_gemm_f32_masked(static_cast<const float*>(l.S), static_cast<const float*>(l.T),
                                    static_cast<float*>(l.P), l.m, l.n, l.k, l.batch, s);
    return hipErrorInvalidValue;
  }
  switch (l.prec) {
    case RBC_PREC_F64:
      return launch_gemm_f64(static_cast<const double*>(l.S), static_cast<const double*>(l.T),
                             static_cast<double*>(l.P), l.m, l.n, l.k, l.batch, s);
    case RBC_PREC_F32:
      return launch_gemm_f32(static_cast<const float*>(l.S), static_cast<const float*>(l.T),
                             static_cast<float*>(l.P), l.m, l.n, l.k, l.batch, l.tile, s);
    case RBC_PREC_F16S:
      return launch_gemm_f16s(static_cast<const uint16_t*>(l.S), static_cast<const uint16_t*>(l.T),
                              static_cast<float*>(l.P), l.m, l.n, l.k, l.batch, l.tile, l.eS, l.eT, s);
    case RBC_PREC_FP8C:
      return launch_gemm_fp8c(static_cast<const uint8_t*>(l.S), static_cast<const uint8_t*>(l.T),
                              static_cast<float*>(l.P), l.m, l.n, l.k, l.batch, l.tile, l.eS, l.eT, s);
    case RBC_PREC_BF16X3:
      return launch_gemm_bf16x3(static_cast<const uint16_t*>(l.S), static_cast<const uint16_t*>(l.T),
                                static_cast<float*>(l.P), l.m, l.n, l.k, l.batch, l.tile, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch(const LeafGatherLaunch& l, hipStream_t s) {
  return launch_gemm_f32_gathered(l.g, l.P, l.m, l.n, l.k, l.batch, l.tile, s, l.scatter ? &l.ls : nullptr);
}

hipError_t launch(const ScatterLaunch& l, hipStream_t s) {
  return launch_scatter(l.tp, l.ta, l.to, l.vec, l.nl, l.br, l.bc, l.R, l.p, s);
}

}  // namespace rbc
