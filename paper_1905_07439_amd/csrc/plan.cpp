// Planner: leaf sizes, zero padding, fused level groups and the workspace
// layout of F-hat^(Q) (Section 2.1.1, eq. recursive-random-formula).
//
// The recursion is evaluated breadth-first over fused groups of levels: the
// gather of a group turns every block entering it into the prod R_d blocks of
// its deepest level in one kernel pass, the leaf kernel multiplies all
// prod_d R_d leaf pairs in one batched launch, and the scatter of a group
// folds its products back through W.  Padding (end of Section 2.1.1) is
// virtual: reads outside A or B return zero, writes outside C are dropped.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "core.hpp"

namespace rbc {

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }
static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Fused group shapes the block-combination kernels are compiled for: one
// level of any shape, or two or three Strassen-shaped levels (2x2x2, R = 7).
// A thread holds prod (b_row b_col) source values of the group, at most 64.
bool fused_supported(int b1, int b2, int b3, int R, int nl) {
  if (nl <= 1) return true;
  const bool strassen_shape = b1 == 2 && b2 == 2 && b3 == 2 && R == 7;
  return (nl == 2 || nl == 3) && strassen_shape;
}

// Most levels one pass fuses.  Three fused levels in one thread need about
// 100 values in registers, which costs occupancy: gathers take two.  Scatters
// take three (scatter = true): k_scatter3 spreads the top level over the
// wavefronts of its workgroup.  The environment variable RBC_MAX_FUSED_LEVELS
// overrides both.
static int max_fused_levels(bool scatter = false) {
  const char* e = std::getenv("RBC_MAX_FUSED_LEVELS");
  if (e && *e) {
    const int v = std::atoi(e);
    if (v >= 1 && v <= 3) return v;
  }
  if (scatter) return 3;
  return 2;
}

static bool same_shape(const Scheme& a, const Scheme& b) {
  return a.b1 == b.b1 && a.b2 == b.b2 && a.b3 == b.b3 && a.R == b.R;
}

// Fused groups over levels [0, d_end), formed from the deepest level upwards so
// that the boundaries between passes sit where the intermediate blocks are
// fewest, with their block dimensions (bottom blocks of levels below d_end
// included: the leaves are always mM x mK and mK x mN).
// Levels [d, g_d1) fused into one pass give each thread R_d times the sequential
// work of the pass below; that pays only when the pass has enough parallel work:
// (top blocks entering the pass) x (elements of one bottom block), the larger of
// the A and B sides, at least 2^18.  Measured (products per second, Strassen):
// below it one-level passes won (f64 N = 256, Q = 3: 54.5 -> 34.9 us; fp8c N = 512,
// Q = 2: 38.6 -> 28.5 us; f32 N = 1024, Q = 3: 74.4 -> 64.5 us), from it on the fused
// pass won (fp8c N = 2048, Q = 2: 91.7 vs 109.5 us; f16s 89 vs 109 us; f32 N = 4096,
// Q = 2: 977 vs 1054 us; Q = 3 at N = 2048: 203 vs 231 us).  RBC_MAX_FUSED_LEVELS set
// in the environment overrides the rule.
static bool enough_work(const Plan& p, int d, int g_d1) {
  const char* env = std::getenv("RBC_MAX_FUSED_LEVELS");
  if (p.fuse_max || (env && *env)) return true;
  double n_in = 1, a = (double)p.mM * p.mK, b = (double)p.mK * p.mN;
  for (int e = 0; e < d; ++e) n_in *= p.levels[e].R;
  for (int e = g_d1; e < p.Q; ++e) {
    const Scheme& s = p.levels[e];
    a *= (double)s.b1 * s.b2, b *= (double)s.b2 * s.b3;
  }
  return n_in * (a > b ? a : b) >= 262144.0;
}

static std::vector<Group> form_groups(const Plan& p, int d_end, int max_nl) {
  const std::vector<Scheme>& levels = p.levels;
  std::vector<Group> gs;
  for (int d = d_end - 1; d >= 0; --d) {
    const Scheme& s = levels[d];
    if (!gs.empty()) {
      Group& g = gs.back();  // the group just below, levels [g.d0, g.d1)
      const int nl = g.d1 - g.d0 + 1;
      if (nl <= max_nl && same_shape(s, levels[g.d0]) && fused_supported(s.b1, s.b2, s.b3, s.R, nl) &&
          enough_work(p, d, g.d1)) {
        g.d0 = d;
        continue;
      }
    }
    Group g;
    g.d0 = d, g.d1 = d + 1;
    g.b1 = s.b1, g.b2 = s.b2, g.b3 = s.b3;
    gs.push_back(g);
  }
  std::reverse(gs.begin(), gs.end());
  if (p.Q == 0) {  // plain product: one empty group copies A, B in and C out
    Group g;
    g.b1 = g.b2 = g.b3 = 1;
    gs.push_back(g);
  }
  int64_t n_in = 1;
  for (Group& g : gs) {
    int64_t q1 = 1, q2 = 1, q3 = 1, below1 = 1, below2 = 1, below3 = 1;
    for (int d = g.d0; d < g.d1; ++d) q1 *= levels[d].b1, q2 *= levels[d].b2, q3 *= levels[d].b3;
    for (int d = g.d1; d < p.Q; ++d)
      below1 *= levels[d].b1, below2 *= levels[d].b2, below3 *= levels[d].b3;
    g.n_in = n_in;
    g.Rg = 1;
    for (int d = g.d0; d < g.d1; ++d) g.Rg *= levels[d].R;
    g.a_rows_bot = p.mM * below1, g.a_cols_bot = p.mK * below2;
    g.b_rows_bot = p.mK * below2, g.b_cols_bot = p.mN * below3;
    g.c_rows_bot = p.mM * below1, g.c_cols_bot = p.mN * below3;
    g.a_rows_top = g.a_rows_bot * q1, g.a_cols_top = g.a_cols_bot * q2;
    g.b_rows_top = g.b_rows_bot * q2, g.b_cols_top = g.b_cols_bot * q3;
    g.c_rows_top = g.c_rows_bot * q1, g.c_cols_top = g.c_cols_bot * q3;
    n_in *= g.Rg;
  }
  return gs;
}

// At most two nonzero coefficients (as f32, the precision the kernels read)
// in every column r of U and of V: the leaf product's loads can then form the
// operands (LeafGather).
static bool two_terms(const Scheme& s) {
  for (int r = 0; r < s.R; ++r) {
    int nu = 0, nv = 0;
    for (int i = 0; i < s.b1 * s.b2; ++i) nu += (float)s.U[i * s.R + r] != 0.0f;
    for (int i = 0; i < s.b2 * s.b3; ++i) nv += (float)s.V[i * s.R + r] != 0.0f;
    if (nu > 2 || nv > 2) return false;
  }
  return true;
}

// RBC_LEAF_GATHER=0 turns the leaf gather off for every new plan, =1 on
// wherever it qualifies; unset, it is on where the cost model below favours it.
static int leaf_gather_env() {
  const char* e = std::getenv("RBC_LEAF_GATHER");
  return (e && (e[0] == '0' || e[0] == '1')) ? e[0] - '0' : -1;
}

// RBC_LEAF_SCATTER=1 turns the leaf scatter on for every new plan that takes
// the leaf gather; unset or 0, it is off (it costs more than it saves: f32
// Strassen F-hat^(3) at N = 4096, leaf 0.78 -> 1.10 ms against a scatter
// 0.117 -> 0.058 ms; of the 0.32 ms, about 0.14 ms are the release fences'
// L2 write-backs, one per leaf tile, and 0.18 ms the combinations, whose
// loads the waiting tile slots cannot hide).
static int leaf_scatter_env() {
  const char* e = std::getenv("RBC_LEAF_SCATTER");
  return (e && (e[0] == '0' || e[0] == '1')) ? e[0] - '0' : -1;
}

// f32 bytes the gathers of A and B move over `gs` (each top block read once,
// each bottom block written once).
static double gather_bytes(const Plan& p, const std::vector<Group>& gs) {
  double b = 0;
  for (size_t gi = 0; gi < gs.size(); ++gi) {
    const Group& g = gs[gi];
    const double n_out = (double)g.n_in * g.Rg;
    b += gi == 0 ? (double)p.M * p.K + (double)p.K * p.N
                 : (double)g.n_in * ((double)g.a_rows_top * g.a_cols_top + (double)g.b_rows_top * g.b_cols_top);
    b += n_out * ((double)g.a_rows_bot * g.a_cols_bot + (double)g.b_rows_bot * g.b_cols_bot);
  }
  return 4 * b;
}

// Whether the leaf gather pays: the gathers it saves (at 5 TB/s, what they
// reach) against the leaf product's slowdown from loading up to two
// sub-blocks per operand (about 9% at 125 TF/s; measured at N = 4096: Q = 3
// gathers 130 -> 57 us each and the leaf 749 -> 806 us, a gain; Q = 2 gathers
// 53 -> 41 us and the leaf 810 -> 890 us, a loss).
static bool leaf_gather_pays(const Plan& p) {
  const double saved_us = (gather_bytes(p, p.groups) - gather_bytes(p, p.fgroups)) / 5e6;
  const double flops = 2.0 * p.n_leaves * (double)p.mM * p.mK * p.mN;
  return saved_us > 0.09 * flops / 125e6;
}

void layout_leaf_scatter(Plan& p) {
  if (!p.leaf_scatter_ok || p.off_cnt) return;
  size_t off = align256(p.ws_bytes);
  for (size_t gi = 0; gi < p.fgroups.size(); ++gi) {
    Group& g = p.fgroups[gi];
    const size_t nb = (size_t)g.n_in * g.Rg;
    g.off_c_bot = off, off = align256(off + nb * g.c_rows_bot * g.c_cols_bot * 4);
  }
  const Group& g = p.fgroups.back();
  p.off_pc = g.off_c_bot;
  p.n_cnt = (int64_t)g.n_in * g.Rg * (p.mM / 64) * (p.mN / 64);
  p.off_cnt = off, off = align256(off + (size_t)p.n_cnt * 4);
  p.ws_bytes = off;
}

rbc_status make_plan(int64_t M, int64_t K, int64_t N, const std::vector<Scheme>& levels,
                     rbc_prec prec, int leaf_tile, Plan& out, bool fuse_max) {
  if (M < 1 || K < 1 || N < 1) return fail(RBC_EINVAL, "empty product %lldx%lldx%lld", (long long)M,
                                          (long long)K, (long long)N);
  if ((int)levels.size() > kMaxLevels) return fail(RBC_EINVAL, "at most %d levels", kMaxLevels);
  if (prec != RBC_PREC_F64 && prec != RBC_PREC_F32 && prec != RBC_PREC_BF16X3 && prec != RBC_PREC_F16S &&
      prec != RBC_PREC_FP8C)
    return fail(RBC_EUNSUPPORTED, "precision %d not implemented", (int)prec);
  Plan p;
  p.M = M, p.K = K, p.N = N;
  p.Q = (int)levels.size();
  p.prec = prec;
  p.levels = levels;
  p.fuse_max = fuse_max;

  int64_t P1 = 1, P2 = 1, P3 = 1;
  p.n_leaves = 1;
  for (const Scheme& s : levels) {
    P1 *= s.b1, P2 *= s.b2, P3 *= s.b3;
    p.n_leaves *= s.R;
  }
  const int64_t lm = ceil_div(M, P1), lk = ceil_div(K, P2), ln = ceil_div(N, P3);

  // Leaf GEMM tile.
  if (leaf_tile == -1) {  // exact blocks: leaves of any size, masked leaf kernels
    if (prec != RBC_PREC_F64 && prec != RBC_PREC_F32)
      return fail(RBC_EUNSUPPORTED, "exact blocks (leaf_tile -1) for f64 and f32 only");
    p.exact_blocks = true;
    p.tile_m = p.tile_n = p.tile_k = 1;
  } else if (prec == RBC_PREC_F64) {
    if (leaf_tile == 0) leaf_tile = 16;
    if (leaf_tile != 16) return fail(RBC_EUNSUPPORTED, "f64 leaf tile must be 16");
    p.tile_m = p.tile_n = 16, p.tile_k = 4;
  } else if (prec == RBC_PREC_F16S || prec == RBC_PREC_FP8C) {
    if (leaf_tile == 0) {
      // the tile with the least padded leaf area (ties: the larger tile)
      int64_t best = -1;
      for (int t : {128, 96, 64, 32}) {
        const int64_t area = round_up(lm, t) * round_up(ln, t);
        if (best < 0 || area < best) best = area, leaf_tile = t;
      }
    }
    if (leaf_tile != 32 && leaf_tile != 64 && leaf_tile != 96 && leaf_tile != 128)
      return fail(RBC_EUNSUPPORTED, "f16s / fp8c leaf tile must be 32, 64, 96 or 128");
    p.tile_m = p.tile_n = leaf_tile;
    p.tile_k = prec == RBC_PREC_FP8C ? 64 : 32;
  } else {
    if (leaf_tile == 0) {
      // 128 unless it pads the leaf by more than 1/8
      const bool big = round_up(lm, 128) * 8 <= lm * 9 && round_up(ln, 128) * 8 <= ln * 9;
      leaf_tile = big ? 128 : 64;
    }
    if (leaf_tile != 64 && leaf_tile != 128)
      return fail(RBC_EUNSUPPORTED, "f32/bf16x3 leaf tile must be 64 or 128");
    p.tile_m = p.tile_n = leaf_tile;
    p.tile_k = prec == RBC_PREC_BF16X3 ? 32 : 16;
  }
  p.mM = round_up(lm, p.tile_m);
  p.mK = round_up(lk, p.tile_k);
  p.mN = round_up(ln, p.tile_n);
  p.Mp = p.mM * P1, p.Kp = p.mK * P2, p.Np = p.mN * P3;

  p.comb_bytes = prec == RBC_PREC_F64 ? 8 : 4;
  p.recomb_bytes = (prec == RBC_PREC_F64 || prec == RBC_PREC_BF16X3) ? 8 : 4;
  // bf16x3: hi + lo planes of 2 bytes; f16s: one plane of 2 bytes
  // fp8c: hi + lo planes of 1 byte
  const int leaf_op_bytes = prec == RBC_PREC_F64 ? 8 : ((prec == RBC_PREC_F16S || prec == RBC_PREC_FP8C) ? 2 : 4);
  const int prod_bytes = prec == RBC_PREC_F64 ? 8 : 4;

  p.groups = form_groups(p, p.Q, max_fused_levels());
  p.sgroups = form_groups(p, p.Q, max_fused_levels(true));
  p.leaf_gather_ok = prec == RBC_PREC_F32 && !p.exact_blocks && p.Q >= 2 && two_terms(levels[p.Q - 1]);
  if (p.leaf_gather_ok) p.fgroups = form_groups(p, p.Q - 1, max_fused_levels());

  // Workspace: leaf operands, products, then the group-boundary buffers.
  size_t off = 0;
  p.bytes_S = (size_t)p.n_leaves * p.mM * p.mK * leaf_op_bytes;
  p.bytes_T = (size_t)p.n_leaves * p.mK * p.mN * leaf_op_bytes;
  p.bytes_P = (size_t)p.n_leaves * p.mM * p.mN * prod_bytes;
  p.off_S = off, off = align256(off + p.bytes_S);
  p.off_T = off, off = align256(off + p.bytes_T);
  p.off_P = off, off = align256(off + p.bytes_P);
  for (size_t gi = 0; gi < p.groups.size(); ++gi) {
    Group& g = p.groups[gi];
    if (gi + 1 == p.groups.size()) {
      g.off_a_bot = p.off_S, g.off_b_bot = p.off_T, g.off_c_bot = p.off_P;
      continue;
    }
    const size_t nb = (size_t)g.n_in * g.Rg;
    g.off_a_bot = off, off = align256(off + nb * g.a_rows_bot * g.a_cols_bot * p.comb_bytes);
    g.off_b_bot = off, off = align256(off + nb * g.b_rows_bot * g.b_cols_bot * p.comb_bytes);
    g.off_c_bot = off, off = align256(off + nb * g.c_rows_bot * g.c_cols_bot * p.recomb_bytes);
  }
  // Scatter groups: a boundary that `groups` also has shares its buffer; any
  // other takes a buffer of `groups` that no scatter group uses, if one is
  // large enough, else a new one.
  {
    std::vector<bool> used(p.groups.size(), false);
    for (size_t gi = 0; gi + 1 < p.sgroups.size(); ++gi)
      for (size_t h = 0; h + 1 < p.groups.size(); ++h)
        if (p.groups[h].d1 == p.sgroups[gi].d1) used[h] = true;
    for (size_t gi = 0; gi < p.sgroups.size(); ++gi) {
      Group& g = p.sgroups[gi];
      g.off_a_bot = g.off_b_bot = 0;  // gathers never run over these groups
      if (gi + 1 == p.sgroups.size()) {
        g.off_c_bot = p.off_P;
        continue;
      }
      const size_t need = (size_t)g.n_in * g.Rg * g.c_rows_bot * g.c_cols_bot * p.recomb_bytes;
      bool placed = false;
      for (size_t h = 0; h + 1 < p.groups.size() && !placed; ++h) {
        const Group& o = p.groups[h];
        if (o.d1 == g.d1) g.off_c_bot = o.off_c_bot, placed = true;
      }
      for (size_t h = 0; h + 1 < p.groups.size() && !placed; ++h) {
        const Group& o = p.groups[h];
        if (!used[h] && (size_t)o.n_in * o.Rg * o.c_rows_bot * o.c_cols_bot * p.recomb_bytes >= need)
          g.off_c_bot = o.off_c_bot, used[h] = true, placed = true;
      }
      if (!placed) g.off_c_bot = off, off = align256(off + need);
    }
  }
  // Leaf gather: the leaves' parents go where the leaf operands would be when
  // they fit (the two paths never run at once on one workspace).
  for (size_t gi = 0; gi < p.fgroups.size(); ++gi) {
    Group& g = p.fgroups[gi];
    const size_t nb = (size_t)g.n_in * g.Rg;
    const size_t ba = nb * g.a_rows_bot * g.a_cols_bot * 4, bb = nb * g.b_rows_bot * g.b_cols_bot * 4;
    const bool last = gi + 1 == p.fgroups.size();
    if (last && ba <= p.bytes_S) g.off_a_bot = p.off_S;
    else g.off_a_bot = off, off = align256(off + ba);
    if (last && bb <= p.bytes_T) g.off_b_bot = p.off_T;
    else g.off_b_bot = off, off = align256(off + bb);
  }
  p.leaf_scatter_ok = p.leaf_gather_ok && p.mM % 64 == 0 && p.mN % 64 == 0;
  const int env = leaf_gather_env();
  p.leaf_gather = p.leaf_gather_ok && (env < 0 ? leaf_gather_pays(p) : env == 1);
  p.leaf_scatter = p.leaf_gather && p.leaf_scatter_ok && leaf_scatter_env() == 1;
  if (prec == RBC_PREC_F16S || prec == RBC_PREC_FP8C) {
    p.off_aux = off;
    p.bytes_aux = kAuxExpOffset + 2 * (size_t)p.n_leaves * 4;
    off = align256(off + p.bytes_aux);
    // per-leaf path norms: leaf l = (r_0, ..., r_{Q-1}), r_{Q-1} fastest
    p.gA.assign(p.n_leaves, 1.0f), p.gB.assign(p.n_leaves, 1.0f);
    for (int64_t l = 0; l < p.n_leaves; ++l) {
      double ga = 1.0, gb = 1.0;
      int64_t rem = l;
      for (int d = p.Q - 1; d >= 0; --d) {
        const Scheme& s = levels[d];
        const int r = (int)(rem % s.R);
        rem /= s.R;
        double nu = 0, nv = 0;
        for (int i = 0; i < s.b1 * s.b2; ++i) nu += std::fabs(s.U[i * s.R + r]);
        for (int i = 0; i < s.b2 * s.b3; ++i) nv += std::fabs(s.V[i * s.R + r]);
        ga *= nu, gb *= nv;
      }
      p.gA[l] = (float)ga, p.gB[l] = (float)gb;
    }
  }
  p.ws_bytes = std::max<size_t>(off, 256);
  if (p.leaf_scatter) layout_leaf_scatter(p);

  // Host tables per level: U, V, W and (1 - kappa)^-1 W, in f64 and f32.
  for (const Scheme& s : levels) {
    LevelTables t;
    t.U = s.U, t.V = s.V, t.W = s.W;
    const double c = kappa_factor(s);
    t.Wk.resize(s.W.size());
    for (size_t i = 0; i < s.W.size(); ++i) t.Wk[i] = c * s.W[i];
    auto to_f = [](const std::vector<double>& v) {
      std::vector<float> f(v.size());
      for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
      return f;
    };
    t.Uf = to_f(t.U), t.Vf = to_f(t.V), t.Wf = to_f(t.W), t.Wkf = to_f(t.Wk);
    p.tables.push_back(std::move(t));
  }
  out = std::move(p);
  return RBC_OK;
}

}  // namespace rbc
