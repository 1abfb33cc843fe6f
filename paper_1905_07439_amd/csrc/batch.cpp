// Batch engine, host side: task construction, workspace layout, launch and
// graph capture (the task model is described in batch.hpp).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "batch.hpp"
#include "handles.hpp"
#include "launches.hpp"

using namespace rbc;
using namespace rbc::batch;

#define HIP_CHECK(expr)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(RBC_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

namespace {

constexpr size_t kAlign = 256;
int64_t ipow(int64_t b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Item {
  Plan* plan;
  const void* A;
  int64_t lda;
  const void* B;
  int64_t ldb;
  void* C;
  int64_t ldc;
  uint64_t seed;
  rbc_mode mode;
  int kappa_scale;
};

struct Layout {  // byte offsets inside the batch workspace
  size_t tasks = 0, gather = 0, scatter = 0, leaf = 0, scale = 0, ctl = 0, trace = 0, pieces = 0, items = 0,
         total = 0;
  std::vector<size_t> item_ws;
};

}  // namespace

struct rbc_batch_s {
  rbc_batch_options opt;
  int prec = -1;
  std::vector<Item> items;
  // built by prepare
  std::vector<Task> tasks;
  std::vector<GatherParams> gparams;
  std::vector<ScatterParams> sparams;
  std::vector<LeafDesc> lparams;
  std::vector<ScaleDesc> cparams;
  std::vector<int32_t> cslots;  // per scale descriptor: counter word holding max|X| bits
  int64_t n_counters = 0;
  Layout lay;
  // RBC_BATCH_LEVELS: launches in order, each a range of (task, piece) entries
  struct GroupLaunch {
    int32_t level, kind, variant;
    int64_t begin, n;
  };
  std::vector<GroupLaunch> launches;
  std::vector<int32_t> piece_table;  // pairs (task, piece)
  int64_t n_levels = 0;
  std::vector<int32_t> item_gate, item_done;  // per item: counters, from the last build
  std::vector<int64_t> item_first;            // per item: queue index of its first task
  std::vector<int32_t> task_item;             // per task: its item (gates: the gated item)
  char* ws = nullptr;
  int device = -1;
  int grid = 0;
  int64_t timeout_ticks = 0;
  bool prepared = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t graph_stream = nullptr;
  // The task table's upload reads the host vectors: they must not change
  // until this event (recorded after the copies) has completed.
  hipEvent_t uploaded = nullptr;
  bool upload_pending = false;
};

namespace {
rbc_status wait_upload(rbc_batch_s& b) {
  if (b.upload_pending) {
    hipError_t e = hipEventSynchronize(b.uploaded);
    if (e != hipSuccess) return fail(RBC_EHIP, "hipEventSynchronize: %s", hipGetErrorString(e));
    b.upload_pending = false;
  }
  return RBC_OK;
}
}  // namespace

namespace {

int gather_variant(const GatherLaunch& g) {
  if (g.elt != ELT_F32) return -1;
  const int vec = g.vec == 4 ? 4 : 1;
  for (int i = 0; i < kNumGathers; ++i) {
    const CombVariant& v = kGathers[i];
    if (v.out == (int)g.out && v.vec == vec && v.nl == g.nl && v.br == g.br && v.bc == g.bc && v.R == g.R)
      return i;
  }
  return -1;
}

int scatter_variant(const ScatterLaunch& s) {
  if (s.tp != ELT_F32 || s.ta != ELT_F32 || s.to != ELT_F32) return -1;
  const int vec = s.nl >= 2 ? (s.vec >= 2 ? 2 : 1) : (s.vec == 4 ? 4 : 1);
  for (int i = 0; i < kNumScatters; ++i) {
    const CombVariant& v = kScatters[i];
    if (v.vec == vec && v.nl == s.nl && v.br == s.br && v.bc == s.bc && v.R == s.R) return i;
  }
  return -1;
}

// Leaf variant and tile geometry: f32 runs 64 x 64 tiles with the stand-alone
// launch's K slab; f16s keeps the plan's tile; fp8c keeps it except 128,
// which runs as 64.
int leaf_variant(const LeafLaunch& l, int* tile) {
  int t = 0, bk = 32;
  if (l.prec == RBC_PREC_F32) {
    t = 64;
    bk = l.k % 32 == 0 ? 32 : 16;
  } else if (l.prec == RBC_PREC_F16S) {
    t = l.tile;
  } else if (l.prec == RBC_PREC_FP8C) {
    t = l.tile == 128 ? 64 : l.tile;
    bk = 64;
  } else {
    return -1;
  }
  for (int i = 0; i < kNumLeaves; ++i)
    if (kLeaves[i].prec == (int)l.prec && kLeaves[i].tile == t && kLeaves[i].bk == bk) {
      *tile = t;
      return i;
    }
  return -1;
}

rbc_status check_plan(const Plan& p) {
  if (p.prec != RBC_PREC_F32 && p.prec != RBC_PREC_F16S && p.prec != RBC_PREC_FP8C)
    return fail(RBC_EUNSUPPORTED, "batch: precision must be f32, f16s or fp8c");
  if (p.Q < 1) return fail(RBC_EUNSUPPORTED, "batch: plans need at least one level");
  for (const Group& g : p.groups) {
    const int nl = g.d1 - g.d0;
    const Scheme& s = p.levels[g.d0];
    bool ok = false;
    for (const CombVariant& v : kGathers)
      if (v.nl == nl && v.br == s.b1 && v.bc == s.b2 && v.R == s.R && s.b2 == s.b3 && s.b1 == s.b2) ok = true;
    if (!ok)
      return fail(RBC_EUNSUPPORTED, "batch: level shape <%d,%d,%d> R=%d x %d fused is not compiled", s.b1,
                  s.b2, s.b3, s.R, nl);
  }
  return RBC_OK;
}

// Everything one item contributes, before counters and ordering.
struct ItemTasks {
  std::vector<Task> list;  // in dependency (depth-first) order
  int32_t gate = -1;       // counter the entry tasks wait on (previous users of the region)
  int32_t done = -1;       // counter of finished top-level scatter pieces
  int32_t done_need = 0;
};

struct Builder {
  rbc_batch_s& b;
  int64_t target_bytes;

  int pieces_per_task(int64_t piece_bytes) const {
    const int64_t c = target_bytes / std::max<int64_t>(piece_bytes, 1);
    return (int)std::max<int64_t>(1, std::min<int64_t>(c, 1 << 20));
  }

  // Split pieces [0, n) of one unit into tasks.
  void split(std::vector<Task>& out, Task proto, int64_t first, int64_t n, int per) {
    for (int64_t f = first; f < first + n; f += per) {
      Task t = proto;
      t.first = f;
      t.count = (int32_t)std::min<int64_t>(per, first + n - f);
      out.push_back(t);
    }
  }

  rbc_status build_item(const Item& it, char* item_ws, int64_t cbase, ItemTasks& out) {
    Plan& p = *it.plan;
    std::vector<int32_t> s, pm;
    seeded_draws(p, it.seed, it.mode, s, pm);
    Draws dr;
    rbc_status st = check_draws(p, s.data(), pm.data(), dr);
    if (st != RBC_OK) return st;
    std::vector<ScaleLaunch> scA, scB;
    std::vector<GatherLaunch> gA, gB;
    build_gather(p, dr, 0, it.A, it.lda, item_ws, scA, gA);
    build_gather(p, dr, 1, it.B, it.ldb, item_ws, scB, gB);
    // the engine derives the exponents in its own tasks (max|X|, exponents) before the gathers
    for (GatherLaunch& l : gA) l.p.scale_partial = nullptr;
    for (GatherLaunch& l : gB) l.p.scale_partial = nullptr;
    const LeafLaunch lf = build_leaf(p, item_ws);
    std::vector<ScatterLaunch> sc;  // deepest group first
    build_scatter(p, dr, it.kappa_scale != 0, it.C, it.ldc, item_ws, sc, p.groups);
    const int ng = (int)p.groups.size();

    // counters of this item
    int64_t next = cbase;
    out.gate = (int32_t)next++;
    out.done = (int32_t)next++;
    int32_t cmax[2] = {-1, -1}, cexp[2] = {-1, -1}, cbits[2] = {-1, -1};
    const bool scaled = p.prec == RBC_PREC_F16S || p.prec == RBC_PREC_FP8C;
    if (scaled)
      for (int sd = 0; sd < 2; ++sd)
        cmax[sd] = (int32_t)next++, cexp[sd] = (int32_t)next++, cbits[sd] = (int32_t)next++;
    std::vector<int64_t> cg[2], cls;  // per group: first counter index
    for (int sd = 0; sd < 2; ++sd)
      for (int g = 0; g < ng; ++g) cg[sd].push_back(next), next += p.groups[g].n_in;
    for (int g = 0; g < ng; ++g) cls.push_back(next), next += p.groups[g].n_in;
    b.n_counters = next;

    // parameter blocks
    const int32_t gbase = (int32_t)b.gparams.size();
    int gvar[2][8], svar[8];
    int64_t gpieces[2][8], spieces[8];
    for (int sd = 0; sd < 2; ++sd) {
      const std::vector<GatherLaunch>& gl = sd == 0 ? gA : gB;
      for (int g = 0; g < ng; ++g) {
        gvar[sd][g] = gather_variant(gl[g]);
        if (gvar[sd][g] < 0) return fail(RBC_EUNSUPPORTED, "batch: gather variant not compiled");
        b.gparams.push_back(gl[g].p);
        const int vec = kGathers[gvar[sd][g]].vec;
        gpieces[sd][g] = (gl[g].p.rows_bot * gl[g].p.cols_bot / vec + 255) / 256;
      }
    }
    const int32_t sbase = (int32_t)b.sparams.size();
    for (int g = 0; g < ng; ++g) {
      const ScatterLaunch& l = sc[ng - 1 - g];  // sc is deepest first
      svar[g] = scatter_variant(l);
      if (svar[g] < 0) return fail(RBC_EUNSUPPORTED, "batch: scatter variant not compiled");
      b.sparams.push_back(l.p);
      spieces[g] = (l.p.rows_bot * l.p.cols_bot / kScatters[svar[g]].vec + 255) / 256;
    }
    int tile = 0;
    const int lvar = leaf_variant(lf, &tile);
    if (lvar < 0) return fail(RBC_EUNSUPPORTED, "batch: leaf variant not compiled");
    if (lf.m % tile || lf.n % tile || lf.k % kLeaves[lvar].bk)
      return fail(RBC_EINVAL, "batch: leaf dims %lld x %lld x %lld do not fit the tile", (long long)lf.m,
                  (long long)lf.n, (long long)lf.k);
    LeafDesc ld;
    std::memset(&ld, 0, sizeof ld);
    ld.S = lf.S, ld.T = lf.T, ld.P = static_cast<float*>(lf.P);
    ld.m = (int32_t)lf.m, ld.n = (int32_t)lf.n, ld.k = (int32_t)lf.k;
    ld.tiles_n = (int32_t)(lf.n / tile);
    ld.tiles_per_leaf = (int32_t)((lf.m / tile) * ld.tiles_n);
    ld.plane_s = lf.batch * lf.m * lf.k, ld.plane_t = lf.batch * lf.k * lf.n;
    ld.eS = lf.eS, ld.eT = lf.eT;
    const int32_t lidx = (int32_t)b.lparams.size();
    b.lparams.push_back(ld);

    std::vector<Task>& T = out.list;
    Task proto;
    std::memset(&proto, 0, sizeof proto);
    proto.wait[0] = proto.wait[1] = proto.signal = -1;

    // f16s, fp8c: max|A|, max|B|, then the per-leaf exponents
    int64_t max_pieces[2] = {0, 0};
    if (scaled) {
      for (int sd = 0; sd < 2; ++sd) {
        const ScaleLaunch& l = (sd == 0 ? scA : scB)[0];
        ScaleDesc d;
        d.X = l.X, d.ld = l.ld, d.rows = l.rows, d.cols = l.cols;
        d.maxbits = nullptr;  // the counter word cbits[sd], set once the layout is known
        b.cslots.push_back(cbits[sd]);
        d.G = l.G, d.e = l.e, d.n_leaves = l.n_leaves;
        d.pieces = l.rows;  // one piece per row
        d.target = l.target;
        d.level_rows = (int32_t)std::max<int64_t>(1, std::min<int64_t>(1 << 16, (64 << 10) / std::max<int64_t>(4 * d.cols, 1)));
        max_pieces[sd] = d.pieces;
        b.cparams.push_back(d);
      }
    }
    const int32_t cidx = (int32_t)b.cparams.size() - (scaled ? 2 : 0);
    if (scaled) {
      for (int sd = 0; sd < 2; ++sd) {
        Task t = proto;
        t.kind = TK_MAXABS, t.param = cidx + sd, t.signal = cmax[sd];
        t.wait[0] = out.gate, t.need[0] = 0;  // entry task; the need is set with the schedule
        const ScaleDesc& d = b.cparams[cidx + sd];
        split(T, t, 0, max_pieces[sd], pieces_per_task(d.cols * 4));
      }
      for (int sd = 0; sd < 2; ++sd) {
        Task t = proto;
        t.kind = TK_EXPONENTS, t.param = cidx + sd;
        t.wait[0] = cmax[sd], t.need[0] = (int32_t)max_pieces[sd];
        t.signal = cexp[sd], t.count = 1, t.first = 0;
        T.push_back(t);
      }
    }

    const int64_t R_last = p.groups[ng - 1].Rg;
    const int64_t tpl = ld.tiles_per_leaf;
    const int64_t leaf_piece_bytes =
        (int64_t)tile * tile * 4 + (int64_t)2 * tile * lf.k * (scaled ? 2 : 4);

    // depth-first emission
    struct Frame {
      int g;
      int64_t in;
    };
    std::vector<std::pair<Frame, bool>> stack;  // (frame, children done)
    stack.push_back({{0, 0}, false});
    while (!stack.empty()) {
      auto [fr, expanded] = stack.back();
      stack.pop_back();
      const int g = fr.g;
      const Group& G = p.groups[g];
      if (!expanded) {
        for (int sd = 0; sd < 2; ++sd) {
          Task t = proto;
          t.kind = TK_GATHER, t.variant = (int16_t)gvar[sd][g], t.param = gbase + sd * ng + g, t.sub = fr.in;
          if (g > 0) {
            t.wait[0] = (int32_t)(cg[sd][g - 1] + fr.in / p.groups[g - 1].Rg);
            t.need[0] = (int32_t)gpieces[sd][g - 1];
          } else {
            t.wait[0] = out.gate, t.need[0] = 0;  // entry task
          }
          if (g == ng - 1 && scaled) t.wait[1] = cexp[sd], t.need[1] = 1;
          t.signal = (int32_t)(cg[sd][g] + fr.in);
          const CombVariant& v = kGathers[gvar[sd][g]];
          const int64_t nsrc = ipow(v.br * v.bc, v.nl);
          const int out_bytes = (v.out == OUT_F16S || v.out == OUT_FP8X2) ? 2 : 4;
          split(T, t, 0, gpieces[sd][g], pieces_per_task(256 * v.vec * (nsrc * 4 + G.Rg * out_bytes)));
        }
        stack.push_back({fr, true});
        if (g == ng - 1) {
          Task t = proto;
          t.kind = TK_LEAF, t.variant = (int16_t)lvar, t.param = lidx;
          t.wait[0] = (int32_t)(cg[0][g] + fr.in), t.need[0] = (int32_t)gpieces[0][g];
          t.wait[1] = (int32_t)(cg[1][g] + fr.in), t.need[1] = (int32_t)gpieces[1][g];
          t.signal = (int32_t)(cls[g] + fr.in);
          split(T, t, fr.in * R_last * tpl, R_last * tpl, pieces_per_task(leaf_piece_bytes));
        } else {
          for (int64_t r = G.Rg; r-- > 0;) stack.push_back({{g + 1, fr.in * G.Rg + r}, false});
        }
      } else {
        Task t = proto;
        t.kind = TK_SCATTER, t.variant = (int16_t)svar[g], t.param = sbase + g, t.sub = fr.in;
        t.wait[0] = (int32_t)(cls[g] + fr.in);
        t.need[0] = (int32_t)(g == ng - 1 ? R_last * tpl : G.Rg * spieces[g + 1]);
        if (g > 0) t.signal = (int32_t)(cls[g - 1] + fr.in / p.groups[g - 1].Rg);
        else t.signal = out.done, out.done_need = (int32_t)spieces[0];
        const CombVariant& v = kScatters[svar[g]];
        const int64_t nout = ipow(v.br * v.bc, v.nl);
        split(T, t, 0, spieces[g], pieces_per_task(256 * v.vec * (G.Rg * 4 + nout * 4)));
      }
    }
    return RBC_OK;
  }
};

// Queue schedule: chunks of the items' task lists (or their gate tasks) in
// the order the queue holds them.
struct Chunk {
  size_t item;
  bool gates;
  size_t begin, end;
};

struct Schedule {
  std::vector<size_t> offs;               // item region offsets
  std::vector<std::vector<size_t>> deps;  // earlier items whose region an item reuses
  std::vector<Chunk> chunks;
  size_t region_bytes = 0;
};

// Interleave the items' task lists (a window of items, round robin in chunks,
// so that tasks of other items fill the waits of one item; the order inside
// an item is kept, so its dependencies still come first) and give every item
// a region of the item area.  With a budget the area is a ring: an item
// reuses the bytes of earlier items and waits for them to finish, and it
// enters the window only once every such item has all its tasks queued, so
// the waits point backwards in the queue.
rbc_status make_schedule(const rbc_batch_s& b, const std::vector<size_t>& order,
                         const std::vector<ItemTasks>& per, Schedule& sc) {
  const size_t n = b.items.size();
  sc.offs.assign(n, 0);
  sc.deps.assign(n, {});
  sc.chunks.clear();
  std::vector<size_t> size(n);
  size_t total = 0, biggest = 0;
  for (size_t i = 0; i < n; ++i) {
    size[i] = align_up(b.items[i].plan->ws_bytes);
    total += size[i];
    biggest = std::max(biggest, size[i]);
  }
  const size_t budget = b.opt.item_budget > 0 ? align_up((size_t)b.opt.item_budget) : 0;
  const bool ring = budget > 0 && budget < total;
  if (ring && biggest > budget)
    return fail(RBC_EINVAL, "batch: item budget %zu bytes < %zu needed by one product", budget, biggest);
  sc.region_bytes = ring ? budget : total;
  const int window = b.opt.window > 0 ? b.opt.window : 32;
  const size_t chunk = 32;
  struct Live {
    size_t item, lo, hi;
  };
  std::vector<Live> live;
  std::vector<char> is_active(n, 0);
  std::vector<size_t> pos(n, 0), active;
  size_t next = 0, cursor = 0;
  while (next < order.size() || !active.empty()) {
    while ((int)active.size() < window && next < order.size()) {
      const size_t j = order[next];
      size_t lo = cursor;
      if (ring && lo + size[j] > budget) lo = 0;
      const size_t hi = lo + size[j];
      bool blocked = false;
      std::vector<size_t> deps;
      for (const Live& l : live)
        if (l.lo < hi && lo < l.hi) {
          if (is_active[l.item]) blocked = true;
          deps.push_back(l.item);
        }
      if (blocked) break;
      // The new region supersedes the overlapped bytes; what is left of an
      // overlapped region stays live for its item.
      std::vector<Live> kept;
      for (const Live& l : live) {
        if (!(l.lo < hi && lo < l.hi)) {
          kept.push_back(l);
          continue;
        }
        if (l.lo < lo) kept.push_back({l.item, l.lo, lo});
        if (hi < l.hi) kept.push_back({l.item, hi, l.hi});
      }
      kept.push_back({j, lo, hi});
      live.swap(kept);
      sc.offs[j] = lo;
      sc.deps[j] = deps;
      cursor = hi;
      is_active[j] = 1;
      active.push_back(j);
      ++next;
      if (!deps.empty()) sc.chunks.push_back({j, true, 0, deps.size()});
    }
    for (size_t a = 0; a < active.size();) {
      const size_t i = active[a];
      const size_t end = std::min(per[i].list.size(), pos[i] + chunk);
      sc.chunks.push_back({i, false, pos[i], end});
      pos[i] = end;
      if (pos[i] == per[i].list.size()) {
        is_active[i] = 0;
        active.erase(active.begin() + a);
      } else {
        ++a;
      }
    }
  }
  return RBC_OK;
}

// Task construction with item regions at items_base + offs (items_base
// nullptr: only the counts and sizes are meaningful).
rbc_status build_items(rbc_batch_s& b, char* items_base, const std::vector<size_t>& offs,
                       const std::vector<size_t>& order, std::vector<ItemTasks>& per) {
  b.gparams.clear(), b.sparams.clear(), b.lparams.clear(), b.cparams.clear();
  b.cslots.clear();
  b.n_counters = 0;
  Builder bl{b, b.opt.task_bytes > 0 ? b.opt.task_bytes : (int64_t)4 << 20};
  per.assign(b.items.size(), ItemTasks{});
  for (size_t i : order) {
    char* base = items_base ? items_base + offs[i] : nullptr;
    rbc_status st = bl.build_item(b.items[i], base, b.n_counters, per[i]);
    if (st != RBC_OK) return st;
  }
  return RBC_OK;
}

void assemble(rbc_batch_s& b, std::vector<ItemTasks>& per, const Schedule& sc) {
  b.tasks.clear(), b.task_item.clear();
  b.item_gate.assign(per.size(), -1), b.item_done.assign(per.size(), -1), b.item_first.assign(per.size(), -1);
  for (size_t j = 0; j < per.size(); ++j) b.item_gate[j] = per[j].gate, b.item_done[j] = per[j].done;
  for (size_t j = 0; j < per.size(); ++j) {  // entry tasks wait for the previous users of the region
    const int32_t nd = (int32_t)sc.deps[j].size();
    for (Task& t : per[j].list)
      if (t.wait[0] == per[j].gate) {
        if (nd) t.need[0] = nd;
        else t.wait[0] = -1, t.need[0] = 0;
      }
  }
  for (const Chunk& c : sc.chunks) {
    if (b.item_first[c.item] < 0) b.item_first[c.item] = (int64_t)b.tasks.size();
    if (c.gates) {
      for (size_t d : sc.deps[c.item]) {
        Task t;
        std::memset(&t, 0, sizeof t);
        t.kind = TK_GATE;
        t.wait[0] = per[d].done, t.need[0] = per[d].done_need;
        t.wait[1] = -1, t.signal = per[c.item].gate, t.count = 1;
        b.tasks.push_back(t);
        b.task_item.push_back((int32_t)c.item);
      }
    } else {
      b.tasks.insert(b.tasks.end(), per[c.item].list.begin() + c.begin, per[c.item].list.begin() + c.end);
      b.task_item.insert(b.task_item.end(), c.end - c.begin, (int32_t)c.item);
    }
  }
}

// Depth of every task in the dependency graph: 0 for a task without waits,
// else one more than the deepest task that signals a counter it waits on
// (signals precede waits in the queue).  Returns the largest depth.
int32_t task_depths(const rbc_batch_s& b, std::vector<int32_t>& level) {
  const size_t n = b.tasks.size();
  std::vector<int32_t> clevel((size_t)b.n_counters, -1);
  level.assign(n, 0);
  int32_t top = 0;
  for (size_t t = 0; t < n; ++t) {
    const Task& k = b.tasks[t];
    int32_t lv = 0;
    for (int i = 0; i < 2; ++i)
      if (k.wait[i] >= 0) lv = std::max(lv, clevel[(size_t)k.wait[i]] + 1);
    level[t] = lv;
    top = std::max(top, lv);
    if (k.signal >= 0) clevel[(size_t)k.signal] = std::max(clevel[(size_t)k.signal], lv);
  }
  return top;
}

// RBC_ORDER_DEPTH: the persistent kernel's queue sorted by dependency depth
// (stable: queue order within a depth).  Every wait still points backwards.
void order_by_depth(rbc_batch_s& b) {
  std::vector<int32_t> level;
  task_depths(b, level);
  const size_t n = b.tasks.size();
  std::vector<int32_t> order(n);
  for (size_t t = 0; t < n; ++t) order[t] = (int32_t)t;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return level[(size_t)x] < level[(size_t)y]; });
  std::vector<Task> tasks(n);
  std::vector<int32_t> items(n);
  for (size_t i = 0; i < n; ++i) tasks[i] = b.tasks[(size_t)order[i]], items[i] = b.task_item[(size_t)order[i]];
  b.tasks.swap(tasks), b.task_item.swap(items);
  b.item_first.assign(b.item_first.size(), -1);
  for (size_t i = 0; i < n; ++i)
    if (b.item_first[(size_t)b.task_item[i]] < 0) b.item_first[(size_t)b.task_item[i]] = (int64_t)i;
}

// RBC_BATCH_LEVELS: one launch per (dependency depth, kind, variant) listing
// every piece of its tasks.
void make_levels(rbc_batch_s& b) {
  const size_t n = b.tasks.size();
  std::vector<int32_t> level;
  const int32_t top = task_depths(b, level);
  std::vector<int32_t> order(n);
  for (size_t t = 0; t < n; ++t) order[t] = (int32_t)t;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    const Task &a = b.tasks[(size_t)x], &c = b.tasks[(size_t)y];
    if (level[(size_t)x] != level[(size_t)y]) return level[(size_t)x] < level[(size_t)y];
    if (a.kind != c.kind) return a.kind < c.kind;
    return a.variant < c.variant;
  });
  b.launches.clear(), b.piece_table.clear();
  for (int32_t t : order) {
    const Task& k = b.tasks[(size_t)t];
    if (k.kind == TK_GATE) continue;  // ordering only
    if (b.launches.empty() || b.launches.back().level != level[(size_t)t] || b.launches.back().kind != k.kind ||
        b.launches.back().variant != k.variant)
      b.launches.push_back({level[(size_t)t], k.kind, k.variant, (int64_t)b.piece_table.size() / 2, 0});
    // max|X| pieces cover level_rows rows each; every other piece is one workgroup's unit
    const int32_t step = k.kind == TK_MAXABS ? b.cparams[(size_t)k.param].level_rows : 1;
    int64_t np = 0;
    for (int32_t c = 0; c < k.count; c += step, ++np) {
      b.piece_table.push_back(t);
      b.piece_table.push_back((int32_t)(k.first + c));
    }
    b.launches.back().n += np;
  }
  b.n_levels = n ? top + 1 : 0;
}

// Build tasks, parameter blocks and the workspace layout for workspace base
// `ws` (nullptr: sizes only).
rbc_status build(rbc_batch_s& b, char* ws) {
  // Items largest first so that the end of the queue holds short chains.
  std::vector<size_t> order(b.items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
    return b.items[x].plan->ws_bytes > b.items[y].plan->ws_bytes;
  });
  std::vector<ItemTasks> per;
  Schedule sc;
  std::vector<size_t> zero(b.items.size(), 0);
  rbc_status st = build_items(b, nullptr, zero, order, per);
  if (st != RBC_OK) return st;
  if ((st = make_schedule(b, order, per, sc)) != RBC_OK) return st;
  assemble(b, per, sc);
  if (b.tasks.size() > 0x7fffffff) return fail(RBC_EINVAL, "batch: too many tasks");
  const bool levels = b.opt.mode == RBC_BATCH_LEVELS;
  const bool by_depth = !levels && b.opt.order == RBC_ORDER_DEPTH;
  if (levels) make_levels(b);
  if (by_depth) order_by_depth(b);
  Layout& L = b.lay;
  L.tasks = 0;
  L.gather = align_up(L.tasks + b.tasks.size() * sizeof(Task));
  L.scatter = align_up(L.gather + b.gparams.size() * sizeof(GatherParams));
  L.leaf = align_up(L.scatter + b.sparams.size() * sizeof(ScatterParams));
  L.scale = align_up(L.leaf + b.lparams.size() * sizeof(LeafDesc));
  L.ctl = align_up(L.scale + b.cparams.size() * sizeof(ScaleDesc));
  L.trace = align_up(L.ctl + (CTL_WORDS + b.n_counters) * sizeof(int32_t));
  L.pieces = align_up(L.trace + (b.opt.trace && !levels ? b.tasks.size() * 4 * sizeof(uint64_t) : 0));
  L.items = align_up(L.pieces + (levels ? b.piece_table.size() * sizeof(int32_t) : 0));
  L.total = L.items + sc.region_bytes;
  L.item_ws = sc.offs;
  b.ws = ws;
  if (!ws) return RBC_OK;
  if ((st = build_items(b, ws + L.items, sc.offs, order, per)) != RBC_OK) return st;
  assemble(b, per, sc);
  if (levels) make_levels(b);
  if (by_depth) order_by_depth(b);
  int32_t* words = reinterpret_cast<int32_t*>(ws + L.ctl) + CTL_WORDS;
  for (size_t i = 0; i < b.cparams.size(); ++i) b.cparams[i].maxbits = reinterpret_cast<uint32_t*>(words + b.cslots[i]);
  return RBC_OK;
}

}  // namespace

extern "C" {

rbc_status rbc_batch_create(const rbc_batch_options* opt, rbc_batch* out) {
  try {
    if (!out) return fail(RBC_EINVAL, "null output handle");
    *out = nullptr;
    rbc_batch_s* b = new rbc_batch_s;
    std::memset(&b->opt, 0, sizeof b->opt);
    if (opt) b->opt = *opt;
    if (b->opt.timeout_ms <= 0) b->opt.timeout_ms = 5000;
    if (b->opt.mode != RBC_BATCH_PERSISTENT && b->opt.mode != RBC_BATCH_LEVELS) {
      const int mode = b->opt.mode;
      delete b;
      return fail(RBC_EINVAL, "bad batch mode %d", mode);
    }
    if (b->opt.order != RBC_ORDER_PRODUCTS && b->opt.order != RBC_ORDER_DEPTH) {
      const int order = b->opt.order;
      delete b;
      return fail(RBC_EINVAL, "bad batch order %d", order);
    }
    *out = b;
    return RBC_OK;
  } catch (const std::bad_alloc&) {
    return fail(RBC_ENOMEM, "host allocation failed");
  }
}

rbc_status rbc_batch_add(rbc_batch b, rbc_plan plan, const void* A, int64_t lda, const void* B,
                         int64_t ldb, void* C, int64_t ldc, uint64_t seed, rbc_mode mode, int kappa_scale,
                         int64_t* index) {
  try {
    if (!b || !plan) return fail(RBC_EINVAL, "null batch or plan");
    rbc_status ws = wait_upload(*b);
    if (ws != RBC_OK) return ws;
    Plan& p = plan->p;
    if (!A || !B || !C) return fail(RBC_EINVAL, "null matrix pointer");
    if (lda < p.K || ldb < p.N || ldc < p.N) return fail(RBC_EINVAL, "leading dimension too small");
    if (mode < RBC_MODE_FULL || mode > RBC_MODE_NONE) return fail(RBC_EINVAL, "bad mode %d", (int)mode);
    rbc_status st = check_plan(p);
    if (st != RBC_OK) return st;
    if (b->prec >= 0 && b->prec != (int)p.prec)
      return fail(RBC_EINVAL, "batch: every item must use the same precision");
    b->prec = (int)p.prec;
    b->items.push_back(Item{&p, A, lda, B, ldb, C, ldc, seed, mode, kappa_scale});
    b->prepared = false;
    if (index) *index = (int64_t)b->items.size() - 1;
    return RBC_OK;
  } catch (const std::bad_alloc&) {
    return fail(RBC_ENOMEM, "host allocation failed");
  }
}

rbc_status rbc_batch_workspace(rbc_batch b, size_t* bytes) {
  try {
    if (!b || !bytes) return fail(RBC_EINVAL, "null argument");
    rbc_status st = wait_upload(*b);
    if (st != RBC_OK) return st;
    st = build(*b, nullptr);
    if (st != RBC_OK) return st;
    *bytes = b->lay.total;
    return RBC_OK;
  } catch (const std::bad_alloc&) {
    return fail(RBC_ENOMEM, "host allocation failed");
  }
}

rbc_status rbc_batch_prepare(rbc_batch b, void* workspace, size_t ws_bytes, void* stream) {
  try {
    if (!b) return fail(RBC_EINVAL, "null batch");
    if (b->items.empty()) return fail(RBC_EINVAL, "empty batch");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign)
      return fail(RBC_EINVAL, "workspace must be non-null and 256-byte aligned");
    rbc_status st = wait_upload(*b);
    if (st != RBC_OK) return st;
    for (Item& it : b->items) {
      st = ensure_device(*it.plan);
      if (st != RBC_OK) return st;
    }
    st = build(*b, static_cast<char*>(workspace));
    if (st != RBC_OK) return st;
    if (ws_bytes < b->lay.total)
      return fail(RBC_EINVAL, "workspace of %zu bytes < %zu needed", ws_bytes, b->lay.total);
    HIP_CHECK(hipGetDevice(&b->device));
    int bpc = 0, cus = 0, rate_khz = 0;
    HIP_CHECK(batch_occupancy(b->prec, &bpc));
    HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
    HIP_CHECK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, b->device));
    if (bpc < 1) return fail(RBC_EHIP, "batch kernel cannot be resident");
    b->grid = b->opt.grid > 0 ? std::min(b->opt.grid, bpc * cus) : bpc * cus;
    b->timeout_ticks = (int64_t)b->opt.timeout_ms * (rate_khz > 0 ? rate_khz : 100000);
    hipStream_t s = (hipStream_t)stream;
    char* ws = static_cast<char*>(workspace);
    const Layout& L = b->lay;
    HIP_CHECK(hipMemcpyAsync(ws + L.tasks, b->tasks.data(), b->tasks.size() * sizeof(Task),
                             hipMemcpyHostToDevice, s));
    if (!b->gparams.empty())
      HIP_CHECK(hipMemcpyAsync(ws + L.gather, b->gparams.data(), b->gparams.size() * sizeof(GatherParams),
                               hipMemcpyHostToDevice, s));
    if (!b->sparams.empty())
      HIP_CHECK(hipMemcpyAsync(ws + L.scatter, b->sparams.data(), b->sparams.size() * sizeof(ScatterParams),
                               hipMemcpyHostToDevice, s));
    if (!b->lparams.empty())
      HIP_CHECK(hipMemcpyAsync(ws + L.leaf, b->lparams.data(), b->lparams.size() * sizeof(LeafDesc),
                               hipMemcpyHostToDevice, s));
    if (!b->cparams.empty())
      HIP_CHECK(hipMemcpyAsync(ws + L.scale, b->cparams.data(), b->cparams.size() * sizeof(ScaleDesc),
                               hipMemcpyHostToDevice, s));
    if (b->opt.mode == RBC_BATCH_LEVELS && !b->piece_table.empty())
      HIP_CHECK(hipMemcpyAsync(ws + L.pieces, b->piece_table.data(), b->piece_table.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, s));
    // the host vectors stay unchanged in the batch until the copies are done
    if (!b->uploaded) HIP_CHECK(hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming));
    HIP_CHECK(hipEventRecord(b->uploaded, s));
    b->upload_pending = true;
    if (b->exec) (void)hipGraphExecDestroy(b->exec), b->exec = nullptr;
    if (b->graph) (void)hipGraphDestroy(b->graph), b->graph = nullptr;
    b->prepared = true;
    return RBC_OK;
  } catch (const std::bad_alloc&) {
    return fail(RBC_ENOMEM, "host allocation failed");
  }
}

}  // extern "C"

namespace {

rbc_status enqueue(rbc_batch_s& b, hipStream_t s) {
  KernelArgs a;
  const Layout& L = b.lay;
  if (b.opt.mode == RBC_BATCH_LEVELS) {
    HIP_CHECK(launch_zero_words(reinterpret_cast<int32_t*>(b.ws + L.ctl), CTL_WORDS + b.n_counters, s));
    const Task* tasks = reinterpret_cast<const Task*>(b.ws + L.tasks);
    const int32_t* pieces = reinterpret_cast<const int32_t*>(b.ws + L.pieces);
    for (const auto& g : b.launches)
      HIP_CHECK(launch_group(b.prec, g.kind, g.variant, tasks, pieces + 2 * g.begin,
                             reinterpret_cast<const GatherParams*>(b.ws + L.gather),
                             reinterpret_cast<const ScatterParams*>(b.ws + L.scatter),
                             reinterpret_cast<const LeafDesc*>(b.ws + L.leaf),
                             reinterpret_cast<const ScaleDesc*>(b.ws + L.scale), g.n, s));
    return RBC_OK;
  }
  a.tasks = reinterpret_cast<const Task*>(b.ws + L.tasks);
  a.n_tasks = (int64_t)b.tasks.size();
  a.gather = reinterpret_cast<const GatherParams*>(b.ws + L.gather);
  a.scatter = reinterpret_cast<const ScatterParams*>(b.ws + L.scatter);
  a.leaf = reinterpret_cast<const LeafDesc*>(b.ws + L.leaf);
  a.scale = reinterpret_cast<const ScaleDesc*>(b.ws + L.scale);
  a.ctl = reinterpret_cast<int32_t*>(b.ws + L.ctl);
  a.n_ctl = CTL_WORDS + b.n_counters;
  a.timeout_ticks = b.timeout_ticks;
  a.trace = b.opt.trace ? reinterpret_cast<uint64_t*>(b.ws + L.trace) : nullptr;
  HIP_CHECK(launch_batch(b.prec, a, b.grid, s));
  return RBC_OK;
}

}  // namespace

extern "C" {

rbc_status rbc_batch_launch(rbc_batch b, void* stream, int use_graph) {
  try {
    if (!b) return fail(RBC_EINVAL, "null batch");
    if (!b->prepared) return fail(RBC_EINVAL, "batch not prepared");
    hipStream_t s = (hipStream_t)stream;
    int dev = -1;
    HIP_CHECK(hipGetDevice(&dev));
    if (dev != b->device) return fail(RBC_EINVAL, "batch prepared on device %d, current %d", b->device, dev);
    if (!use_graph) return enqueue(*b, s);
    if (!s) return fail(RBC_EINVAL, "graph capture needs a non-default stream");
    if (!b->exec || b->graph_stream != s) {
      if (b->exec) (void)hipGraphExecDestroy(b->exec), b->exec = nullptr;
      if (b->graph) (void)hipGraphDestroy(b->graph), b->graph = nullptr;
      HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      rbc_status st = enqueue(*b, s);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(s, &g);
      if (st != RBC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return fail(RBC_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
      b->graph = g;
      HIP_CHECK(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
      b->graph_stream = s;
    }
    HIP_CHECK(hipGraphLaunch(b->exec, s));
    return RBC_OK;
  } catch (const std::bad_alloc&) {
    return fail(RBC_ENOMEM, "host allocation failed");
  }
}

rbc_status rbc_batch_check(rbc_batch b, void* stream) {
  if (!b) return fail(RBC_EINVAL, "null batch");
  if (!b->prepared) return fail(RBC_EINVAL, "batch not prepared");
  HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
  int32_t ctl[CTL_WORDS];
  HIP_CHECK(hipMemcpy(ctl, b->ws + b->lay.ctl, sizeof ctl, hipMemcpyDeviceToHost));
  if (ctl[CTL_ABORT])
    return fail(RBC_EHIP, "batch: a dependency wait exceeded %d ms (task %d); results are incomplete",
                b->opt.timeout_ms, ctl[CTL_STUCK_TASK] - 1);
  return RBC_OK;
}

rbc_status rbc_batch_get_info(rbc_batch b, rbc_batch_info* info) {
  if (!b || !info) return fail(RBC_EINVAL, "null argument");
  std::memset(info, 0, sizeof *info);
  info->n_items = (int64_t)b->items.size();
  info->n_tasks = (int64_t)b->tasks.size();
  info->n_counters = b->n_counters;
  info->grid = b->grid;
  info->prec = b->prec;
  info->workspace_bytes = b->lay.total;
  info->levels = b->n_levels;
  info->launches = (int64_t)b->launches.size();
  info->control_bytes = b->lay.items;
  for (const Task& t : b->tasks) {
    if (t.kind == TK_GATHER) info->gather_tasks++;
    else if (t.kind == TK_LEAF) info->leaf_tasks++;
    else if (t.kind == TK_SCATTER) info->scatter_tasks++;
    else if (t.kind == TK_GATE) info->gate_tasks++;
    else info->scale_tasks++;
  }
  return RBC_OK;
}

rbc_status rbc_batch_task_table(rbc_batch b, rbc_batch_task* out, int64_t cap, int64_t* n) {
  static_assert(sizeof(rbc_batch_task) == sizeof(Task), "task record layout");
  if (!b || !n) return fail(RBC_EINVAL, "null argument");
  if (cap < 0 || (cap > 0 && !out)) return fail(RBC_EINVAL, "bad output buffer");
  *n = (int64_t)b->tasks.size();
  const int64_t k = std::min<int64_t>(cap, *n);
  if (k > 0) std::memcpy(out, b->tasks.data(), (size_t)k * sizeof(Task));
  return RBC_OK;
}

rbc_status rbc_batch_trace(rbc_batch b, uint64_t* out, int64_t cap, int64_t* n, double* ticks_per_us) {
  if (!b || !n) return fail(RBC_EINVAL, "null argument");
  if (!b->opt.trace || !b->prepared || b->opt.mode != RBC_BATCH_PERSISTENT)
    return fail(RBC_EINVAL, "batch has no trace (persistent mode, options.trace, then prepare)");
  *n = (int64_t)b->tasks.size();
  if (ticks_per_us) {
    int rate_khz = 0;
    HIP_CHECK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, b->device));
    *ticks_per_us = rate_khz / 1000.0;
  }
  if (cap < 0 || (cap > 0 && !out)) return fail(RBC_EINVAL, "bad output buffer");
  const int64_t k = std::min<int64_t>(cap, *n);
  if (k > 0) HIP_CHECK(hipMemcpy(out, b->ws + b->lay.trace, (size_t)k * 4 * sizeof(uint64_t), hipMemcpyDeviceToHost));
  return RBC_OK;
}

rbc_status rbc_batch_get_item(rbc_batch b, int64_t index, rbc_batch_item* out) {
  if (!b || !out) return fail(RBC_EINVAL, "null argument");
  if (index < 0 || index >= (int64_t)b->items.size()) return fail(RBC_EINVAL, "item %lld out of range", (long long)index);
  if ((size_t)index >= b->item_first.size()) return fail(RBC_EINVAL, "batch not built: query the workspace first");
  out->region_offset = b->lay.items + b->lay.item_ws[index];
  out->region_bytes = align_up(b->items[index].plan->ws_bytes);
  out->first_task = b->item_first[index];
  out->gate_counter = b->item_gate[index];
  out->done_counter = b->item_done[index];
  return RBC_OK;
}

rbc_status rbc_batch_set_grid(rbc_batch b, int grid) {
  if (!b) return fail(RBC_EINVAL, "null batch");
  if (grid < 0) return fail(RBC_EINVAL, "grid must be >= 0");
  b->opt.grid = grid;
  if (b->prepared) {
    int bpc = 0, cus = 0;
    HIP_CHECK(batch_occupancy(b->prec, &bpc));
    HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
    b->grid = grid > 0 ? std::min(grid, bpc * cus) : bpc * cus;
    if (b->exec) (void)hipGraphExecDestroy(b->exec), b->exec = nullptr;
    if (b->graph) (void)hipGraphDestroy(b->graph), b->graph = nullptr;
  }
  return RBC_OK;
}

void rbc_batch_destroy(rbc_batch b) {
  if (!b) return;
  (void)wait_upload(*b);
  if (b->uploaded) (void)hipEventDestroy(b->uploaded);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  delete b;
}

}  // extern "C"
