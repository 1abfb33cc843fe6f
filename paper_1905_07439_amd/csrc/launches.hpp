// Host-side construction of the kernel launches of one product: the same
// descriptions drive the per-stage launches (api.cpp) and the batch engine's
// task table (batch.cpp).
#pragma once

#include <vector>

#include "core.hpp"
#include "kernels.hpp"

namespace rbc {

// Per-level draws, concatenated as in include/rbc.h.
struct Draws {
  std::vector<int32_t> s, pm;
  std::vector<size_t> off;
};

rbc_status check_draws(const Plan& p, const int32_t* signs, const int32_t* perms, Draws& d);
void seeded_draws(const Plan& p, uint64_t seed, rbc_mode mode, std::vector<int32_t>& s,
                  std::vector<int32_t>& pm);
rbc_status check_ws(const Plan& p, void* ws, size_t bytes);
// Upload the coefficient tables of every level on first use on a device.
rbc_status ensure_device(Plan& p);
// One product with the plan's draws given (validated, per level), the workspace
// supplied by the caller: the body of rbc_matmul and rbc_matmul_draws.
rbc_status matmul_impl(Plan& p, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                       int64_t ldc, const int32_t* signs, const int32_t* perms, int kappa_scale,
                       void* ws, size_t ws_bytes, void* stream);

struct ScaleLaunch {  // f16s, fp8c: partial maxima of |X| (launch), per-leaf exponent inputs
  const float* X;
  int64_t ld, rows, cols;
  float* partial;  // kScalePartials partial maxima
  const float* G;
  int32_t* e;
  int64_t n_leaves;
  float target;  // bound of the scaled operand: 2^15 (f16), 448 (e4m3)
};

struct GatherLaunch {
  GatherParams p;
  Elt elt;
  GatherOut out;
  int vec, nl, br, bc, R;
};

struct LeafLaunch {
  rbc_prec prec;
  const void* S;
  const void* T;
  void* P;
  int64_t m, n, k, batch;
  int tile;
  bool masked;  // leaves of any size (exact-block plans)
  const int32_t* eS;
  const int32_t* eT;
};

struct LeafGatherLaunch {  // f32 leaf products with the deepest level gathered in the loads
  LeafGather g;
  float* P;
  int64_t m, n, k, batch;
  int tile;
  bool scatter;              // and the deepest level's scatter after each tile (ls)
  LeafScatter ls;
};

struct ScatterLaunch {
  ScatterParams p;
  Elt tp, ta, to;
  int vec, nl, br, bc, R;
};

// which = 0: A (M x K), 1: B (K x N).  `scale` is filled for f16s and fp8c plans.
// leaf_gather: the gathers of levels [0, Q - 1) only (Plan::fgroups), whose
// output build_leaf_gather's launch reads.
void build_gather(const Plan& p, const Draws& dr, int which, const void* X, int64_t ldx, char* ws,
                  std::vector<ScaleLaunch>& scale, std::vector<GatherLaunch>& out, bool leaf_gather = false);
LeafLaunch build_leaf(const Plan& p, char* ws);
// Requires p.leaf_gather_ok; leaf_scatter (requires p.leaf_scatter_ok): the
// launch also writes the parents' product blocks (kappa_scale as for the scatter).
LeafGatherLaunch build_leaf_gather(const Plan& p, const Draws& dr, char* ws, bool leaf_scatter = false,
                                   bool kappa_scale = false);
// In execution order (deepest group first), over `groups`: Plan::groups (the
// batch engine), Plan::sgroups (rbc_matmul, the stage calls) or, with
// from_parents (leaf scatter), Plan::fgroups: the passes of levels [0, Q - 1)
// from the parents' product blocks.
void build_scatter(const Plan& p, const Draws& dr, bool kappa_scale, void* C, int64_t ldc, char* ws,
                   std::vector<ScatterLaunch>& out, const std::vector<Group>& groups, bool from_parents = false);

hipError_t launch(const ScaleLaunch& l, hipStream_t s);
hipError_t launch(const ScaleLaunch& a, const ScaleLaunch& b, hipStream_t s);  // both in one launch
hipError_t launch(const GatherLaunch& l, hipStream_t s);
// Two gathers in one launch when they share element type, output and shape
// (else one after the other); the same results either way.
hipError_t launch(const GatherLaunch& a, const GatherLaunch& b, hipStream_t s);
hipError_t launch(const LeafLaunch& l, hipStream_t s);
hipError_t launch(const LeafGatherLaunch& l, hipStream_t s);
hipError_t launch(const ScatterLaunch& l, hipStream_t s);

}  // namespace rbc
