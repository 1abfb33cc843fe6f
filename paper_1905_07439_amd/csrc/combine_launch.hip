// Element-type dispatch of the fused block-combination kernels (combine.hpp);
// each type combination is instantiated in its own translation unit.
#include "combine.hpp"

namespace rbc {
namespace comb {
RBC_GATHER_COMBOS(RBC_DECL_G)
RBC_SCATTER_COMBOS(RBC_DECL_S)
}  // namespace comb

namespace {

hipError_t gather_pair(Elt elt, GatherOut out, int vec, int nl, int br, int bc, int R, const GatherPair& p,
                       hipStream_t s) {
  if (elt == ELT_F64 && out == OUT_SAME) return comb::gather_dispatch<double, OUT_SAME>(vec, nl, br, bc, R, p, s);
  if (elt == ELT_F32 && out == OUT_SAME) return comb::gather_dispatch<float, OUT_SAME>(vec, nl, br, bc, R, p, s);
  if (elt == ELT_F32 && out == OUT_BF16X2)
    return comb::gather_dispatch<float, OUT_BF16X2>(vec, nl, br, bc, R, p, s);
  if (elt == ELT_F32 && out == OUT_F16S)
    return comb::gather_dispatch<float, OUT_F16S>(vec, nl, br, bc, R, p, s);
  if (elt == ELT_F32 && out == OUT_FP8X2)
    return comb::gather_dispatch<float, OUT_FP8X2>(vec, nl, br, bc, R, p, s);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_gather(Elt elt, GatherOut out, int vec, int nl, int br, int bc, int R,
                         const GatherParams& p, hipStream_t s) {
  if (p.rows_bot * p.cols_bot == 0 || p.n_in == 0) return hipSuccess;
  GatherPair pp;
  pp.a = p, pp.b = p, pp.sides = 1;
  return gather_pair(elt, out, vec, nl, br, bc, R, pp, s);
}

hipError_t launch_gather2(Elt elt, GatherOut out, int vec, int nl, int br, int bc, int R,
                          const GatherParams& pa, const GatherParams& pb, hipStream_t s) {
  const bool ea = pa.rows_bot * pa.cols_bot == 0 || pa.n_in == 0;
  const bool eb = pb.rows_bot * pb.cols_bot == 0 || pb.n_in == 0;
  if (ea || eb) {  // an empty side: the other alone
    if (!ea) return launch_gather(elt, out, vec, nl, br, bc, R, pa, s);
    if (!eb) return launch_gather(elt, out, vec, nl, br, bc, R, pb, s);
    return hipSuccess;
  }
  GatherPair pp;
  pp.a = pa, pp.b = pb, pp.sides = 2;
  return gather_pair(elt, out, vec, nl, br, bc, R, pp, s);
}

hipError_t launch_scatter(Elt tp, Elt ta, Elt to, int vec, int nl, int br, int bc, int R,
                          const ScatterParams& p, hipStream_t s) {
  if (p.rows_bot * p.cols_bot == 0 || p.n_out == 0) return hipSuccess;
  if (tp == ELT_F64 && ta == ELT_F64 && to == ELT_F64)
    return comb::scatter_dispatch<double, double, double>(vec, nl, br, bc, R, p, s);
  if (tp == ELT_F32 && ta == ELT_F32 && to == ELT_F32)
    return comb::scatter_dispatch<float, float, float>(vec, nl, br, bc, R, p, s);
  if (tp == ELT_F32 && ta == ELT_F64 && to == ELT_F64)
    return comb::scatter_dispatch<float, double, double>(vec, nl, br, bc, R, p, s);
  if (tp == ELT_F32 && ta == ELT_F64 && to == ELT_F32)
    return comb::scatter_dispatch<float, double, float>(vec, nl, br, bc, R, p, s);
  if (tp == ELT_F64 && ta == ELT_F64 && to == ELT_F32)
    return comb::scatter_dispatch<double, double, float>(vec, nl, br, bc, R, p, s);
  return hipErrorInvalidValue;
}

}  // namespace rbc
