// Fused block-combination kernels: the gather (forming S_r = sum u-hat A_kl and
// T_r = sum v-hat B_k'l') and the scatter (C_ij = sum_r w-hat P_r) of
// eq. recursive-random-formula, several levels per pass.
//
// One thread owns one element position (y, x) of the bottom block and walks
// the group's levels depth first in registers: it loads the prod(b_row b_col)
// values of the top block that map onto (y, x), forms every level's sums in
// the fixed order of the folded formula (eq. randomized-algorithm), and
// writes the prod R bottom values (gather), or loads the prod R products and
// accumulates upwards (scatter).  Every load and store of a wavefront is
// contiguous along x, each top element is read once and each bottom element
// written once, so the kernels move the algorithmic minimum of bytes.
//
// Summation order (the fl model of Section 2.2, sequential sums): S_r over
// (k, l) in row-major order and C_ij over ascending r, skipping zero
// coefficients; the first term is fl(c * x), then acc = fl(acc + fl(c * x)).
// Contraction into fused multiply-adds is disabled (pragma below, and
// -ffp-contract=off for every translation unit that instantiates these).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "devptr.hpp"
#include "scale.hpp"
#include "kernels.hpp"
#include "occupancy.hpp"

#pragma clang fp contract(off)

#ifndef RBC_NT_LOADS
#define RBC_NT_LOADS 1
#endif
#ifndef RBC_LEVEL_BARRIER
#define RBC_LEVEL_BARRIER 0
#endif


namespace rbc {
namespace comb {

__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// Folded coefficient of block (k, l) in product r: table entry at the permuted
// block times the two signs (eq. randomized-algorithm).  With UNIFORM (the
// same value for every lane) the index is made uniform and the read-only
// table is read through the constant address space, so the coefficient
// arrives by a scalar load instead of a waited vector load: the Strassen
// scatters' looped level went from 130 to 118 us (N = 4096, Q = 3, f32).
template <typename T, int BC, bool UNIFORM = false>
__device__ __forceinline__ T coef(const SideLevel& L, int k, int l, int r, int R) {
  if constexpr (UNIFORM) {
    typedef __attribute__((address_space(4))) const T ctab_t;
    const uint64_t a = reinterpret_cast<uintptr_t>(L.tab);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const ctab_t* tab = (const ctab_t*)(((uint64_t)hi << 32) | lo);
    const int idx = __builtin_amdgcn_readfirstlane((L.pr[k] * BC + L.pc[l]) * R + r);
    const int sg = __builtin_amdgcn_readfirstlane(L.sr[k] * L.sc[l]);
    const T c = tab[idx];
    return sg < 0 ? -c : c;
  } else {
    const gbl<const T>* tab = global_ptr(static_cast<const T*>(L.tab));
    const T c = tab[(L.pr[k] * BC + L.pc[l]) * R + r];
    return (L.sr[k] * L.sc[l] < 0) ? -c : c;
  }
}

// Levels [0, NS) of a group read their folded coefficients from a table staged
// in LDS once per workgroup (stage_coefs) instead of from the level's table in
// global memory.  A level's product loop is unrolled when R is compiled in, at
// most 8, and the level is the group's last; the rest loop over r.  Measured
// at N = 4096 unless stated:
//  - f64 (latency-bound sizes): every level staged; N = 64, two Strassen
//    levels, the whole product went from 67 to 51 us.
//  - R not compiled in or above 8 (Laderman's 23): every level staged; f32
//    Laderman Q = 2 scatter 224 -> 199 us, fp8 gathers 211 -> 188 us, f16
//    gathers (N = 2048) 79 -> 64 us, a whole fp8 product at N = 384 86 -> 56 us.
//  - Strassen, gathers to reduced-precision leaf operands: the looped outer
//    level staged (fp8, Q = 2: 77 -> 73-75 us).
//  - Strassen f32 gathers and scatters: nothing staged (the outer gather
//    level staged was 128 -> 131 us at Q = 3, the scatter 117 -> 125 us);
//    the scatter's looped level reads by scalar loads.
template <typename T, int NL, int R>
constexpr bool stage_all() {
  return sizeof(T) == 8 || R == 0 || R > 8;
}
// f16 outputs: the last level's product loop is not unrolled (its coefficients
// staged with the rest): N = 4096, Strassen Q = 2, the f16 gathers went from 69
// to 60.5 us.  For e4m3 outputs the same change freed the 138 spilled SGPRs but
// was mixed (large products 5% faster, N <= 1024 3% slower), so they stay unrolled.
template <int OUTF>
constexpr bool gather_rolled() {
  return OUTF == OUT_F16S;
}
template <typename T, int OUTF, int NL, int R>
constexpr int gather_staged() {
  return (stage_all<T, NL, R>() || gather_rolled<OUTF>()) ? NL : (OUTF != OUT_SAME && NL > 1 ? NL - 1 : 0);
}
template <typename T, int NL, int R>
constexpr int scatter_staged() {
  return stage_all<T, NL, R>() ? NL : 0;
}

// The staged coefficients of levels [0, NS) in LDS as [level][block kl][product
// r], r < R (kMaxR for a level whose count is not compiled in; entries past the
// level's count are zero).
template <int NS, int BB, int R>
constexpr int coef_entries() {
  return NS ? NS * BB * (R ? R : kMaxR) : 1;  // one unused entry when nothing is staged
}

// Every thread of the workgroup calls this; it ends with a barrier when it
// stages anything.
template <typename T, int NS, int BR, int BC, int R, int NT = 256>
__device__ __forceinline__ void stage_coefs(const SideLevel* lev, T* lds) {
  constexpr int BB = BR * BC, RM = R ? R : kMaxR;
  if constexpr (NS > 0) {
    for (int i = threadIdx.x; i < NS * BB * RM; i += NT) {
      const int lt = i / (BB * RM), rem = i - lt * (BB * RM), kl = rem / RM, r = rem - kl * RM;
      const SideLevel& L = lev[lt];
      const int RR = R ? R : L.R;
      lds[i] = r < RR ? coef<T, BC>(L, kl / BC, kl % BC, r, RR) : T(0);
    }
    __syncthreads();
  }
}

// The staging of one gather or scatter variant (callers declare
// coef_entries floats of LDS and stage them before the first block).
template <typename T, int OUTF, int NL, int BR, int BC, int R>
constexpr int gather_coef_entries() {
  return coef_entries<gather_staged<T, OUTF, NL, R>(), BR * BC, R>();
}
template <typename T, int NL, int BR, int BC, int R>
constexpr int scatter_coef_entries() {
  return coef_entries<scatter_staged<T, NL, R>(), BR * BC, R>();
}
template <typename T, int OUTF, int NL, int BR, int BC, int R>
__device__ __forceinline__ void stage_gather_coefs(const SideLevel* lev, T* lds) {
  stage_coefs<T, gather_staged<T, OUTF, NL, R>(), BR, BC, R>(lev, lds);
}
template <typename T, int NL, int BR, int BC, int R>
__device__ __forceinline__ void stage_scatter_coefs(const SideLevel* lev, T* lds) {
  stage_coefs<T, scatter_staged<T, NL, R>(), BR, BC, R>(lev, lds);
}

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// V consecutive element positions per thread: the loads and stores of a
// wavefront cover 64 V contiguous elements of every block it touches.
template <typename T, int V>
using VecT = T __attribute__((ext_vector_type(V)));

template <typename T, int V>
__device__ __forceinline__ VecT<T, V> vload(const gbl<const T>* p) {
#if RBC_NT_LOADS
  return __builtin_nontemporal_load(reinterpret_cast<const gbl<const VecT<T, V>>*>(p));
#else
  return *reinterpret_cast<const gbl<const VecT<T, V>>*>(p);
#endif
}

template <typename T, int V>
__device__ __forceinline__ void vstore(gbl<T>* p, VecT<T, V> v) {
  *reinterpret_cast<gbl<VecT<T, V>>*>(p) = v;
}
template <typename T, int V>
__device__ __forceinline__ void vstore_nt(gbl<T>* p, VecT<T, V> v) {
  __builtin_nontemporal_store(v, reinterpret_cast<gbl<VecT<T, V>>*>(p));
}

template <typename T, int OUTF, int V>
struct GatherEmit {
  void* dst;
  int64_t dst_batch, plane, off;
  const int32_t* exps;  // f16s: LDS copy of the exponents of outputs exp_base, exp_base + 1, ...
  int64_t exp_base;
  bool nt;              // streaming stores (GatherParams::nt_store)
  __device__ __forceinline__ void operator()(int64_t idx, VecT<T, V> v) const {
    if constexpr (OUTF == OUT_SAME) {
      gbl<T>* d = global_ptr(static_cast<T*>(dst)) + idx * dst_batch + off;
      if (nt) vstore_nt<T, V>(d, v);
      else vstore<T, V>(d, v);
    } else if constexpr (OUTF == OUT_FP8X2) {
      // scaled split: y = 2^e v, hi = rn_e4m3(y), lo = rn_e4m3(16 (y - hi)) (y - hi is exact);
      // the conversions are the hardware's OCP e4m3 round-to-nearest-even ones
      const int ex = exps[idx - exp_base];
      float y[4], r[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) y[e] = e < V ? ldexpf((float)v[e < V ? e : 0], ex) : 0.f;
      int hi = __builtin_amdgcn_cvt_pk_fp8_f32(y[0], y[1], 0, false);
      if constexpr (V == 4) hi = __builtin_amdgcn_cvt_pk_fp8_f32(y[2], y[3], hi, true);
      r[0] = 16.0f * (y[0] - __builtin_amdgcn_cvt_f32_fp8(hi, 0));
      r[1] = 16.0f * (y[1] - __builtin_amdgcn_cvt_f32_fp8(hi, 1));
      r[2] = 16.0f * (y[2] - __builtin_amdgcn_cvt_f32_fp8(hi, 2));
      r[3] = 16.0f * (y[3] - __builtin_amdgcn_cvt_f32_fp8(hi, 3));
      int lo = __builtin_amdgcn_cvt_pk_fp8_f32(r[0], r[1], 0, false);
      if constexpr (V == 4) lo = __builtin_amdgcn_cvt_pk_fp8_f32(r[2], r[3], lo, true);
      gbl<uint8_t>* d = global_ptr(static_cast<uint8_t*>(dst)) + idx * dst_batch + off;
      if constexpr (V == 4) {
        *reinterpret_cast<gbl<uint32_t>*>(d) = (uint32_t)hi;
        *reinterpret_cast<gbl<uint32_t>*>(d + plane) = (uint32_t)lo;
      } else if constexpr (V == 2) {
        *reinterpret_cast<gbl<uint16_t>*>(d) = (uint16_t)hi;
        *reinterpret_cast<gbl<uint16_t>*>(d + plane) = (uint16_t)lo;
      } else {
        d[0] = (uint8_t)hi;
        d[plane] = (uint8_t)lo;
      }
    } else if constexpr (OUTF == OUT_F16S) {
      // scaled leaf operand: rn_f16(2^e v), e chosen per leaf so nothing overflows
      const int ex = exps[idx - exp_base];
      VecT<uint16_t, V> h;
#pragma unroll
      for (int e = 0; e < V; ++e) h[e] = __builtin_bit_cast(uint16_t, (_Float16)ldexpf((float)v[e], ex));
      vstore<uint16_t, V>(global_ptr(static_cast<uint16_t*>(dst)) + idx * dst_batch + off, h);
    } else {
      // leaf operand split: hi = rn_bf16(v), lo = rn_bf16(v - hi) (v - hi is exact in f32)
      VecT<uint16_t, V> hi, lo;
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const float f = (float)v[e];
        hi[e] = bf16_rne(f);
        lo[e] = bf16_rne(f - bf16_to_float(hi[e]));
      }
      gbl<uint16_t>* d = global_ptr(static_cast<uint16_t*>(dst)) + idx * dst_batch + off;
      vstore<uint16_t, V>(d, hi);
      vstore<uint16_t, V>(d + plane, lo);
    }
  }
};

// Level T of a gather group: v holds BB^(NL-T) values of the current block,
// block (k, l) of this level occupying the SUB consecutive values at
// (k * BC + l) * SUB.  R > 0 is the compiled product count, R == 0 reads it
// from the level descriptor.
template <typename T, int V, int NL, int BR, int BC, int R, int NS, bool ROLL, int LT, typename Emit>
__device__ __forceinline__ void gather_level(const VecT<T, V>* v, const SideLevel* lev, const T* ct, int64_t idx,
                                             const Emit& emit) {
  if constexpr (LT == NL) {
    emit(idx, v[0]);
  } else {
    constexpr int BB = BR * BC;
    constexpr int SUB = ipow(BB, NL - LT - 1);
    const SideLevel& L = lev[LT];
    const int RR = R ? R : L.R;
    // Unroll only the innermost level's product loop, when R is compiled in and small.
    constexpr int UNR = (R == 0 || R > 8 || LT + 1 < NL || ROLL) ? 1 : R;
#pragma unroll UNR
    for (int r = 0; r < RR; ++r) {
      if constexpr (UNR == 1 && RBC_LEVEL_BARRIER) __asm__ volatile("" ::: "memory");
      VecT<T, V> acc[SUB];
#pragma unroll
      for (int j = 0; j < SUB; ++j) acc[j] = VecT<T, V>(T(0));
      // Branch-free sequential sum: a zero coefficient leaves acc untouched (selects on
      // uniform conditions instead of branches keep the scalar registers free).
      bool first = true;
#pragma unroll
      for (int kl = 0; kl < BB; ++kl) {
        T c;
        if constexpr (LT < NS) c = ct[(LT * BB + kl) * (R ? R : kMaxR) + r];
        else c = coef<T, BC>(L, kl / BC, kl % BC, r, RR);
        const bool nz = c != T(0);
#pragma unroll
        for (int j = 0; j < SUB; ++j) {
          const VecT<T, V> t = c * v[kl * SUB + j];
          const VecT<T, V> sum = first ? t : acc[j] + t;
          acc[j] = nz ? sum : acc[j];
        }
        first = first && !nz;
      }
      gather_level<T, V, NL, BR, BC, R, NS, ROLL, LT + 1>(acc, lev, ct, idx * RR + r, emit);
    }
  }
}

// Gathers over levels whose U (A side, KIND 0) or V (B side, KIND 1) table has
// Strassen's pattern (SideLevel::strassen).  Every product then sums at most two
// blocks, and the sum of two terms does not depend on their order (IEEE
// addition commutes, signed zeros included), so the walk can take the blocks in
// table-block order: the thread loads the source sub-block (k, l) that table
// block b = (pr[k], pc[l]) reads into slot b (b a digit per level), and the
// blocks that feed each product are known at compile time.  v: NSRC values,
// table block b of level LT at (b * SUB) + j.  The roundings are those of
// gather_level (fl(c x), then one addition).
template <typename T, int V, int NL, int NS, int KIND, int LT, typename Emit>
__device__ __forceinline__ void gather_level_sw(const VecT<T, V>* v, const SideLevel* lev, const T* ct,
                                                const int8_t (*kof)[4], const int8_t (*lof)[4], int64_t idx,
                                                const Emit& emit) {
  if constexpr (LT == NL) {
    emit(idx, v[0]);
  } else {
    constexpr int SUB = ipow(4, NL - LT - 1);
    const SideLevel& L = lev[LT];
#pragma unroll
    for (int r = 0; r < 7; ++r) {
      const int b1 = KIND == 0 ? kStrassenUNz[r][0] : kStrassenVNz[r][0];
      const int b2 = KIND == 0 ? kStrassenUNz[r][1] : kStrassenVNz[r][1];
      auto c_of = [&](int b) -> T {
        const int k = kof[LT][b], l = lof[LT][b];
        if constexpr (LT < NS)
          return ct[(LT * 4 + k * 2 + l) * 7 + r];
        else
          return coef<T, 2, true>(L, k, l, r, 7);
      };
      const T c1 = c_of(b1);
      VecT<T, V> acc[SUB];
#pragma unroll
      for (int j = 0; j < SUB; ++j) acc[j] = c1 * v[b1 * SUB + j];
      if (b2 >= 0) {
        const T c2 = c_of(b2);
#pragma unroll
        for (int j = 0; j < SUB; ++j) acc[j] = acc[j] + c2 * v[b2 * SUB + j];
      }
      gather_level_sw<T, V, NL, NS, KIND, LT + 1>(acc, lev, ct, kof, lof, idx * 7 + r, emit);
    }
  }
}

// Outputs of one top block in a gather group (R == 0: the level's own count,
// at most kMaxR for a single level).
template <int NL, int R>
constexpr int group_outputs() {
  return R ? ipow(R, NL) : kMaxR;
}

// f16s, fp8: the scale exponents of top block `in`'s outputs into LDS (every
// thread of the workgroup calls this; it ends with a barrier), so that each
// output block's exponent is one LDS read.  With p.scale_partial the exponents
// are derived here, e = floor(log2(target / (G max|X|))) from the partial
// maxima of |X| and the per-leaf path norms, and the workgroup with `writer`
// set also stores them for the leaf product; otherwise they are read from
// p.scale_exp.
template <int NL, int R>
__device__ __forceinline__ void load_exponents(const GatherParams& p, int64_t in, int32_t* lds,
                                               bool writer = false) {
  const int n = R ? ipow(R, NL) : p.lev[0].R;
  if (p.scale_partial) {
    float m = 0.f;
    for (int i = threadIdx.x; i < p.scale_nparts; i += 256) m = fmaxf(m, global_ptr(p.scale_partial)[i]);
    const float mx = scale::block_max(m);
    const gbl<const float>* G = global_ptr(p.scale_G) + in * n;
    gbl<int32_t>* e = global_ptr(p.scale_exp) + in * n;
    for (int j = threadIdx.x; j < n; j += 256) {
      const int32_t x = scale::leaf_exponent(mx, G[j], p.scale_target);
      lds[j] = x;
      if (writer) e[j] = x;
    }
  } else {
    const gbl<const int32_t>* e = global_ptr(p.scale_exp) + in * n;
    for (int j = threadIdx.x; j < n; j += 256) lds[j] = e[j];
  }
  __syncthreads();
}

// Whether gather_block takes the walk specialized to Strassen's pattern where
// the tables allow it (gather_level_sw).  It saves arithmetic but holds more
// registers: f32 gathers of four positions per thread, bound by HBM already,
// ran 10% slower with it (N = 4096, Q = 3: 49 -> 54 us a side).  Reduced-
// precision outputs gained: fp8c N = 4096, Q = 4 212 -> 170 us a side, f16s
// Q = 2 61 -> 54 us, bf16x3 N = 3072 79 -> 71 us; f64 81 -> 73 us; f32 with
// one position per thread (N = 1000) 17 -> 14 us.  The batch engine's
// persistent kernel chooses for itself (it takes the walk everywhere).
template <typename T, int OUTF, int V>
constexpr bool gather_sw_default() {
  return !(OUTF == OUT_SAME && sizeof(T) == 4 && V == 4);
}

// One workgroup's share of a gather: 256 threads x V positions (block bx of
// the position range) of top block `in`.  Used by k_gather and by the batch
// engine's kernels.  exps: for f16s outputs, top block `in`'s exponents in LDS
// (load_exponents).  SW: see gather_sw_default.
template <typename T, int OUTF, int V, int NL, int BR, int BC, int R, bool SW = gather_sw_default<T, OUTF, V>()>
__device__ __forceinline__ void gather_block(const GatherParams& p, const T* ct, int64_t bx, int64_t in,
                                             const int32_t* exps) {
  constexpr int BB = BR * BC;
  constexpr int NSRC = ipow(BB, NL);
  const int64_t npos = p.rows_bot * p.cols_bot;
  const int64_t pos = (bx * 256 + threadIdx.x) * V;
  if (pos >= npos) return;
  const int64_t y = pos / p.cols_bot, x = pos - y * p.cols_bot;  // cols_bot % V == 0
  const gbl<const T>* src = global_ptr(static_cast<const T*>(p.src)) + in * p.src_batch;
  // Strassen's pattern at every level of a group of one or two levels: slot s
  // holds the source sub-block that table block s (digit per level) reads
  bool sw = false;
  int8_t kof[kMaxGroupLevels][4] = {}, lof[kMaxGroupLevels][4] = {};
  if constexpr (SW && BR == 2 && BC == 2 && R == 7 && NL <= 2 && NL >= 1) {
    sw = true;
#pragma unroll
    for (int t = 0; t < NL; ++t) {
      sw = sw && p.lev[t].strassen != 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        kof[t][b] = p.lev[t].pr[0] == (b >> 1) ? 0 : 1;
        lof[t][b] = p.lev[t].pc[0] == (b & 1) ? 0 : 1;
      }
    }
  }
  VecT<T, V> v[NSRC];
#pragma unroll
  for (int s = 0; s < NSRC; ++s) {
    int64_t row = y, col = x, hs = p.rows_bot, ws = p.cols_bot;
    int rem = s;
#pragma unroll
    for (int t = 0; t < NL; ++t) {  // least significant digit = deepest level
      const int d = rem % BB;
      rem /= BB;
      const int lt = NL - 1 - t;
      const int kr = sw ? kof[lt][d] : d / BC, lc = sw ? lof[lt][d] : d % BC;
      row += kr * hs;
      col += lc * ws;
      hs *= BR;
      ws *= BC;
    }
    if (row < p.src_rows && col + V <= p.src_cols) {
      v[s] = vload<T, V>(src + row * p.ld_src + col);  // aligned: checked by the host
    } else {
#pragma unroll
      for (int e = 0; e < V; ++e)
        v[s][e] = (row < p.src_rows && col + e < p.src_cols) ? src[row * p.ld_src + col + e] : T(0);
    }
  }
  const int64_t n_out = R ? ipow(R, NL) : p.lev[0].R;
  GatherEmit<T, OUTF, V> e{p.dst, p.dst_batch, p.plane, pos, exps, in * n_out, p.nt_store != 0};
  constexpr int NS = gather_staged<T, OUTF, NL, R>();
  if constexpr (SW && BR == 2 && BC == 2 && R == 7 && NL <= 2 && NL >= 1) {
    if (sw) {
      if (p.side == 0)
        gather_level_sw<T, V, NL, NS, 0, 0>(v, p.lev, ct, kof, lof, in, e);
      else
        gather_level_sw<T, V, NL, NS, 1, 0>(v, p.lev, ct, kof, lof, in, e);
      return;
    }
  }
  gather_level<T, V, NL, BR, BC, R, NS, gather_rolled<OUTF>(), 0>(v, p.lev, ct, in, e);
}

// One side's share of a gather launch.
template <typename T, int OUTF, int V, int NL, int BR, int BC, int R>
__device__ __forceinline__ void gather_side(const GatherParams& p) {
  __shared__ T ct[gather_coef_entries<T, OUTF, NL, BR, BC, R>()];
  stage_gather_coefs<T, OUTF, NL, BR, BC, R>(p.lev, ct);
  if constexpr (OUTF == OUT_F16S || OUTF == OUT_FP8X2) {
    __shared__ int32_t exps[group_outputs<NL, R>()];
    for (int64_t in = blockIdx.y; in < p.n_in; in += gridDim.y) {
      if (in != blockIdx.y) __syncthreads();  // the previous block's readers are done
      load_exponents<NL, R>(p, in, exps, blockIdx.x == 0);
      gather_block<T, OUTF, V, NL, BR, BC, R>(p, ct, blockIdx.x, in, exps);
    }
  } else {
    for (int64_t in = blockIdx.y; in < p.n_in; in += gridDim.y)
      gather_block<T, OUTF, V, NL, BR, BC, R>(p, ct, blockIdx.x, in, nullptr);
  }
}

// Two gathers of one shape in one grid (the A and B sides of a level group):
// blockIdx.z selects the side; blocks past a side's positions or top blocks
// do nothing.  Each branch reads its own parameter block where it lies (a
// reference chosen between the two at run time made the compiler copy both
// into scratch memory).
// f16 outputs: held to 128 VGPRs (four workgroups per CU) without spills; at
// N = 4096, Q = 2 the f16 gather went from 60 to 51 us.  The e4m3 emission
// spills at that bound, and two positions per thread were slower (71 us).
template <typename T, int OUTF, int V, int NL, int BR, int BC, int R>
__global__ __launch_bounds__(256, OUTF == OUT_F16S ? 4 : 1) void k_gather(GatherParams pa, GatherParams pb) {
  if (blockIdx.z == 0)
    gather_side<T, OUTF, V, NL, BR, BC, R>(pa);
  else
    gather_side<T, OUTF, V, NL, BR, BC, R>(pb);
}

// Level LT of a scatter group: returns in `out` the BB^(NL-LT) values of the
// block at this level for subproblem prefix idx.
template <typename TP, typename TA, int V, int NL, int BR, int BC, int R, int NS, int LT>
__device__ __forceinline__ void scatter_level(const gbl<const TP>* src, int64_t src_batch, int64_t off,
                                              const SideLevel* lev, const TA* ct, int64_t idx, VecT<TA, V>* out) {
  if constexpr (LT == NL) {
    const VecT<TP, V> x = vload<TP, V>(src + idx * src_batch + off);
#pragma unroll
    for (int e = 0; e < V; ++e) out[0][e] = (TA)x[e];
  } else {
    constexpr int BB = BR * BC;
    constexpr int SUB = ipow(BB, NL - LT - 1);
    const SideLevel& L = lev[LT];
    const int RR = R ? R : L.R;
    bool first[BB];
#pragma unroll
    for (int ij = 0; ij < BB; ++ij) first[ij] = true;
#pragma unroll
    for (int j = 0; j < BB * SUB; ++j) out[j] = VecT<TA, V>(TA(0));
    constexpr int UNR = (R == 0 || R > 8 || LT + 1 < NL) ? 1 : R;
#pragma unroll UNR
    for (int r = 0; r < RR; ++r) {
      if constexpr (UNR == 1 && RBC_LEVEL_BARRIER) __asm__ volatile("" ::: "memory");
      VecT<TA, V> sub[SUB];
      scatter_level<TP, TA, V, NL, BR, BC, R, NS, LT + 1>(src, src_batch, off, lev, ct, idx * RR + r, sub);
#pragma unroll
      for (int ij = 0; ij < BB; ++ij) {
        TA c;
        if constexpr (LT < NS)
          c = ct[(LT * BB + ij) * (R ? R : kMaxR) + r];
        else
          c = coef<TA, BC, UNR == 1>(L, ij / BC, ij % BC, r, RR);
        const bool nz = c != TA(0);
#pragma unroll
        for (int j = 0; j < SUB; ++j) {
          const VecT<TA, V> t = c * sub[j];
          const VecT<TA, V> sum = first[ij] ? t : out[ij * SUB + j] + t;
          out[ij * SUB + j] = nz ? sum : out[ij * SUB + j];
        }
        first[ij] = first[ij] && !nz;
      }
    }
  }
}

// Scatters over levels whose W table has Strassen's zero pattern
// (SideLevel::strassen).  Output block ij of such a level reads table block
// b = (pr[k] * 2 + pc[l]) for (k, l) = (ij / 2, ij % 2); with the level's row
// and column permutations fixed (pr[0] = PR0, pc[0] = PC0) b is a compile-time
// function of ij, and so are the products that feed it (kStrassenWNz[b]), so
// the zero terms are never formed.  The first term stands alone and the rest
// are added in ascending r, as in scatter_level.
template <int PR0, int PC0>
__host__ __device__ constexpr int sw_block(int ij) {
  return (((ij >> 1) ^ PR0) << 1) | ((ij & 1) ^ PC0);
}

// The folded coefficient of output block ij, product r of a Strassen-shaped
// level: staged in LDS (level LT < NS) or the table entry by a scalar load,
// uniform either way.
template <typename TA, int NS, int LT>
__device__ __forceinline__ TA coef_u(const SideLevel* lev, const TA* ct, int ij, int r) {
  if constexpr (LT < NS)
    return ct[(LT * 4 + ij) * 7 + r];
  else
    return coef<TA, 2, true>(lev[LT], ij / 2, ij % 2, r, 7);
}

// Levels LO and LO + 1 of a scatter group (the latter its deepest, with
// Strassen's pattern) for prefix idx at level LO: out[ij1 * 4 + ij2] = block
// ij1 of level LO, sub-block ij2, the same roundings as scatter_level<.., LO>.
// The next level-LO product's seven loads are issued before the current one
// is combined.  Level LO skips a zero coefficient by a (uniform) branch, its
// sums starting at -0 so that the first term's sum is that term, sign of zero
// included; a sum that took no term is set to +0 at the end.
template <typename TP, typename TA, int V, int NS, int LO, int PR0, int PC0>
__device__ __forceinline__ void scatter2_sw(const gbl<const TP>* src, int64_t src_batch, int64_t off,
                                            const SideLevel* lev, const TA* ct, int64_t idx, VecT<TA, V>* out) {
  TA c2[4][4];
#pragma unroll
  for (int ij2 = 0; ij2 < 4; ++ij2) {
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int b = sw_block<PR0, PC0>(ij2);
      c2[ij2][n] = n < kStrassenWNzCount[b] ? coef_u<TA, NS, LO + 1>(lev, ct, ij2, kStrassenWNz[b][n]) : TA(0);
    }
  }
  bool any1[4] = {false, false, false, false};
#pragma unroll
  for (int j = 0; j < 16; ++j) out[j] = VecT<TA, V>(TA(-0.0));
  const gbl<const TP>* base = src + idx * 49 * src_batch + off;
  VecT<TA, V> x[7];
#pragma unroll
  for (int r2 = 0; r2 < 7; ++r2) {
    const VecT<TP, V> v = vload<TP, V>(base + r2 * src_batch);
#pragma unroll
    for (int e = 0; e < V; ++e) x[r2][e] = (TA)v[e];
  }
#pragma unroll 1
  for (int r1 = 0; r1 < 7; ++r1) {
    VecT<TP, V> xn[7];
    if (r1 + 1 < 7) {
#pragma unroll
      for (int r2 = 0; r2 < 7; ++r2) xn[r2] = vload<TP, V>(base + ((r1 + 1) * 7 + r2) * src_batch);
    }
    VecT<TA, V> p2[4];
#pragma unroll
    for (int ij2 = 0; ij2 < 4; ++ij2) {
      const int b = sw_block<PR0, PC0>(ij2);
      p2[ij2] = c2[ij2][0] * x[kStrassenWNz[b][0]];
#pragma unroll
      for (int n = 1; n < 4; ++n)
        if (n < kStrassenWNzCount[b]) p2[ij2] = p2[ij2] + c2[ij2][n] * x[kStrassenWNz[b][n]];
    }
#pragma unroll
    for (int ij1 = 0; ij1 < 4; ++ij1) {
      const TA c = coef_u<TA, NS, LO>(lev, ct, ij1, r1);
      if (c != TA(0)) {
        __asm__ volatile("");  // a uniform branch, not four selects per term
#pragma unroll
        for (int ij2 = 0; ij2 < 4; ++ij2) out[ij1 * 4 + ij2] = out[ij1 * 4 + ij2] + c * p2[ij2];
        any1[ij1] = true;
      }
    }
#pragma unroll
    for (int r2 = 0; r2 < 7; ++r2)
#pragma unroll
      for (int e = 0; e < V; ++e) x[r2][e] = (TA)xn[r2][e];
  }
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (!any1[j / 4]) out[j] = VecT<TA, V>(TA(0));
}

// scatter2_sw with level LO's table of Strassen's pattern as well, its case
// (pr[0], pc[0]) = (QR, QC) fixed: the products that feed each block of level
// LO are known at compile time too (kStrassenWNz[sw_block<QR, QC>(ij1)]), so
// the level-LO loop is unrolled and neither level forms a zero term or tests
// a coefficient.  Every output has at least two terms; the first stands alone.
template <typename TP, typename TA, int V, int NS, int LO, int PR0, int PC0, int QR, int QC>
__device__ __forceinline__ void scatter2_sww(const gbl<const TP>* src, int64_t src_batch, int64_t off,
                                             const SideLevel* lev, const TA* ct, int64_t idx, VecT<TA, V>* out) {
  TA c2[4][4], c1[4][4];
#pragma unroll
  for (int ij = 0; ij < 4; ++ij) {
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int b2 = sw_block<PR0, PC0>(ij), b1 = sw_block<QR, QC>(ij);
      c2[ij][n] = n < kStrassenWNzCount[b2] ? coef_u<TA, NS, LO + 1>(lev, ct, ij, kStrassenWNz[b2][n]) : TA(0);
      c1[ij][n] = n < kStrassenWNzCount[b1] ? coef_u<TA, NS, LO>(lev, ct, ij, kStrassenWNz[b1][n]) : TA(0);
    }
  }
  const gbl<const TP>* base = src + idx * 49 * src_batch + off;
#pragma unroll
  for (int r1 = 0; r1 < 7; ++r1) {
    VecT<TA, V> x[7];
#pragma unroll
    for (int r2 = 0; r2 < 7; ++r2) {
      const VecT<TP, V> v = vload<TP, V>(base + (r1 * 7 + r2) * src_batch);
#pragma unroll
      for (int e = 0; e < V; ++e) x[r2][e] = (TA)v[e];
    }
    VecT<TA, V> p2[4];
#pragma unroll
    for (int ij2 = 0; ij2 < 4; ++ij2) {
      const int b = sw_block<PR0, PC0>(ij2);
      p2[ij2] = c2[ij2][0] * x[kStrassenWNz[b][0]];
#pragma unroll
      for (int n = 1; n < 4; ++n)
        if (n < kStrassenWNzCount[b]) p2[ij2] = p2[ij2] + c2[ij2][n] * x[kStrassenWNz[b][n]];
    }
#pragma unroll
    for (int ij1 = 0; ij1 < 4; ++ij1) {
      const int b = sw_block<QR, QC>(ij1);
#pragma unroll
      for (int n = 0; n < 4; ++n)
        if (n < kStrassenWNzCount[b] && kStrassenWNz[b][n] == r1) {
#pragma unroll
          for (int ij2 = 0; ij2 < 4; ++ij2) {
            const VecT<TA, V> t = c1[ij1][n] * p2[ij2];
            out[ij1 * 4 + ij2] = n == 0 ? t : out[ij1 * 4 + ij2] + t;
          }
        }
    }
  }
}

// Calls f with std::integral_constant<int, c> for a permutation case c in 0..3.
template <typename F>
__device__ __forceinline__ void sw_case(int c, F&& f) {
  if (c == 0)
    f(std::integral_constant<int, 0>());
  else if (c == 1)
    f(std::integral_constant<int, 1>());
  else if (c == 2)
    f(std::integral_constant<int, 2>());
  else
    f(std::integral_constant<int, 3>());
}

// The deepest level alone, with Strassen's pattern: out[ij] = block ij for
// prefix idx, the products that feed it known at compile time (PR0, PC0 as
// above), first term alone, r ascending.
template <typename TP, typename TA, int V, int NS, int PR0, int PC0>
__device__ __forceinline__ void scatter1_sw(const gbl<const TP>* src, int64_t src_batch, int64_t off,
                                            const SideLevel* lev, const TA* ct, int64_t idx, VecT<TA, V>* out) {
  const gbl<const TP>* base = src + idx * 7 * src_batch + off;
  VecT<TA, V> x[7];
#pragma unroll
  for (int r = 0; r < 7; ++r) {
    const VecT<TP, V> v = vload<TP, V>(base + r * src_batch);
#pragma unroll
    for (int e = 0; e < V; ++e) x[r][e] = (TA)v[e];
  }
#pragma unroll
  for (int ij = 0; ij < 4; ++ij) {
    const int b = sw_block<PR0, PC0>(ij);
    out[ij] = coef_u<TA, NS, 0>(lev, ct, ij, kStrassenWNz[b][0]) * x[kStrassenWNz[b][0]];
#pragma unroll
    for (int n = 1; n < 4; ++n)
      if (n < kStrassenWNzCount[b])
        out[ij] = out[ij] + coef_u<TA, NS, 0>(lev, ct, ij, kStrassenWNz[b][n]) * x[kStrassenWNz[b][n]];
  }
}

// Output sub-block s of a scatter group (digits base BR * BC, the deepest
// level's least significant) at bottom position (y, x) of top block dst.
template <typename TA, typename TO, int V, int NL, int BR, int BC>
__device__ __forceinline__ void scatter_store(const ScatterParams& p, gbl<TO>* dst, int64_t y, int64_t x, int s,
                                              const VecT<TA, V>& v) {
  constexpr int BB = BR * BC;
  int64_t row = y, col = x, hs = p.rows_bot, ws = p.cols_bot;
  int rem = s;
#pragma unroll
  for (int t = 0; t < NL; ++t) {
    const int d = rem % BB;
    rem /= BB;
    row += (d / BC) * hs;
    col += (d % BC) * ws;
    hs *= BR;
    ws *= BC;
  }
  VecT<TO, V> w;
#pragma unroll
  for (int e = 0; e < V; ++e) w[e] = (TO)v[e];
  if (row < p.dst_rows && col + V <= p.dst_cols) {
    *reinterpret_cast<gbl<VecT<TO, V>>*>(dst + row * p.ld_dst + col) = w;  // aligned: checked by the host
  } else {
#pragma unroll
    for (int e = 0; e < V; ++e)
      if (row < p.dst_rows && col + e < p.dst_cols) dst[row * p.ld_dst + col + e] = w[e];
  }
}

// One workgroup's share of a scatter: 256 threads x V positions (block bx)
// of top block o.
template <typename TP, typename TA, typename TO, int V, int NL, int BR, int BC, int R>
__device__ __forceinline__ void scatter_block(const ScatterParams& p, const TA* ct, int64_t bx, int64_t o) {
  constexpr int NOUT = ipow(BR * BC, NL);
  const int64_t npos = p.rows_bot * p.cols_bot;
  const int64_t pos = (bx * 256 + threadIdx.x) * V;
  if (pos >= npos) return;
  const int64_t y = pos / p.cols_bot, x = pos - y * p.cols_bot;
  const gbl<const TP>* src = global_ptr(static_cast<const TP*>(p.src));
  VecT<TA, V> out[NOUT];
  constexpr int NS = scatter_staged<TA, NL, R>();
  // Strassen's pattern in the deepest level's table: its case (pr[0], pc[0])
  int sw = -1;
  if constexpr (BR == 2 && BC == 2 && R == 7 && (NL == 1 || NL == 2)) {
    const SideLevel& D = p.lev[NL - 1];
    if (D.strassen) sw = D.pr[0] * 2 + D.pc[0];
  }
  if constexpr (BR == 2 && BC == 2 && R == 7 && NL == 2) {
    const int sw0 = p.lev[0].strassen ? p.lev[0].pr[0] * 2 + p.lev[0].pc[0] : -1;
    if (sw >= 0 && sw0 >= 0)
      sw_case(sw, [&](auto k1) {
        constexpr int c1 = decltype(k1)::value;
        sw_case(sw0, [&](auto k0) {
          constexpr int c0 = decltype(k0)::value;
          scatter2_sww<TP, TA, V, NS, 0, (c1 >> 1), (c1 & 1), (c0 >> 1), (c0 & 1)>(src, p.src_batch, pos, p.lev, ct,
                                                                                   o, out);
        });
      });
    else if (sw == 0)
      scatter2_sw<TP, TA, V, NS, 0, 0, 0>(src, p.src_batch, pos, p.lev, ct, o, out);
    else if (sw == 1)
      scatter2_sw<TP, TA, V, NS, 0, 0, 1>(src, p.src_batch, pos, p.lev, ct, o, out);
    else if (sw == 2)
      scatter2_sw<TP, TA, V, NS, 0, 1, 0>(src, p.src_batch, pos, p.lev, ct, o, out);
    else if (sw == 3)
      scatter2_sw<TP, TA, V, NS, 0, 1, 1>(src, p.src_batch, pos, p.lev, ct, o, out);
    else
      scatter_level<TP, TA, V, NL, BR, BC, R, NS, 0>(src, p.src_batch, pos, p.lev, ct, o, out);
  } else if constexpr (BR == 2 && BC == 2 && R == 7 && NL == 1) {
    if (sw == 0)
      scatter1_sw<TP, TA, V, NS, 0, 0>(src, p.src_batch, pos, p.lev, ct, o, out);
    else if (sw == 1)
      scatter1_sw<TP, TA, V, NS, 0, 1>(src, p.src_batch, pos, p.lev, ct, o, out);
    else if (sw == 2)
      scatter1_sw<TP, TA, V, NS, 1, 0>(src, p.src_batch, pos, p.lev, ct, o, out);
    else if (sw == 3)
      scatter1_sw<TP, TA, V, NS, 1, 1>(src, p.src_batch, pos, p.lev, ct, o, out);
    else
      scatter_level<TP, TA, V, NL, BR, BC, R, NS, 0>(src, p.src_batch, pos, p.lev, ct, o, out);
  } else {
    scatter_level<TP, TA, V, NL, BR, BC, R, NS, 0>(src, p.src_batch, pos, p.lev, ct, o, out);
  }
  gbl<TO>* dst = global_ptr(static_cast<TO*>(p.dst)) + o * p.dst_batch;
#pragma unroll
  for (int s = 0; s < NOUT; ++s) scatter_store<TA, TO, V, NL, BR, BC>(p, dst, y, x, s, out[s]);
}

template <typename TP, typename TA, typename TO, int V, int NL, int BR, int BC, int R>
__global__ __launch_bounds__(256) void k_scatter(ScatterParams p) {
  __shared__ TA ct[scatter_coef_entries<TA, NL, BR, BC, R>()];
  stage_scatter_coefs<TA, NL, BR, BC, R>(p.lev, ct);
  for (int64_t o = blockIdx.y; o < p.n_out; o += gridDim.y)
    scatter_block<TP, TA, TO, V, NL, BR, BC, R>(p, ct, blockIdx.x, o);
}

// The top level of a three-level group with Strassen's pattern for the 8
// output sub-blocks j0 .. j0 + 7 of top block ij (uniform): acc[q] = the sum
// over the nonzero products r of c_r m[r][j0 + q], first term alone, r
// ascending.  The table block, and with it the products, is chosen by a
// uniform branch.
template <typename TA, int V, int NS>
__device__ __forceinline__ void scatter3_top_sw(const SideLevel* lev, const TA* ct, int ij, int j0,
                                                const VecT<TA, V>* m, int lane, VecT<TA, V>* acc) {
  auto body = [&](auto bconst) {
    constexpr int b = decltype(bconst)::value;
    TA c[4];
#pragma unroll
    for (int n = 0; n < kStrassenWNzCount[b]; ++n) c[n] = coef_u<TA, NS, 0>(lev, ct, ij, kStrassenWNz[b][n]);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      acc[q] = c[0] * m[(kStrassenWNz[b][0] * 16 + j0 + q) * 64 + lane];
#pragma unroll
      for (int n = 1; n < kStrassenWNzCount[b]; ++n)
        acc[q] = acc[q] + c[n] * m[(kStrassenWNz[b][n] * 16 + j0 + q) * 64 + lane];
    }
  };
  const int b = __builtin_amdgcn_readfirstlane(lev[0].pr[ij >> 1] * 2 + lev[0].pc[ij & 1]);
  if (b == 0)
    body(std::integral_constant<int, 0>());
  else if (b == 1)
    body(std::integral_constant<int, 1>());
  else if (b == 2)
    body(std::integral_constant<int, 2>());
  else
    body(std::integral_constant<int, 3>());
}

// Three fused levels of 2 x 2 blocks and 7 products each.  A task is one top
// block and 64 V positions of the bottom block; a persistent workgroup of 512
// threads walks its tasks in a two-stage pipeline with two LDS buffers.  In
// step t every wavefront w first combines the top level of task t - 1 for its
// 8 output sub-blocks 8 w .. 8 w + 7 (top block w / 2, so the coefficients are
// uniform) over ascending r and stores them; then wavefront w < 7 forms, for
// task t and the top level's product w, the 16 sub-block values of the two
// lower levels (the walk and order of one thread of k_scatter, specialized
// where the tables have Strassen's pattern) and leaves them in LDS.  One barrier per step.  Every output is the same
// sequence of roundings as in k_scatter, so the bits are the same.  Measured
// on the f32 scatter of N = 4096, Q = 3 (one box): two passes (k_scatter over
// levels [1, 3), then level 0) 143 us; one thread holding all 64 outputs of a
// position, about 100 values in registers, 124-132 us; this kernel with the
// general walk 122-131 us, with only loads in the walk 80 us (the walk's
// selects and multiplies bound it, not the memory), with the deepest level's
// walk specialized to Strassen's pattern 94 us, and with the middle level's as
// well (scatter2_sww) 83 us.
template <typename TP, typename TA, typename TO, int V>
__global__ __launch_bounds__(512) void k_scatter3(ScatterParams p) {
  constexpr int NL = 3, BR = 2, BC = 2, R = 7, SUB = 16;
  constexpr int NS = scatter_staged<TA, NL, R>();
  __shared__ TA ct[scatter_coef_entries<TA, NL, BR, BC, R>()];
  __shared__ VecT<TA, V> mid[2][R * SUB * 64];
  stage_coefs<TA, NS, BR, BC, R, 512>(p.lev, ct);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ij = w >> 1, j0 = (w & 1) * 8;
  const int64_t npos = p.rows_bot * p.cols_bot;
  const int64_t nblk = (npos + 64 * V - 1) / (64 * V);
  const int64_t ntask = nblk * p.n_out;
  const int64_t mine = blockIdx.x < ntask ? (ntask - 1 - blockIdx.x) / gridDim.x + 1 : 0;
  const gbl<const TP>* src = global_ptr(static_cast<const TP*>(p.src));
  // Strassen's pattern in the top level's table; in the middle and deepest
  // levels', the case (pr[0], pc[0]) of their specialized walks (-1: none)
  const bool sw0 = p.lev[0].strassen != 0;
  const int sw1 = p.lev[1].strassen ? p.lev[1].pr[0] * 2 + p.lev[1].pc[0] : -1;
  const int sw2 = p.lev[2].strassen ? p.lev[2].pr[0] * 2 + p.lev[2].pc[0] : -1;
  for (int64_t t = 0; t <= mine; ++t) {
    if (t > 0) {
      const int64_t task = blockIdx.x + (t - 1) * gridDim.x;
      const int64_t o = task / nblk, pos = ((task - o * nblk) * 64 + lane) * V;
      const VecT<TA, V>* m = mid[(t - 1) & 1];
      VecT<TA, V> acc[8];
      if (sw0) {
        scatter3_top_sw<TA, V, NS>(p.lev, ct, ij, j0, m, lane, acc);
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = VecT<TA, V>(TA(0));
        bool first = true;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          TA c;
          if constexpr (NS > 0)
            c = ct[ij * R + r];
          else
            c = coef<TA, BC, true>(p.lev[0], ij / BC, ij % BC, r, R);
          const bool nz = c != TA(0);
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const VecT<TA, V> tv = c * m[(r * SUB + j0 + q) * 64 + lane];
            const VecT<TA, V> sum = first ? tv : acc[q] + tv;
            acc[q] = nz ? sum : acc[q];
          }
          first = first && !nz;
        }
      }
      if (pos < npos) {
        const int64_t y = pos / p.cols_bot, x = pos - y * p.cols_bot;
        gbl<TO>* dst = global_ptr(static_cast<TO*>(p.dst)) + o * p.dst_batch;
#pragma unroll
        for (int q = 0; q < 8; ++q) scatter_store<TA, TO, V, NL, BR, BC>(p, dst, y, x, ij * SUB + j0 + q, acc[q]);
      }
    }
    if (w < R && t < mine) {
      const int64_t task = blockIdx.x + t * gridDim.x;
      const int64_t o = task / nblk, pos = ((task - o * nblk) * 64 + lane) * V;
      VecT<TA, V> sub[SUB];
      if (pos < npos) {
        const gbl<const TP>* s0 = src;
        const int64_t pr = o * R + w;
        if (sw2 >= 0 && sw1 >= 0) {
          sw_case(sw2, [&](auto k2) {
            constexpr int c2 = decltype(k2)::value;
            sw_case(sw1, [&](auto k1) {
              constexpr int c1 = decltype(k1)::value;
              scatter2_sww<TP, TA, V, NS, 1, (c2 >> 1), (c2 & 1), (c1 >> 1), (c1 & 1)>(s0, p.src_batch, pos, p.lev,
                                                                                      ct, pr, sub);
            });
          });
        } else if (sw2 == 0)
          scatter2_sw<TP, TA, V, NS, 1, 0, 0>(s0, p.src_batch, pos, p.lev, ct, pr, sub);
        else if (sw2 == 1)
          scatter2_sw<TP, TA, V, NS, 1, 0, 1>(s0, p.src_batch, pos, p.lev, ct, pr, sub);
        else if (sw2 == 2)
          scatter2_sw<TP, TA, V, NS, 1, 1, 0>(s0, p.src_batch, pos, p.lev, ct, pr, sub);
        else if (sw2 == 3)
          scatter2_sw<TP, TA, V, NS, 1, 1, 1>(s0, p.src_batch, pos, p.lev, ct, pr, sub);
        else
          scatter_level<TP, TA, V, NL, BR, BC, R, NS, 1>(src, p.src_batch, pos, p.lev, ct, pr, sub);
      } else {
#pragma unroll
        for (int j = 0; j < SUB; ++j) sub[j] = VecT<TA, V>(TA(0));
      }
#pragma unroll
      for (int j = 0; j < SUB; ++j) mid[t & 1][(w * SUB + j) * 64 + lane] = sub[j];
    }
    __syncthreads();
  }
}

inline dim3 grid_for(int64_t npos, int64_t nbatch) {
  const int64_t gx = (npos + 255) / 256;
  const int64_t gy = nbatch < 65535 ? nbatch : 65535;
  return dim3((unsigned)gx, (unsigned)gy, 1);
}

template <typename T, int OUTF, int V, int NL, int BR, int BC, int R>
hipError_t run_gather(const GatherPair& pp, hipStream_t s) {
  const GatherParams& a = pp.a;
  const GatherParams& b = pp.sides == 2 ? pp.b : pp.a;
  const int64_t na = a.rows_bot * a.cols_bot / V, nb = b.rows_bot * b.cols_bot / V;
  dim3 g = grid_for(na > nb ? na : nb, a.n_in > b.n_in ? a.n_in : b.n_in);
  g.z = pp.sides == 2 ? 2 : 1;
  hipLaunchKernelGGL((k_gather<T, OUTF, V, NL, BR, BC, R>), g, dim3(256), 0, s, a, b);
  return hipGetLastError();
}

template <typename TP, typename TA, typename TO, int V, int NL, int BR, int BC, int R>
hipError_t run_scatter(const ScatterParams& p, hipStream_t s) {
  if constexpr (NL == 3 && BR == 2 && BC == 2 && R == 7) {
    // one position per thread whatever the alignment allows: with two, the
    // walk's registers and the doubled LDS buffers leave one workgroup per CU
    constexpr int VV = 1;
    const int64_t ntask = (p.rows_bot * p.cols_bot / VV + 63) / 64 * p.n_out;
    void (*kfn)(ScatterParams) = k_scatter3<TP, TA, TO, VV>;
    const int64_t slots = resident_blocks(reinterpret_cast<const void*>(kfn), 512);
    const int64_t g = slots > 0 && slots < ntask ? slots : ntask;
    hipLaunchKernelGGL(kfn, dim3((unsigned)g), dim3(512), 0, s, p);
  } else {
    hipLaunchKernelGGL((k_scatter<TP, TA, TO, V, NL, BR, BC, R>),
                       grid_for(p.rows_bot * p.cols_bot / V, p.n_out), dim3(256), 0, s, p);
  }
  return hipGetLastError();
}

// Shape dispatch.  F is a functor template taking <NL, BR, BC, R>.
template <template <int, int, int, int> class F, typename P>
hipError_t dispatch_shape(int nl, int br, int bc, int R, const P& p, hipStream_t s) {
  if (nl == 0) return F<0, 1, 1, 1>::run(p, s);
  if (nl == 3 && br == 2 && bc == 2 && R == 7) return F<3, 2, 2, 7>::run(p, s);
  if (nl == 2 && br == 2 && bc == 2 && R == 7) return F<2, 2, 2, 7>::run(p, s);
  if (nl == 1 && br == 2 && bc == 2 && R == 7) return F<1, 2, 2, 7>::run(p, s);
  if (nl == 1 && br == 3 && bc == 3 && R == 23) return F<1, 3, 3, 23>::run(p, s);
  if (nl != 1) return hipErrorInvalidValue;
#define RBC_SHAPE(a, b) \
  if (br == a && bc == b) return F<1, a, b, 0>::run(p, s);
  RBC_SHAPE(1, 1) RBC_SHAPE(1, 2) RBC_SHAPE(1, 3) RBC_SHAPE(1, 4)
  RBC_SHAPE(2, 1) RBC_SHAPE(2, 2) RBC_SHAPE(2, 3) RBC_SHAPE(2, 4)
  RBC_SHAPE(3, 1) RBC_SHAPE(3, 2) RBC_SHAPE(3, 3) RBC_SHAPE(3, 4)
  RBC_SHAPE(4, 1) RBC_SHAPE(4, 2) RBC_SHAPE(4, 3) RBC_SHAPE(4, 4)
#undef RBC_SHAPE
  return hipErrorInvalidValue;
}

template <typename T, int OUTF, int V>
struct GatherOf {
  template <int NL, int BR, int BC, int R>
  struct F {
    static hipError_t run(const GatherPair& p, hipStream_t s) {
      return run_gather<T, OUTF, V, NL, BR, BC, R>(p, s);
    }
  };
};

template <typename TP, typename TA, typename TO, int V>
struct ScatterOf {
  template <int NL, int BR, int BC, int R>
  struct F {
    static hipError_t run(const ScatterParams& p, hipStream_t s) {
      return run_scatter<TP, TA, TO, V, NL, BR, BC, R>(p, s);
    }
  };
};

// vec: positions per thread (1, 2 or 4), chosen by the host from the
// alignment of every pointer, leading dimension and block stride involved.
template <typename T, int OUTF>
hipError_t gather_dispatch(int vec, int nl, int br, int bc, int R, const GatherPair& p, hipStream_t s) {
  if (vec == 4) return dispatch_shape<GatherOf<T, OUTF, 4>::template F>(nl, br, bc, R, p, s);
  if (vec == 2) return dispatch_shape<GatherOf<T, OUTF, 2>::template F>(nl, br, bc, R, p, s);
  return dispatch_shape<GatherOf<T, OUTF, 1>::template F>(nl, br, bc, R, p, s);
}

template <typename TP, typename TA, typename TO>
hipError_t scatter_dispatch(int vec, int nl, int br, int bc, int R, const ScatterParams& p,
                            hipStream_t s) {
  if (vec == 4) return dispatch_shape<ScatterOf<TP, TA, TO, 4>::template F>(nl, br, bc, R, p, s);
  if (vec == 2) return dispatch_shape<ScatterOf<TP, TA, TO, 2>::template F>(nl, br, bc, R, p, s);
  return dispatch_shape<ScatterOf<TP, TA, TO, 1>::template F>(nl, br, bc, R, p, s);
}

#define RBC_GATHER_COMBOS(X) \
  X(double, OUT_SAME) X(float, OUT_SAME) X(float, OUT_BF16X2) X(float, OUT_F16S) X(float, OUT_FP8X2)
#define RBC_SCATTER_COMBOS(X)                                                          \
  X(double, double, double) X(float, float, float) X(float, double, double)            \
  X(float, double, float) X(double, double, float)

#define RBC_DECL_G(T, O)                                                                   \
  extern template hipError_t gather_dispatch<T, O>(int, int, int, int, int, const GatherPair&, \
                                                   hipStream_t);
#define RBC_DECL_S(A, B, C)                                                                          \
  extern template hipError_t scatter_dispatch<A, B, C>(int, int, int, int, int, const ScatterParams&, \
                                                        hipStream_t);

}  // namespace comb
}  // namespace rbc
