// Schemes: storage, validation by the Brent equations, builtin exact schemes.
//
// Brent equations (Section 1, eq. requirement): sum_r u_klr v_k'l'r w_ijr =
// delta(k,i) delta(l',j) delta(l,k') for every index 6-tuple.  tau is the
// Frobenius norm of the residual Y - X (Definition 1, eqs. def-x, def-y),
// kappa the mean defect on the n^3 entries where X = 1 (eq. epsilon-def;
// divided by b1 b2 b3 for rectangular blocks).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "core.hpp"

namespace rbc {

static thread_local std::string g_last_error;

rbc_status fail(rbc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

void clear_error() { g_last_error.clear(); }

const char* last_error_text() { return g_last_error.c_str(); }

static bool is_integer(double x) { return std::isfinite(x) && std::floor(x) == x && std::fabs(x) < 1e15; }

void analyse(Scheme& s) {
  const int b1 = s.b1, b2 = s.b2, b3 = s.b3, R = s.R;
  auto U = [&](int k, int l, int r) { return s.U[(k * b2 + l) * R + r]; };
  auto V = [&](int k, int l, int r) { return s.V[(k * b3 + l) * R + r]; };
  auto W = [&](int i, int j, int r) { return s.W[(i * b3 + j) * R + r]; };
  s.integral = true;
  for (double x : s.U) s.integral &= is_integer(x);
  for (double x : s.V) s.integral &= is_integer(x);
  for (double x : s.W) s.integral &= is_integer(x);

  // Brute force over [b1] x [b2] x [b2] x [b3] x [b1] x [b3].
  long double res2 = 0, y2 = 0;
  int64_t ires2 = 0, iy2 = 0;
  for (int k = 0; k < b1; ++k)
    for (int l = 0; l < b2; ++l)
      for (int kp = 0; kp < b2; ++kp)
        for (int lp = 0; lp < b3; ++lp)
          for (int i = 0; i < b1; ++i)
            for (int j = 0; j < b3; ++j) {
              const int x = (k == i && lp == j && l == kp) ? 1 : 0;
              if (s.integral) {
                int64_t y = 0;
                for (int r = 0; r < R; ++r)
                  y += (int64_t)U(k, l, r) * (int64_t)V(kp, lp, r) * (int64_t)W(i, j, r);
                ires2 += (y - x) * (y - x);
                iy2 += y * y;
              } else {
                long double y = 0;
                for (int r = 0; r < R; ++r) y += (long double)U(k, l, r) * V(kp, lp, r) * W(i, j, r);
                res2 += (y - x) * (y - x);
                y2 += y * y;
              }
            }
  if (s.integral) {
    s.tau = std::sqrt((double)ires2);
    s.ynorm = std::sqrt((double)iy2);
  } else {
    s.tau = (double)std::sqrt(res2);
    s.ynorm = (double)std::sqrt(y2);
  }

  // kappa: defect summed over the (i, l, j) triples where X = 1.
  double total = 0;
  for (int i = 0; i < b1; ++i)
    for (int l = 0; l < b2; ++l)
      for (int j = 0; j < b3; ++j) {
        double y = 0;
        for (int r = 0; r < R; ++r) y += U(i, l, r) * V(l, j, r) * W(i, j, r);
        total += 1.0 - y;
      }
  s.kappa_total = total;
  s.kappa = total / (double)(b1 * b2 * b3);

  // q = sqrt(sum_r ||U_r||^2 ||V_r||^2 ||W_r||^2) (eq. square-root-of-sum)
  double q2 = 0;
  for (int r = 0; r < R; ++r) {
    double nu = 0, nv = 0, nw = 0;
    for (int k = 0; k < b1; ++k)
      for (int l = 0; l < b2; ++l) nu += U(k, l, r) * U(k, l, r);
    for (int k = 0; k < b2; ++k)
      for (int l = 0; l < b3; ++l) nv += V(k, l, r) * V(k, l, r);
    for (int i = 0; i < b1; ++i)
      for (int j = 0; j < b3; ++j) nw += W(i, j, r) * W(i, j, r);
    q2 += nu * nv * nw;
  }
  s.q = std::sqrt(q2);
}

rbc_status make_scheme(int b1, int b2, int b3, int R, const double* U, const double* V,
                       const double* W, double residual_tol, Scheme& out) {
  if (b1 < 1 || b2 < 1 || b3 < 1 || b1 > kMaxB || b2 > kMaxB || b3 > kMaxB)
    return fail(RBC_EINVAL, "block partition <%d,%d,%d> outside 1..%d", b1, b2, b3, kMaxB);
  if (R < 1 || R > kMaxR) return fail(RBC_EINVAL, "R = %d outside 1..%d", R, kMaxR);
  if (!U || !V || !W) return fail(RBC_EINVAL, "null tensor pointer");
  Scheme s;
  s.b1 = b1, s.b2 = b2, s.b3 = b3, s.R = R;
  s.U.assign(U, U + b1 * b2 * R);
  s.V.assign(V, V + b2 * b3 * R);
  s.W.assign(W, W + b1 * b3 * R);
  for (double x : s.U) if (!std::isfinite(x)) return fail(RBC_EINVAL, "non-finite entry in U");
  for (double x : s.V) if (!std::isfinite(x)) return fail(RBC_EINVAL, "non-finite entry in V");
  for (double x : s.W) if (!std::isfinite(x)) return fail(RBC_EINVAL, "non-finite entry in W");
  analyse(s);
  if (!(s.tau <= residual_tol))
    return fail(RBC_ESCHEME, "Brent residual tau = %.6g exceeds tolerance %.6g", s.tau, residual_tol);
  if (std::fabs(1.0 - s.kappa) < 1e-12)
    return fail(RBC_ESCHEME, "kappa = %.17g: (1 - kappa)^-1 undefined", s.kappa);
  out = std::move(s);
  return RBC_OK;
}

// Strassen (1969), in the form of Golub & Van Loan:
//   P1 = (A11+A22)(B11+B22), P2 = (A21+A22)B11, P3 = A11(B12-B22), P4 = A22(B21-B11),
//   P5 = (A11+A12)B22, P6 = (A21-A11)(B11+B12), P7 = (A12-A22)(B21+B22);
//   C11 = P1+P4-P5+P7, C12 = P3+P5, C21 = P2+P4, C22 = P1-P2+P3+P6.
// Each row lists, per product, the coefficients of blocks 11, 12, 21, 22.
static const int kStrassenA[7][4] = {{1, 0, 0, 1}, {0, 0, 1, 1}, {1, 0, 0, 0}, {0, 0, 0, 1},
                                     {1, 1, 0, 0}, {-1, 0, 1, 0}, {0, 1, 0, -1}};
static const int kStrassenB[7][4] = {{1, 0, 0, 1}, {1, 0, 0, 0}, {0, 1, 0, -1}, {-1, 0, 1, 0},
                                     {0, 0, 0, 1}, {1, 1, 0, 0}, {0, 0, 1, 1}};
static const int kStrassenC[7][4] = {{1, 0, 0, 1}, {0, 0, 1, -1}, {0, 1, 0, 1}, {1, 0, 1, 0},
                                     {-1, 1, 0, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}};

// Laderman (1976), rank 23 for 3x3 blocks.  Per product, the coefficients of
// blocks 11 12 13 21 22 23 31 32 33 of A and of B; then, per output block,
// the products summed with coefficient +1.
static const int kLadermanA[23][9] = {
    {1, 1, 1, -1, -1, 0, 0, -1, -1}, {1, 0, 0, -1, 0, 0, 0, 0, 0},  {0, 0, 0, 0, 1, 0, 0, 0, 0},
    {-1, 0, 0, 1, 1, 0, 0, 0, 0},    {0, 0, 0, 1, 1, 0, 0, 0, 0},   {1, 0, 0, 0, 0, 0, 0, 0, 0},
    {-1, 0, 0, 0, 0, 0, 1, 1, 0},    {-1, 0, 0, 0, 0, 0, 1, 0, 0},  {0, 0, 0, 0, 0, 0, 1, 1, 0},
    {1, 1, 1, 0, -1, -1, -1, -1, 0}, {0, 0, 0, 0, 0, 0, 0, 1, 0},   {0, 0, -1, 0, 0, 0, 0, 1, 1},
    {0, 0, 1, 0, 0, 0, 0, 0, -1},    {0, 0, 1, 0, 0, 0, 0, 0, 0},   {0, 0, 0, 0, 0, 0, 0, 1, 1},
    {0, 0, -1, 0, 1, 1, 0, 0, 0},    {0, 0, 1, 0, 0, -1, 0, 0, 0},  {0, 0, 0, 0, 1, 1, 0, 0, 0},
    {0, 1, 0, 0, 0, 0, 0, 0, 0},     {0, 0, 0, 0, 0, 1, 0, 0, 0},   {0, 0, 0, 1, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 1, 0, 0},     {0, 0, 0, 0, 0, 0, 0, 0, 1}};
static const int kLadermanB[23][9] = {
    {0, 0, 0, 0, 1, 0, 0, 0, 0},      {0, -1, 0, 0, 1, 0, 0, 0, 0}, {-1, 1, 0, 1, -1, -1, -1, 0, 1},
    {1, -1, 0, 0, 1, 0, 0, 0, 0},     {-1, 1, 0, 0, 0, 0, 0, 0, 0}, {1, 0, 0, 0, 0, 0, 0, 0, 0},
    {1, 0, -1, 0, 0, 1, 0, 0, 0},     {0, 0, 1, 0, 0, -1, 0, 0, 0}, {-1, 0, 1, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, 0, 0, 0},      {-1, 0, 1, 1, -1, -1, -1, 1, 0}, {0, 0, 0, 0, 1, 0, 1, -1, 0},
    {0, 0, 0, 0, 1, 0, 0, -1, 0},     {0, 0, 0, 0, 0, 0, 1, 0, 0},  {0, 0, 0, 0, 0, 0, -1, 1, 0},
    {0, 0, 0, 0, 0, 1, 1, 0, -1},     {0, 0, 0, 0, 0, 1, 0, 0, -1}, {0, 0, 0, 0, 0, 0, -1, 0, 1},
    {0, 0, 0, 1, 0, 0, 0, 0, 0},      {0, 0, 0, 0, 0, 0, 0, 1, 0},  {0, 0, 1, 0, 0, 0, 0, 0, 0},
    {0, 1, 0, 0, 0, 0, 0, 0, 0},      {0, 0, 0, 0, 0, 0, 0, 0, 1}};
static const int kLadermanC[9][8] = {  // product numbers (1-based), 0 terminates
    {6, 14, 19, 0},          {1, 4, 5, 6, 12, 14, 15, 0}, {6, 7, 9, 10, 14, 16, 18, 0},
    {2, 3, 4, 6, 14, 16, 17, 0}, {2, 4, 5, 6, 20, 0},     {14, 16, 17, 18, 21, 0},
    {6, 7, 8, 11, 12, 13, 14, 0}, {12, 13, 14, 15, 22, 0}, {6, 7, 8, 9, 23, 0}};

// Rank-10 approximate scheme for <3,2,2> (an APA: Y(lam) = X + O(lam), 1/lam in
// W), built as in Bini et al. 1979: a 2x2 problem with one A block missing has
// an approximate rank-5 formula; two copies cover the 3x2 A and share C's middle
// row.  Local formula on a11, a12, a21 (a22 missing), B full, five terms of the
// form sign * (A part) (B part) (C part), each part "unit + lam * pert":
struct ApaPart {
  int unit[2][2];  // (row, col) entries with coefficient 1, row < 0: unused
  int pert[2];     // the entry with coefficient lam, row < 0: none
};
struct ApaTerm {
  int sign;
  ApaPart a, b, c;  // c entries are output blocks (row, col) of the local C
};
static const ApaTerm kApaLocal[5] = {
    {+1, {{{0, 1}, {-1, 0}}, {0, 0}}, {{{0, 1}, {-1, 0}}, {1, 1}}, {{{0, 1}, {-1, 0}}, {-1, 0}}},
    {+1, {{{1, 0}, {-1, 0}}, {0, 0}}, {{{0, 0}, {-1, 0}}, {-1, 0}}, {{{0, 0}, {-1, 0}}, {1, 0}}},
    {-1, {{{0, 1}, {-1, 0}}, {-1, 0}}, {{{0, 1}, {-1, 0}}, {-1, 0}}, {{{0, 0}, {0, 1}}, {1, 1}}},
    {-1, {{{1, 0}, {-1, 0}}, {-1, 0}}, {{{0, 0}, {0, 1}}, {1, 0}}, {{{0, 0}, {-1, 0}}, {-1, 0}}},
    {+1, {{{0, 1}, {1, 0}}, {-1, 0}}, {{{0, 1}, {-1, 0}}, {1, 0}}, {{{0, 0}, {-1, 0}}, {1, 1}}},
};
// Copy c maps local A/C row i to global row kApaRow[c][i] and local A column
// (= B row) j to global kApaCol[c][j]; B and C columns are unchanged.
static const int kApaRow[2][2] = {{0, 1}, {2, 1}};
static const int kApaCol[2][2] = {{0, 1}, {1, 0}};

static void apa322(double lam, std::vector<double>& U, std::vector<double>& V, std::vector<double>& W) {
  const int R = 10;
  U.assign(6 * R, 0), V.assign(4 * R, 0), W.assign(6 * R, 0);
  for (int c = 0; c < 2; ++c)
    for (int t = 0; t < 5; ++t) {
      const ApaTerm& T = kApaLocal[t];
      const int r = 5 * c + t;
      const int* rows = kApaRow[c];
      const int* cols = kApaCol[c];
      for (int e = 0; e < 2; ++e) {
        if (T.a.unit[e][0] >= 0) U[(rows[T.a.unit[e][0]] * 2 + cols[T.a.unit[e][1]]) * R + r] += 1;
        if (T.b.unit[e][0] >= 0) V[(cols[T.b.unit[e][0]] * 2 + T.b.unit[e][1]) * R + r] += 1;
        if (T.c.unit[e][0] >= 0) W[(rows[T.c.unit[e][0]] * 2 + T.c.unit[e][1]) * R + r] += T.sign / lam;
      }
      if (T.a.pert[0] >= 0) U[(rows[T.a.pert[0]] * 2 + cols[T.a.pert[1]]) * R + r] += lam;
      if (T.b.pert[0] >= 0) V[(cols[T.b.pert[0]] * 2 + T.b.pert[1]) * R + r] += lam;
      if (T.c.pert[0] >= 0) W[(rows[T.c.pert[0]] * 2 + T.c.pert[1]) * R + r] += T.sign;  // lam / lam
    }
}

// Cyclic rotation <b1,b2,b3> -> <b2,b3,b1>: the Brent equations are invariant
// under A -> B, B -> C^T, C -> A^T, so U' = V, V'(k,i) = W(i,k), W'(j,i) = U(i,j).
static void rotate_scheme(int& b1, int& b2, int& b3, int R, std::vector<double>& U, std::vector<double>& V,
                          std::vector<double>& W) {
  std::vector<double> U2 = V, V2(W.size()), W2(U.size());
  for (int i = 0; i < b1; ++i)
    for (int k = 0; k < b3; ++k)
      for (int r = 0; r < R; ++r) V2[(k * b1 + i) * R + r] = W[(i * b3 + k) * R + r];
  for (int i = 0; i < b1; ++i)
    for (int j = 0; j < b2; ++j)
      for (int r = 0; r < R; ++r) W2[(j * b1 + i) * R + r] = U[(i * b2 + j) * R + r];
  const int t = b1;
  b1 = b2, b2 = b3, b3 = t;
  U.swap(U2), V.swap(V2), W.swap(W2);
}

// ---- approximate schemes of Section 3.1 (perturbed exact schemes) ----------
//
// Each of U, V, W gets i.i.d. N(0, sigma^2) noise on every entry equal to +1
// and on n_zero = 5 entries equal to 0 drawn uniformly without replacement.
// The random numbers come from Philox4x64-10 with key (aux_seed, 1) (the level
// draws use key word 1 = 0), blocks at counters (1,0,0,0), (2,0,0,0), ...,
// four words each, consumed in order:
//   tensor by tensor (U, V, W): one normal per +1 entry in row-major order;
//   then the picks: positions of the zero entries in row-major order, partial
//   Fisher-Yates: for i = 0..n_zero-1, j = i + floor(word (nz - i) / 2^64),
//   swap; the first n_zero positions are picked; then one normal per pick in
//   pick order.
// A word maps to u = (floor(word / 2^12) + 1/2) 2^-52 in (0, 1), exact in
// double; a normal takes two words, u1 then u2, and is the Box-Muller value
// sqrt(-2 ln u1) cos(2 pi u2) (Box and Muller 1958).  An entry becomes
// x + sigma z with one rounding for the product and one for the sum.
namespace {
struct AuxStream {
  uint64_t key[2], ctr[4] = {0, 0, 0, 0}, buf[4];
  int pos = 4;
  explicit AuxStream(uint64_t aux_seed) { key[0] = aux_seed, key[1] = 1; }
  uint64_t next() {
    if (pos == 4) {
      ++ctr[0];
      philox4x64_10(ctr, key, buf);
      pos = 0;
    }
    return buf[pos++];
  }
};

double open_unit(uint64_t w) { return ((double)(w >> 12) + 0.5) * 0x1p-52; }

double box_muller(AuxStream& st) {
  const double u1 = open_unit(st.next());
  const double u2 = open_unit(st.next());
  const double two_pi = 6.283185307179586;  // 2 pi rounded to double
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(two_pi * u2);
}

void perturb_tensor(std::vector<double>& T, double sigma, int n_zero, AuxStream& st) {
#pragma STDC FP_CONTRACT OFF
  std::vector<size_t> zeros;
  for (size_t i = 0; i < T.size(); ++i)
    if (T[i] == 0.0) zeros.push_back(i);
  for (size_t i = 0; i < T.size(); ++i)
    if (T[i] == 1.0) {
      const double noise = sigma * box_muller(st);
      T[i] = T[i] + noise;
    }
  const size_t nz = zeros.size(), picks = (size_t)n_zero < nz ? (size_t)n_zero : nz;
  for (size_t i = 0; i < picks; ++i) {
    const unsigned __int128 p = (unsigned __int128)st.next() * (uint64_t)(nz - i);
    const size_t j = i + (size_t)(uint64_t)(p >> 64);
    const size_t t = zeros[i];
    zeros[i] = zeros[j];
    zeros[j] = t;
  }
  for (size_t i = 0; i < picks; ++i) {
    const double noise = sigma * box_muller(st);
    T[zeros[i]] = T[zeros[i]] + noise;
  }
}
}  // namespace

rbc_status builtin_scheme(const char* name, double lambda, uint64_t aux_seed, Scheme& out) {
  if (!name) return fail(RBC_EINVAL, "null scheme name");
  if (!std::strncmp(name, "perturbed_", 10)) {
    if (std::strcmp(name + 10, "strassen") && std::strcmp(name + 10, "laderman"))
      return fail(RBC_EINVAL, "unknown builtin scheme '%s' (perturbed_strassen, perturbed_laderman)", name);
    if (!(lambda >= 0.0) || !(lambda <= 1.0))
      return fail(RBC_EINVAL, "%s: sigma = %g outside [0, 1]", name, lambda);
    Scheme base;
    rbc_status st = builtin_scheme(name + 10, 0.0, 0, base);
    if (st != RBC_OK) return st;
    AuxStream rng(aux_seed);
    perturb_tensor(base.U, lambda, 5, rng);
    perturb_tensor(base.V, lambda, 5, rng);
    perturb_tensor(base.W, lambda, 5, rng);
    return make_scheme(base.b1, base.b2, base.b3, base.R, base.U.data(), base.V.data(), base.W.data(),
                       INFINITY, out);
  }
  const bool apa = !std::strcmp(name, "apa322") || !std::strcmp(name, "apa223") || !std::strcmp(name, "apa232");
  if (apa) {
    if (!(lambda > 0.0) || !(lambda <= 1.0))
      return fail(RBC_EINVAL, "%s: lambda = %g outside (0, 1]", name, lambda);
  } else if (lambda != 0.0 || aux_seed != 0) {
    return fail(RBC_EINVAL, "exact scheme '%s' takes lambda = 0 and aux_seed = 0", name);
  }
  std::vector<double> U, V, W;
  int b1, b2, b3, R;
  if (!std::strcmp(name, "strassen")) {
    b1 = b2 = b3 = 2, R = 7;
    U.assign(4 * R, 0), V.assign(4 * R, 0), W.assign(4 * R, 0);
    for (int r = 0; r < R; ++r)
      for (int e = 0; e < 4; ++e) {
        U[e * R + r] = kStrassenA[r][e];
        V[e * R + r] = kStrassenB[r][e];
        W[e * R + r] = kStrassenC[r][e];
      }
  } else if (!std::strcmp(name, "laderman")) {
    b1 = b2 = b3 = 3, R = 23;
    U.assign(9 * R, 0), V.assign(9 * R, 0), W.assign(9 * R, 0);
    for (int r = 0; r < R; ++r)
      for (int e = 0; e < 9; ++e) {
        U[e * R + r] = kLadermanA[r][e];
        V[e * R + r] = kLadermanB[r][e];
      }
    for (int e = 0; e < 9; ++e)
      for (int t = 0; kLadermanC[e][t]; ++t) W[e * R + kLadermanC[e][t] - 1] = 1;
  } else if (!std::strncmp(name, "naive:", 6)) {
    if (std::sscanf(name + 6, "%d,%d,%d", &b1, &b2, &b3) != 3)
      return fail(RBC_EINVAL, "expected naive:b1,b2,b3, got '%s'", name);
    if (b1 < 1 || b2 < 1 || b3 < 1 || b1 > kMaxB || b2 > kMaxB || b3 > kMaxB || b1 * b2 * b3 > kMaxR)
      return fail(RBC_EINVAL, "naive scheme <%d,%d,%d> out of range", b1, b2, b3);
    R = b1 * b2 * b3;
    U.assign(b1 * b2 * R, 0), V.assign(b2 * b3 * R, 0), W.assign(b1 * b3 * R, 0);
    for (int i = 0; i < b1; ++i)
      for (int l = 0; l < b2; ++l)
        for (int j = 0; j < b3; ++j) {
          const int r = (i * b2 + l) * b3 + j;
          U[(i * b2 + l) * R + r] = 1;
          V[(l * b3 + j) * R + r] = 1;
          W[(i * b3 + j) * R + r] = 1;
        }
  } else if (apa) {
    b1 = 3, b2 = 2, b3 = 2, R = 10;
    apa322(lambda, U, V, W);
    const int turns = name[3] == '3' ? 0 : (name[5] == '3' ? 1 : 2);  // 322, 223, 232
    for (int t = 0; t < turns; ++t) rotate_scheme(b1, b2, b3, R, U, V, W);
    return make_scheme(b1, b2, b3, R, U.data(), V.data(), W.data(), INFINITY, out);
  } else {
    return fail(RBC_EINVAL, "unknown builtin scheme '%s'", name);
  }
  return make_scheme(b1, b2, b3, R, U.data(), V.data(), W.data(), 0.0, out);
}

}  // namespace rbc
