// Per-level random signed permutations and the fold of the coefficients.
//
// Section 2.1 draws i.i.d. Rademacher signs s_i(j) and random permutations pi_i
// with P[pi_i(j) = k] = 1/n, independently per recursion level (Section 2.1.1).
// The generator is Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC 2011): ten rounds of two 64x64->128-bit
// multiplies with the published multipliers, the key bumped by the published
// Weyl constants between rounds.
#include <cstring>

#include "core.hpp"

namespace rbc {

static inline void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  const unsigned __int128 p = (unsigned __int128)a * b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint64_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c[0], &hi0, &lo0);
    mulhilo64(M1, c[2], &hi1, &lo1);
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
    c[0] = n0, c[1] = n1, c[2] = n2, c[3] = n3;
  }
  std::memcpy(out, c, sizeof c);
}

namespace {
// Word stream of one level: blocks at counters (1, d, 0, 0), (2, d, 0, 0), ...
struct Stream {
  uint64_t key[2], ctr[4], buf[4];
  int pos = 4;
  Stream(uint64_t seed, int depth) {
    key[0] = seed, key[1] = 0;
    ctr[0] = 0, ctr[1] = (uint64_t)depth, ctr[2] = 0, ctr[3] = 0;
  }
  uint64_t next() {
    if (pos == 4) {
      ++ctr[0];
      philox4x64_10(ctr, key, buf);
      pos = 0;
    }
    return buf[pos++];
  }
};
}  // namespace

void draw_level(uint64_t seed, int depth, int b1, int b2, int b3, rbc_mode mode, int32_t* signs,
                int32_t* perms) {
  Stream st(seed, depth);
  const int b[3] = {b1, b2, b3};
  int o = 0;
  for (int t = 0; t < 3; ++t)
    for (int j = 0; j < b[t]; ++j) signs[o++] = (st.next() >> 63) ? -1 : 1;
  o = 0;
  for (int t = 0; t < 3; ++t) {
    int32_t* p = perms + o;
    for (int j = 0; j < b[t]; ++j) p[j] = j;
    for (int i = b[t] - 1; i >= 1; --i) {
      uint64_t hi, lo;
      mulhilo64(st.next(), (uint64_t)(i + 1), &hi, &lo);
      const int j = (int)hi;
      const int32_t tmp = p[i];
      p[i] = p[j];
      p[j] = tmp;
    }
    o += b[t];
  }
  const int n = b1 + b2 + b3;
  if (mode == RBC_MODE_PERMS || mode == RBC_MODE_NONE)
    for (int j = 0; j < n; ++j) signs[j] = 1;
  if (mode == RBC_MODE_SIGNS || mode == RBC_MODE_NONE) {
    o = 0;
    for (int t = 0; t < 3; ++t) {
      for (int j = 0; j < b[t]; ++j) perms[o + j] = j;
      o += b[t];
    }
  }
}

bool valid_draw(int b1, int b2, int b3, const int32_t* signs, const int32_t* perms) {
  const int b[3] = {b1, b2, b3};
  int o = 0;
  for (int t = 0; t < 3; ++t) {
    int seen = 0;
    for (int j = 0; j < b[t]; ++j) {
      if (signs[o + j] != 1 && signs[o + j] != -1) return false;
      const int v = perms[o + j];
      if (v < 0 || v >= b[t] || (seen >> v & 1)) return false;
      seen |= 1 << v;
    }
    o += b[t];
  }
  return true;
}

double kappa_factor(const Scheme& s) { return 1.0 / (1.0 - s.kappa); }

void fold(const Scheme& s, const int32_t* signs, const int32_t* perms, bool kappa_scale, double* Uh,
          double* Vh, double* Wh) {
  const int b1 = s.b1, b2 = s.b2, b3 = s.b3, R = s.R;
  const int32_t *s1 = signs, *s2 = signs + b1, *s3 = signs + b1 + b2;
  const int32_t *p1 = perms, *p2 = perms + b1, *p3 = perms + b1 + b2;
  const double c = kappa_scale ? kappa_factor(s) : 1.0;
  for (int k = 0; k < b1; ++k)
    for (int l = 0; l < b2; ++l)
      for (int r = 0; r < R; ++r)
        Uh[(k * b2 + l) * R + r] = s.U[(p1[k] * b2 + p2[l]) * R + r] * (double)(s1[k] * s2[l]);
  for (int k = 0; k < b2; ++k)
    for (int l = 0; l < b3; ++l)
      for (int r = 0; r < R; ++r)
        Vh[(k * b3 + l) * R + r] = s.V[(p2[k] * b3 + p3[l]) * R + r] * (double)(s2[k] * s3[l]);
  for (int i = 0; i < b1; ++i)
    for (int j = 0; j < b3; ++j)
      for (int r = 0; r < R; ++r)
        Wh[(i * b3 + j) * R + r] = (c * (double)(s1[i] * s3[j])) * s.W[(p1[i] * b3 + p3[j]) * R + r];
}

}  // namespace rbc
