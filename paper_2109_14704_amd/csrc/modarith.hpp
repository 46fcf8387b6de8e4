// 64-bit modular arithmetic for gfx950 built from 32-bit multiplies.
//
// gfx950 has no 64x64 multiplier; v_mad_u64_u32 (32x32+64 -> 64) and
// v_mul_hi_u32 issue at full VALU rate, so every 64-bit product below is
// spelled as 32-bit partial products the compiler maps onto those
// instructions (the paper's mul_low_high lesson, section III-A-2, restated
// for this ISA).  Moduli satisfy q < 2^60 (so 16q < 2^64).
#pragma once
#include <stdint.h>

#include "records.hpp"
#ifdef HENTT_HOST_TEST
// Host build of this header for the CPU property tests of the arithmetic.
#define __device__
#define __forceinline__ inline
static inline uint32_t __umulhi(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }
#else
#include <hip/hip_runtime.h>
#endif

namespace hentt {

__device__ __forceinline__ uint32_t lo32(uint64_t x) { return (uint32_t)x; }
__device__ __forceinline__ uint32_t hi32(uint64_t x) { return (uint32_t)(x >> 32); }
__device__ __forceinline__ uint64_t mad32(uint32_t a, uint32_t b, uint64_t c) { return (uint64_t)a * b + c; }

// floor(a*b / 2^64), exact.
__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) {
  uint32_t a0 = lo32(a), a1 = hi32(a), b0 = lo32(b), b1 = hi32(b);
  uint64_t m1 = mad32(a1, b0, __umulhi(a0, b0));
  uint64_t m2 = mad32(a0, b1, lo32(m1));
  return mad32(a1, b1, hi32(m1)) + hi32(m2);
}

// Full 128-bit product a*b as (hi, lo).
__device__ __forceinline__ void mul128(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
  uint32_t a0 = lo32(a), a1 = hi32(a), b0 = lo32(b), b1 = hi32(b);
  uint64_t p00 = mad32(a0, b0, 0);
  uint64_t m1 = mad32(a1, b0, hi32(p00));
  uint64_t m2 = mad32(a0, b1, lo32(m1));
  lo = ((uint64_t)lo32(m2) << 32) | lo32(p00);
  hi = mad32(a1, b1, hi32(m1)) + hi32(m2);
}

// Quotient estimate for Shoup's product: floor(W' Y / 2^64) minus 0, 1 or 2.
// Only the three high partial products enter (a1 b1 and the high halves of
// the cross products); the low product a0 b0 and the low halves of the
// cross products, which together carry less than 3 into bit 64, are dropped.
// Three multiplies instead of four, and no carry chain.
__device__ __forceinline__ uint64_t shoup_q(uint64_t Ws, uint64_t Y) {
  const uint32_t a0 = lo32(Ws), a1 = hi32(Ws), b0 = lo32(Y), b1 = hi32(Y);
  const uint64_t s = (uint64_t)__umulhi(a1, b0) + __umulhi(a0, b1);
  return mad32(a1, b1, s);
}

// Shoup product (Harvey 2014, the butterfly of Algorithm 1 in section III-B):
// W Y mod q up to a multiple of q, W' = floor(W 2^64 / q), nq = -q mod 2^64.
// With the estimate above the result lies in [0, 4q) for any Y < 2^64
// (exact quotient: [0, 2q); each missing unit of the quotient adds q).
__device__ __forceinline__ uint64_t shoup(uint64_t W, uint64_t Ws, uint64_t Y, uint64_t nq) {
  return W * Y + shoup_q(Ws, Y) * nq;  // = W Y - Q q  (mod 2^64)
}

// x >= m ? x - m : x, given nm = -m mod 2^64 (one 64-bit add, one compare).
__device__ __forceinline__ uint64_t csubn(uint64_t x, uint64_t nm) {
  const uint64_t d = x + nm;
  return d < x ? d : x;
}
__device__ __forceinline__ uint64_t csub(uint64_t x, uint64_t m) { return x >= m ? x - m : x; }

// Forward (Cooley-Tukey) lazy butterfly, Algorithm 1 with a wider lazy range:
// X, Y in [0, 8q) on entry and exit (q < 2^60); X' = X + W Y, Y' = X - W Y
// (mod q).  X is brought below 4q, T = W Y mod q lies in [0, 4q), so X + T and
// X - T + 4q stay in [0, 8q).
__device__ __forceinline__ void ct_bfly(uint64_t &X, uint64_t &Y, uint64_t W, uint64_t Ws, const ModQ &m) {
  const uint64_t x = csubn(X, m.nq4);
  const uint64_t T = shoup(W, Ws, Y, m.nq);
  X = x + T;
  Y = (x + m.q4) - T;
}

// Forward butterfly of the library's transforms, with the correction of X
// taken every second stage: values lie in [0, 16q) (q < 2^60, so 16q < 2^64).
// CORR: X (below 16q) is first brought below 8q, and the outputs lie below
// 12q; otherwise X must already be below 12q and the outputs lie below 16q.
// A pass corrects at its even-numbered stages (the first one included), so
// two uncorrected stages never follow each other and a pass may start from
// any values below 16q.  T lies in [0, 4q) for any Y < 2^64.
template <bool CORR>
__device__ __forceinline__ void ct_bfly16(uint64_t &X, uint64_t &Y, uint64_t W, uint64_t Ws, const ModQ &m) {
  uint64_t x = X;
  if constexpr (CORR) x = csubn(X, m.nq4 + m.nq4);  // -8q mod 2^64
  const uint64_t T = shoup(W, Ws, Y, m.nq);
  X = x + T;
  Y = (x + m.q4) - T;
}

// Inverse (Gentleman-Sande) lazy butterfly after Harvey: X, Y in [0, 4q) on
// entry and exit; X' = X + Y, Y' = W (X - Y) (mod q).
__device__ __forceinline__ void gs_bfly(uint64_t &X, uint64_t &Y, uint64_t W, uint64_t Ws, const ModQ &m) {
  const uint64_t s = X + Y;
  const uint64_t d = (X + m.q4) - Y;
  X = csubn(s, m.nq4);
  Y = shoup(W, Ws, d, m.nq);
}

// Canonical reductions: from [0, 8q) and from [0, 4q) to [0, q).
__device__ __forceinline__ uint64_t reduce_8q(uint64_t x, const ModQ &m) {
  return csubn(csubn(csubn(x, m.nq4), m.nq2), m.nq);
}
__device__ __forceinline__ uint64_t reduce_4q(uint64_t x, const ModQ &m) { return csubn(csubn(x, m.nq2), m.nq); }
// From [0, 16q) (forward outputs of ct_bfly16 passes) to [0, q).
__device__ __forceinline__ uint64_t reduce_16q(uint64_t x, const ModQ &m) {
  return csubn(csubn(csubn(csubn(x, m.nq4 + m.nq4), m.nq4), m.nq2), m.nq);
}

// Any x < 2^64 to [0, 2q) by a quotient estimate, for q > 2^33 (bit length
// k >= 34), with c = floor(2^(k+31) / q) (below 2^32) and sh = k - 33:
// e = floor(hi32(x) c / 2^(k-1)) never exceeds x / q and falls short of it
// by less than 2 (the low word of x weighs less than 2^32 / q < 1/2, the
// truncation of c less than hi32(x) / 2^(k-1) < 1/2, the floor less than 1),
// so x - e q lies in [0, 2q).  One multiply-high, a shift and the 32 x 64-bit
// product e q, against a chain of conditional subtractions.
__device__ __forceinline__ uint64_t reduce_est(uint64_t x, uint64_t nq, uint32_t c, uint32_t sh) {
  const uint32_t e = __umulhi(hi32(x), c) >> sh;
  // x - e q (mod 2^64): the low product in the multiply-add's accumulator,
  // e times the high word of -q added to the high word alone
  const uint64_t r = mad32(e, lo32(nq), x);
  uint32_t t = e * hi32(nq);
#ifndef HENTT_HOST_TEST
  // kept a plain multiply and add: fused into one more 32x32+64 multiply-add
  // it costs two register moves
  asm("" : "+v"(t));
#endif
  return ((uint64_t)(hi32(r) + t) << 32) | lo32(r);
}
// c of reduce_est from the Barrett constant mu = floor(2^(2k) / q):
// floor(mu / 2^(k-31)) = floor(2^(k+31) / q).
__device__ __forceinline__ uint32_t est_c(uint64_t mu, uint32_t k) { return (uint32_t)(mu >> (k - 31)); }

// Barrett reduction of a 128-bit z < 2^(2k+1) modulo q, 2^(k-1) <= q < 2^k
// (k <= 60), with mu = floor(2^(2k) / q): quotient estimate
// floor(floor(z / 2^(k-1)) * mu / 2^(k+1)) is short by at most 3.
__device__ __forceinline__ uint64_t barrett(uint64_t zhi, uint64_t zlo, uint64_t q, uint64_t mu, uint32_t k) {
  // z1 = z >> (k-1), fits in 64 bits since z < 2^(2k+1) and k <= 60
  uint32_t sh = k - 1;
  uint64_t z1 = (zlo >> sh) | (zhi << (64 - sh));
  uint64_t ph, pl;
  mul128(z1, mu, ph, pl);
  uint32_t sh2 = k + 1;
  uint64_t q3 = (pl >> sh2) | (ph << (64 - sh2));
  uint64_t r = zlo - q3 * q;
  r = csub(r, q);
  r = csub(r, q);
  r = csub(r, q);
  return r;
}

// a * b mod q for canonical a, b.
__device__ __forceinline__ uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q, uint64_t mu, uint32_t k) {
  uint64_t h, l;
  mul128(a, b, h, l);
  return barrett(h, l, q, mu, k);
}

// (a*b + c*d) mod q with a single reduction (mad_mod, section III-A-1).
__device__ __forceinline__ uint64_t madmod(uint64_t a, uint64_t b, uint64_t c, uint64_t d, uint64_t q, uint64_t mu,
                                           uint32_t k) {
  uint64_t h1, l1, h2, l2;
  mul128(a, b, h1, l1);
  mul128(c, d, h2, l2);
  uint64_t l = l1 + l2;
  uint64_t h = h1 + h2 + (l < l1 ? 1 : 0);
  return barrett(h, l, q, mu, k);
}

// Multiply-accumulate with one reduction (mad_mod, section III-A-1):
// (a b + e) mod q and (a b + c d + e) mod q for canonical inputs.  The sums
// stay below 2 q^2 < 2^(2k+1), the Barrett bound above.
__device__ __forceinline__ uint64_t mac1mod(uint64_t a, uint64_t b, uint64_t e, uint64_t q, uint64_t mu, uint32_t k) {
  uint64_t h, l;
  mul128(a, b, h, l);
  const uint64_t s = l + e;
  return barrett(h + (s < l ? 1 : 0), s, q, mu, k);
}
__device__ __forceinline__ uint64_t mac2mod(uint64_t a, uint64_t b, uint64_t c, uint64_t d, uint64_t e, uint64_t q,
                                            uint64_t mu, uint32_t k) {
  uint64_t h1, l1, h2, l2;
  mul128(a, b, h1, l1);
  mul128(c, d, h2, l2);
  const uint64_t l = l1 + l2;
  const uint64_t h = h1 + h2 + (l < l1 ? 1 : 0);
  const uint64_t s = l + e;
  return barrett(h + (s < l ? 1 : 0), s, q, mu, k);
}

// Montgomery reduction (Montgomery 1985) with R = 2^64, for the products
// whose factor R^-1 is cancelled elsewhere (folded into the N^-1 scaling of
// the inverse transform that follows them).  For T = hi 2^64 + lo < q R and
// qinv = -q^-1 mod 2^64, m = lo qinv mod 2^64 makes T + m q a multiple of R;
// its low word is zero, with a carry out exactly when lo != 0, so
// (T + m q) / R = hi + floor(m q / 2^64) + [lo != 0], which is T R^-1 mod q
// in [0, 2q).  Two half products (a low one, a high one) and no correction
// steps, where Barrett takes a full 128-bit product, a low product, two
// variable shifts and three conditional subtractions.
__device__ __forceinline__ uint64_t redc(uint64_t hi, uint64_t lo, uint64_t q, uint64_t qinv) {
  const uint64_t m = lo * qinv;
  return hi + mulhi64(m, q) + (lo != 0 ? 1 : 0);
}
// a b R^-1 mod q in [0, 2q) for a b < q R.
__device__ __forceinline__ uint64_t mont_mul(uint64_t a, uint64_t b, uint64_t q, uint64_t qinv) {
  uint64_t h, l;
  mul128(a, b, h, l);
  return redc(h, l, q, qinv);
}
// (a b + c d) R^-1 mod q in [0, 2q) for a b + c d < q R (one reduction).
__device__ __forceinline__ uint64_t mont_mad(uint64_t a, uint64_t b, uint64_t c, uint64_t d, uint64_t q,
                                            uint64_t qinv) {
  uint64_t h1, l1, h2, l2;
  mul128(a, b, h1, l1);
  mul128(c, d, h2, l2);
  const uint64_t l = l1 + l2;
  return redc(h1 + h2 + (l < l1 ? 1 : 0), l, q, qinv);
}

}  // namespace hentt
