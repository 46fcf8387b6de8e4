// 64-bit modular arithmetic for gfx950 built from 32-bit multiplies.
//
// gfx950 has no 64x64 multiplier; v_mad_u64_u32 (32x32+64 -> 64) and
// v_mul_hi_u32 issue at full VALU rate, so every 64-bit product below is
// spelled as 32-bit partial products the compiler maps onto those
// instructions (the paper's mul_low_high lesson, section III-A-2, restated
// for this ISA).  Moduli satisfy q < 2^60 (so 16q < 2^64).
#pragma once
#include <stdint.h>
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

// Shoup product: W*Y mod q up to one multiple of q, W' = floor(W 2^64 / q).
// Result in [0, 2q) for any Y < 2^64 (Harvey 2014, the butterfly of
// Algorithm 1 in section III-B).
__device__ __forceinline__ uint64_t shoup(uint64_t W, uint64_t Ws, uint64_t Y, uint64_t q) {
  uint64_t Q = mulhi64(Ws, Y);
  return W * Y - Q * q;
}

__device__ __forceinline__ uint64_t csub(uint64_t x, uint64_t m) { return x >= m ? x - m : x; }

// Forward (Cooley-Tukey) lazy butterfly, Algorithm 1: X, Y in [0, 4q) on
// entry and exit; X' = X + W Y, Y' = X - W Y (mod q).
__device__ __forceinline__ void ct_bfly(uint64_t& X, uint64_t& Y, uint64_t W, uint64_t Ws, uint64_t q,
                                        uint64_t q2) {
  uint64_t x = csub(X, q2);
  uint64_t T = shoup(W, Ws, Y, q);
  X = x + T;
  Y = x - T + q2;
}

// Inverse (Gentleman-Sande) lazy butterfly after Harvey: X, Y in [0, 2q) on
// entry and exit; X' = X + Y, Y' = W (X - Y) (mod q).
__device__ __forceinline__ void gs_bfly(uint64_t& X, uint64_t& Y, uint64_t W, uint64_t Ws, uint64_t q,
                                        uint64_t q2) {
  uint64_t s = X + Y;
  uint64_t d = X - Y + q2;
  X = csub(s, q2);
  Y = shoup(W, Ws, d, q);
}

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

}  // namespace hentt
