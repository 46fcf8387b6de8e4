// Host-side number theory and table construction of the library (plain C++,
// no HIP): modulus checks, the smallest primitive 2N-th root of unity, and the
// per-limb twiddle tables and reduction constants that the kernels read.
// Kept free of device code so that the CPU test suite can build it with
// sanitizers and check its invariants.
#pragma once
#include <stdint.h>
#include <string.h>

#include "records.hpp"

namespace hentt {
namespace host {

typedef unsigned __int128 u128;

inline uint64_t mul(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }
inline uint64_t pow(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1;
  b %= m;
  for (; e; e >>= 1, b = mul(b, b, m))
    if (e & 1) r = mul(r, b, m);
  return r;
}

// Miller-Rabin with the witness set {2, 325, 9375, 28178, 450775, 9780504,
// 1795265022} (Jim Sinclair), deterministic for all n < 2^64.
inline bool is_prime(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t small[] = {2, 3, 5, 7, 11, 13};
  for (uint64_t p : small)
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = __builtin_ctzll(d);
  d >>= s;
  static const uint64_t wit[] = {2, 325, 9375, 28178, 450775, 9780504, 1795265022};
  for (uint64_t a : wit) {
    a %= n;
    if (a == 0) continue;
    uint64_t x = pow(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s && comp; ++r) {
      x = mul(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

// The low `bits` bits of x in reverse order.
inline uint32_t brv(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

// Smallest primitive 2N-th root of unity mod q (q prime, q = 1 mod 2N): take
// a root g of order exactly 2N (c = r^((q-1)/2N) for small bases r, accepted
// when c^N = -1), then scan its odd powers g, g^3, ... for the minimum.
// Returns 0 when no base below 10^6 gives such a root.
inline uint64_t psi(uint64_t q, int log_n) {
  const uint64_t two_n = 2ull << log_n;
  const uint64_t e = (q - 1) / two_n;
  uint64_t g = 0;
  for (uint64_t r = 2; r < 1000000 && r < q; ++r) {
    const uint64_t c = pow(r, e, q);
    if (pow(c, two_n / 2, q) == q - 1) {
      g = c;
      break;
    }
  }
  if (!g) return 0;
  const uint64_t g2 = mul(g, g, q);
  uint64_t best = g, cur = g;
  for (uint64_t j = 1; j < two_n / 2; ++j) {
    cur = mul(cur, g2, q);
    if (cur < best) best = cur;
  }
  return best;
}

inline int bit_length(uint64_t v) { return 64 - __builtin_clzll(v); }

// The library's modulus contract: prime, q = 1 mod 2N, 2^7 < q < 2^60.
inline bool modulus_ok(uint64_t q, int log_n) {
  if (q <= (1ull << 7) || q >= (1ull << 60)) return false;
  if ((q - 1) % (2ull << log_n) != 0) return false;
  return is_prime(q);
}

inline uint64_t shoup_quot(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

// q^-1 mod 2^64 for odd q (Newton's iteration: 3 -> 6 -> ... -> 96 correct bits).
inline uint64_t inv64(uint64_t q) {
  uint64_t x = q;
  for (int i = 0; i < 5; ++i) x *= 2 - q * x;
  return x;
}

// Tables and constants of one limb at N = 2^log_n:
//   fwd[k] = (psi^brv(k), quotient), inv[k] = (psi^-brv(k), quotient), k < N;
//   c: reduction constants with N^-1 and N^-1 psi^-brv(1) (plain inverse);
//   cm: the same with both scaled by R = 2^64 (inverse after Montgomery products);
//   mont: -q^-1 mod 2^64, R mod q and its quotient.
// pw and ipw are caller scratch of N words each.  Returns false if psi is not
// found (q must already satisfy modulus_ok).
inline bool make_limb(uint64_t q, int log_n, Tw *fwd, Tw *inv, LimbConst &c, LimbConst &cm, MontLimb &mont,
                      uint64_t *pw, uint64_t *ipw) {
  const uint32_t N = 1u << log_n;
  const uint64_t p = psi(q, log_n);
  if (!p) return false;
  const uint64_t p_inv = pow(p, q - 2, q);
  pw[0] = ipw[0] = 1;
  for (uint32_t i = 1; i < N; ++i) {
    pw[i] = mul(pw[i - 1], p, q);
    ipw[i] = mul(ipw[i - 1], p_inv, q);
  }
  for (uint32_t k = 0; k < N; ++k) {
    const uint32_t r = brv(k, log_n);
    fwd[k] = Tw{pw[r], shoup_quot(pw[r], q)};
    inv[k] = Tw{ipw[r], shoup_quot(ipw[r], q)};
  }
  memset(&c, 0, sizeof(c));
  c.m.q = q;
  c.m.nq = 0 - q;
  c.m.q2 = 2 * q;
  c.m.nq2 = 0 - 2 * q;
  c.m.q4 = 4 * q;
  c.m.nq4 = 0 - 4 * q;
  c.ninv = pow(N % q, q - 2, q);
  c.ninv_s = shoup_quot(c.ninv, q);
  c.ninvw = mul(c.ninv, N > 1 ? inv[1].w : 1, q);
  c.ninvw_s = shoup_quot(c.ninvw, q);
  c.k = (uint32_t)bit_length(q);
  c.mu = (uint64_t)(((u128)1 << (2 * c.k)) / q);
  const uint64_t r = (uint64_t)(((u128)1 << 64) % q);
  mont = MontLimb{0 - inv64(q), r, shoup_quot(r, q), 0};
  cm = c;
  cm.ninv = mul(c.ninv, r, q);
  cm.ninv_s = shoup_quot(cm.ninv, q);
  cm.ninvw = mul(c.ninvw, r, q);
  cm.ninvw_s = shoup_quot(cm.ninvw, q);
  return true;
}

}  // namespace host
}  // namespace hentt
