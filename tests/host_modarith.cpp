// CPU property test of the device modular arithmetic (modarith.hpp built for
// the host).  Checks the forward butterflies' contracts (the classic one in
// [0, 8q) and the library's alternating one in [0, 16q); X' = X + W Y,
// Y' = X - W Y mod q), the inverse butterfly's [0, 4q) contract, the
// quotient-estimate reduction of any 64-bit word to [0, 2q),
// the Barrett/Shoup/mad_mod products and the Montgomery reduction against
// exact 128-bit arithmetic.
#include <stdint.h>
#include <stdio.h>
#include <random>
#define HENTT_HOST_TEST 1
#include "../paper_2109_14704_amd/csrc/modarith.hpp"

typedef unsigned __int128 u128;
using namespace hentt;

static int fails = 0;
#define EXPECT(c, ...)                       \
  do {                                       \
    if (!(c)) {                              \
      if (fails++ < 10) printf(__VA_ARGS__); \
    }                                        \
  } while (0)

static uint64_t mm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }

int main(int argc, char **argv) {
  long iters = argc > 1 ? atol(argv[1]) : 200000;
  std::mt19937_64 g(2109);
  for (long it = 0; it < iters; ++it) {
    int k = 8 + (int)(g() % 53);                    // bit length 8..60
    uint64_t q = ((g() >> (64 - k)) | (1ull << (k - 1))) | 1;
    if (it % 7 == 0) q = (k == 60) ? ((1ull << 60) - 1) : ((1ull << k) - 1);
    uint64_t a = g(), b = g();
    u128 full = (u128)a * b;
    EXPECT(mulhi64(a, b) == (uint64_t)(full >> 64), "mulhi64 %llx %llx\n", (unsigned long long)a, (unsigned long long)b);
    uint64_t h, l;
    mul128(a, b, h, l);
    EXPECT(h == (uint64_t)(full >> 64) && l == (uint64_t)full, "mul128\n");
    ModQ m;
    m.q = q; m.nq = 0 - q; m.q2 = 2 * q; m.nq2 = 0 - 2 * q; m.q4 = 4 * q; m.nq4 = 0 - 4 * q;
    // Shoup product with the short quotient estimate: [0, 4q) for any Y < 2^64
    uint64_t W = (it % 11 == 0) ? (q - 1) : (it % 13 == 0 ? 0 : g() % q);
    uint64_t Ws = (uint64_t)(((u128)W << 64) / q);
    uint64_t Y = (it % 5 == 0) ? ~0ull : g();
    uint64_t T = shoup(W, Ws, Y, m.nq);
    EXPECT(T < 4 * q && T % q == mm(W, Y % q, q), "shoup q=%llx\n", (unsigned long long)q);
    uint64_t Qe = shoup_q(Ws, Y), Qx = (uint64_t)(((u128)Ws * Y) >> 64);
    EXPECT(Qe <= Qx && Qx - Qe <= 2, "quotient estimate\n");
    // forward butterfly (Algorithm 1, lazy range [0, 8q))
    uint64_t q8 = 8 * q;
    uint64_t X = (it % 3 == 0) ? q8 - 1 : g() % q8, Yb = (it % 4 == 0) ? q8 - 1 : g() % q8;
    uint64_t x1 = X, y1 = Yb;
    ct_bfly(x1, y1, W, Ws, m);
    uint64_t wy = mm(W, Yb % q, q);
    EXPECT(x1 < q8 && y1 < q8, "ct range\n");
    EXPECT(x1 % q == (X % q + wy) % q && y1 % q == (X % q + q - wy) % q, "ct value\n");
    // the library's forward butterfly, lazy range [0, 16q), correcting every
    // second stage: corrected from X < 16q to outputs < 12q, uncorrected from
    // X < 12q to outputs < 16q
    uint64_t q16 = 16 * q, q12 = 12 * q, Yw = (it % 5 == 1) ? ~0ull : g();
    uint64_t Xc = (it % 3 == 1) ? q16 - 1 : g() % q16, Xu = (it % 3 == 2) ? q12 - 1 : g() % q12;
    uint64_t xc = Xc, yc = Yw, xu = Xu, yu = Yw;
    ct_bfly16<true>(xc, yc, W, Ws, m);
    ct_bfly16<false>(xu, yu, W, Ws, m);
    uint64_t wyw = mm(W, Yw % q, q);
    EXPECT(xc < q12 && yc < q12, "ct16 corrected range\n");
    EXPECT(xu < q16 && yu < q16, "ct16 uncorrected range\n");
    EXPECT(xc % q == (Xc % q + wyw) % q && yc % q == (Xc % q + q - wyw) % q, "ct16 corrected value\n");
    EXPECT(xu % q == (Xu % q + wyw) % q && yu % q == (Xu % q + q - wyw) % q, "ct16 uncorrected value\n");
    EXPECT(reduce_16q(Xc, m) == Xc % q, "reduce_16q\n");
    // quotient-estimate reduction (q > 2^33): any 64-bit x to [0, 2q), with c
    // derived from the Barrett constant as the kernels derive it
    if (k >= 34) {
      uint64_t mub = (uint64_t)(((u128)1 << (2 * k)) / q);
      uint32_t c = est_c(mub, (uint32_t)k);
      EXPECT((u128)c == (((u128)1 << (k + 31)) / q), "est_c q=%llx\n", (unsigned long long)q);
      const uint64_t xs[6] = {g(), ~0ull, Xc, q16 - 1, (g() % 16) * q, (g() % 16 + 1) * q - 1};
      for (uint64_t xe : xs) {
        uint64_t r = reduce_est(xe, m.nq, c, (uint32_t)k - 33);
        EXPECT(r < 2 * q && r % q == xe % q, "reduce_est q=%llx x=%llx\n", (unsigned long long)q,
               (unsigned long long)xe);
      }
    }
    // inverse butterfly, lazy range [0, 4q)
    uint64_t Xi = (it % 7 == 0) ? 4 * q - 1 : g() % (4 * q), Yi = (it % 6 == 0) ? 4 * q - 1 : g() % (4 * q);
    uint64_t x2 = Xi, y2 = Yi;
    gs_bfly(x2, y2, W, Ws, m);
    EXPECT(x2 < 4 * q && y2 < 4 * q, "gs range\n");
    EXPECT(x2 % q == (Xi + Yi) % q && y2 % q == mm(W, (Xi % q + q - Yi % q) % q, q), "gs value\n");
    // canonical reductions
    EXPECT(reduce_8q(X, m) == X % q && reduce_4q(Xi, m) == Xi % q, "reduce\n");
    EXPECT(csubn(X, m.nq4) == (X >= 4 * q ? X - 4 * q : X), "csubn\n");
    // Barrett products on canonical inputs
    uint32_t kk = 64 - __builtin_clzll(q);
    uint64_t mu = (uint64_t)(((u128)1 << (2 * kk)) / q);
    uint64_t u = (it % 9 == 0) ? q - 1 : g() % q, v = (it % 10 == 0) ? q - 1 : g() % q;
    uint64_t s = (it % 9 == 0) ? q - 1 : g() % q, t = (it % 10 == 0) ? q - 1 : g() % q;
    EXPECT(mulmod(u, v, q, mu, kk) == mm(u, v, q), "mulmod q=%llx\n", (unsigned long long)q);
    uint64_t want = (uint64_t)(((u128)u * v + (u128)s * t) % q);
    EXPECT(madmod(u, v, s, t, q, mu, kk) == want, "madmod q=%llx\n", (unsigned long long)q);
    // Montgomery products, R = 2^64: x R == T (mod q) and x < 2q for T < q R,
    // at the input ranges the fused product uses (one factor below 4q or 2q)
    uint64_t qinv = q;  // q^-1 mod 2^64 by Newton's iteration (3 -> 96 bits)
    for (int i = 0; i < 5; ++i) qinv *= 2 - q * qinv;
    EXPECT(q * qinv == 1, "q^-1 mod 2^64\n");
    qinv = 0 - qinv;
    uint64_t a4 = (it % 9 == 0) ? 4 * q - 1 : g() % (4 * q), b4 = (it % 10 == 0) ? 4 * q - 1 : g() % (4 * q);
    uint64_t x3 = mont_mul(a4, b4, q, qinv);
    EXPECT(x3 < 2 * q && (((u128)x3 << 64) % q) == ((u128)a4 * b4) % q, "mont_mul q=%llx\n", (unsigned long long)q);
    uint64_t c2 = (it % 11 == 0) ? 2 * q - 1 : g() % (2 * q), d2 = (it % 12 == 0) ? 2 * q - 1 : g() % (2 * q);
    uint64_t a2 = a4 % (2 * q), b2 = b4 % (2 * q);
    uint64_t x4 = mont_mad(a2, d2, c2, b2, q, qinv);
    u128 T4 = (u128)a2 * d2 + (u128)c2 * b2;
    EXPECT(x4 < 2 * q && (((u128)x4 << 64) % q) == T4 % q, "mont_mad q=%llx\n", (unsigned long long)q);
    // the key switch's products: a forward output below 16q times a key word below q
    uint64_t a16 = (it % 13 == 1) ? q16 - 1 : g() % q16, kq = (it % 14 == 1) ? q - 1 : g() % q;
    uint64_t x7 = mont_mul(a16, kq, q, qinv);
    EXPECT(x7 < 2 * q && (((u128)x7 << 64) % q) == ((u128)a16 * kq) % q, "mont_mul 16q x q\n");
    // the fused products' factors straight from a forward pass (below 16q,
    // no reduction) where the bounds allow it: one product for q < 2^56, the
    // tensor's sum of two for q < 2^55
    if (k <= 56) {
      uint64_t f1 = (it % 15 == 0) ? q16 - 1 : g() % q16, f2 = (it % 16 == 0) ? q16 - 1 : g() % q16;
      uint64_t x8 = mont_mul(f1, f2, q, qinv);
      EXPECT(x8 < 2 * q && (((u128)x8 << 64) % q) == ((u128)f1 * f2) % q, "mont_mul 16q x 16q q=%llx\n",
             (unsigned long long)q);
    }
    if (k <= 55) {
      uint64_t f1 = (it % 15 == 1) ? q16 - 1 : g() % q16, f2 = (it % 16 == 1) ? q16 - 1 : g() % q16;
      uint64_t f3 = (it % 17 == 1) ? q16 - 1 : g() % q16, f4 = (it % 18 == 1) ? q16 - 1 : g() % q16;
      uint64_t x9 = mont_mad(f1, f2, f3, f4, q, qinv);
      u128 T9 = (u128)f1 * f2 + (u128)f3 * f4;
      EXPECT(x9 < 2 * q && (((u128)x9 << 64) % q) == T9 % q, "mont_mad 16q q=%llx\n", (unsigned long long)q);
    }
    // the reduction itself at the edge T = q R - 1 and at T = 0
    uint64_t x5 = redc(q - 1, ~0ull, q, qinv), x6 = redc(0, 0, q, qinv);
    EXPECT(x5 < 2 * q && (((u128)x5 << 64) % q) == ((((u128)(q - 1)) << 64) | ~0ull) % q && x6 == 0, "redc edges\n");
  }
  printf(fails ? "FAIL %d\n" : "OK\n", fails);
  return fails ? 1 : 0;
}
