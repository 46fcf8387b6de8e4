// CPU test of the library's host-side number theory and table builder
// (csrc/host_tables.hpp), built by g++ with and without sanitizers:
//   - Miller-Rabin against trial division below 2^17, known primes and
//     strong pseudoprimes;
//   - the smallest primitive 2N-th root against an exhaustive search for
//     small primes;
//   - for 60-bit and 50-bit primes = 1 mod 2^18 at every N = 2^6 .. 2^17, the
//     twiddle-order invariants of the tables (psi_rev[0] = 1,
//     psi_rev[1]^2 = -1, psi_rev[2k]^2 = psi_rev[k],
//     psi_rev[2k+1] = psi_rev[2k] psi_rev[1], psi_rev[k] ipsi_rev[k] = 1), the
//     Shoup quotients W' = floor(W 2^64 / q), N N^-1 = 1, the folded
//     constants N^-1 psi^-brv(1) and N^-1 R, the Montgomery constant
//     -q^-1 mod 2^64 and the Barrett mu = floor(2^(2k) / q).
#include <stdint.h>
#include <stdio.h>
#include <vector>

#include "../paper_2109_14704_amd/csrc/host_tables.hpp"

using namespace hentt;
typedef unsigned __int128 u128;

static int fails = 0;
#define CHECK(c)                                                                        \
  do {                                                                                  \
    if (!(c)) {                                                                         \
      if (fails++ < 20) fprintf(stderr, "FAIL %s:%d %s\n", __FILE__, __LINE__, #c);    \
    }                                                                                   \
  } while (0)

static bool trial(uint64_t n) {
  if (n < 2) return false;
  for (uint64_t d = 2; d * d <= n; ++d)
    if (n % d == 0) return false;
  return true;
}

int main() {
  for (uint64_t n = 0; n < (1u << 17); ++n) CHECK(host::is_prime(n) == trial(n));
  const uint64_t pseudo[] = {2047ull, 3215031751ull, 341550071728321ull, 3825123056546413051ull};
  for (uint64_t n : pseudo) CHECK(!host::is_prime(n));
  CHECK(host::is_prime((1ull << 61) - 1) && host::is_prime(18446744073709551557ull));
  // smallest primitive 2N-th roots by exhaustive search
  const uint64_t smallq[] = {17, 97, 193, 257, 641, 7681, 12289};
  for (uint64_t q : smallq)
    for (int ln = 1; (2ull << ln) <= q - 1; ++ln) {
      if ((q - 1) % (2ull << ln)) continue;
      uint64_t best = 0;
      for (uint64_t r = 2; r < q && !best; ++r) {
        if (host::pow(r, 1ull << ln, q) != q - 1) continue;  // order exactly 2N: r^N = -1
        best = r;
      }
      CHECK(host::psi(q, ln) == best);
    }
  // primes = 1 mod 2^18 below 2^60 and 2^50
  std::vector<uint64_t> qs;
  for (int bits : {60, 50})
    for (uint64_t q = ((1ull << bits) - 1) / (1ull << 18) * (1ull << 18) + 1; qs.size() < (bits == 60 ? 2u : 4u);
         q -= 1ull << 18)
      if (host::is_prime(q)) qs.push_back(q);
  for (uint64_t q : qs) {
    CHECK(host::modulus_ok(q, 17) && !host::modulus_ok(q + 2, 17));
    for (int ln = 6; ln <= 17; ++ln) {
      const uint32_t N = 1u << ln;
      std::vector<Tw> fw(N), iv(N);
      std::vector<uint64_t> pw(N), ipw(N);
      LimbConst c, cm;
      MontLimb mo;
      CHECK(host::make_limb(q, ln, fw.data(), iv.data(), c, cm, mo, pw.data(), ipw.data()));
      CHECK(fw[0].w == 1 && host::mul(fw[1].w, fw[1].w, q) == q - 1);
      for (uint32_t k = 1; k < N / 2; ++k) {
        CHECK(host::mul(fw[2 * k].w, fw[2 * k].w, q) == fw[k].w);
        CHECK(fw[2 * k + 1].w == host::mul(fw[2 * k].w, fw[1].w, q));
      }
      for (uint32_t k = 0; k < N; ++k) {
        CHECK(fw[k].w < q && iv[k].w < q && host::mul(fw[k].w, iv[k].w, q) == 1);
        const u128 a = (u128)fw[k].w << 64, b = (u128)fw[k].ws * q;
        CHECK(b <= a && a - b < q);
        const u128 a2 = (u128)iv[k].w << 64, b2 = (u128)iv[k].ws * q;
        CHECK(b2 <= a2 && a2 - b2 < q);
      }
      CHECK(host::mul(c.ninv, N, q) == 1 && c.ninvw == host::mul(c.ninv, iv[1].w, q));
      const uint64_t R = (uint64_t)(((u128)1 << 64) % q);
      CHECK(cm.ninv == host::mul(c.ninv, R, q) && cm.ninvw == host::mul(c.ninvw, R, q));
      CHECK(mo.qinv * q == ~0ull && mo.r == R);
      CHECK(c.m.q == q && c.m.nq == 0 - q && c.m.q4 == 4 * q && c.m.nq4 == 0 - 4 * q && c.m.nq2 == 0 - 2 * q);
      CHECK(c.k == (uint32_t)host::bit_length(q) && c.mu == (uint64_t)(((u128)1 << (2 * c.k)) / q));
    }
  }
  printf(fails ? "FAIL %d\n" : "OK\n", fails);
  return fails ? 1 : 0;
}
