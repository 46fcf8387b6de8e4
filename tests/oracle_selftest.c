/*
 * Self-test of the CPU oracle (oracle/oracle.c) for the sanitizer build of the
 * CPU suite: built together with oracle.c by gcc with AddressSanitizer and
 * UndefinedBehaviorSanitizer, it drives every routine of the oracle on small
 * shapes and checks the same mathematical pins as the Python suite (a
 * hand-derived example, the O(N^2) definitions, the convolution theorem, round
 * trips, the exact rounding of rescale), so that an out-of-bounds access,
 * overflow or uninitialised read anywhere in the oracle fails the build's run.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

uint64_t or_mulmod(uint64_t a, uint64_t b, uint64_t q);
uint64_t or_powmod(uint64_t a, uint64_t e, uint64_t q);
uint64_t or_invmod(uint64_t a, uint64_t q);
int or_is_prime(uint64_t n);
int or_gen_primes(uint32_t bits, uint64_t M, uint32_t count, uint64_t *out, uint32_t have);
uint32_t or_bitrev(uint32_t x, uint32_t bits);
uint64_t or_psi(uint64_t q, uint32_t log_n);
void or_psi_tables(uint64_t q, uint32_t log_n, uint64_t psi, uint64_t *psi_rev, uint64_t *inv_psi_rev);
void or_dft_fwd(const uint64_t *a, uint64_t *out, uint32_t log_n, uint64_t q, uint64_t psi);
void or_dft_inv(const uint64_t *A, uint64_t *out, uint32_t log_n, uint64_t q, uint64_t psi);
uint64_t or_ntt_fwd_point(const uint64_t *a, uint32_t log_n, uint64_t q, uint64_t psi, uint32_t k);
uint64_t or_ntt_inv_point(const uint64_t *A, uint32_t log_n, uint64_t q, uint64_t psi, uint32_t i);
void or_negacyclic_schoolbook(const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t N, uint64_t q);
uint64_t or_negacyclic_point(const uint64_t *a, const uint64_t *b, uint32_t N, uint64_t q, uint32_t k);
int or_batch_ntt(uint64_t *x, uint32_t batch, uint32_t limbs, uint32_t log_n, const uint64_t *moduli, int dir,
                 int threads);
void or_batch_dyadic(const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t batch, uint32_t limbs, uint32_t N,
                     const uint64_t *moduli);
void or_batch_tensor(const uint64_t *c, const uint64_t *d, uint64_t *out, uint32_t batch, uint32_t limbs, uint32_t N,
                     const uint64_t *moduli);
int or_batch_polymul(const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t batch, uint32_t limbs,
                     uint32_t log_n, const uint64_t *moduli, int threads);
int or_batch_ct_tensor_coeff(const uint64_t *c, const uint64_t *d, uint64_t *out, uint32_t batch, uint32_t limbs,
                             uint32_t log_n, const uint64_t *moduli, int threads);
void or_batch_rescale(const uint64_t *x, uint64_t *out, uint32_t batch, uint32_t limbs, uint32_t N,
                      const uint64_t *moduli);
void or_ct_matmul(const uint64_t *A, const uint64_t *B, uint64_t *C, uint32_t m, uint32_t n, uint32_t k,
                  uint32_t limbs, uint32_t N, const uint64_t *moduli);
int or_relin(const uint64_t *c, const uint64_t *ksk, uint64_t *out, uint32_t batch, uint32_t l, uint32_t log_n,
             const uint64_t *moduli, int threads);

static int fails = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      if (fails++ < 20) fprintf(stderr, "FAIL %s:%d %s\n", __FILE__, __LINE__, #c); \
    }                                                                 \
  } while (0)

static uint64_t rng_state = 0x2109147040ull;
static uint64_t rnd(void) {  /* splitmix64 */
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static uint64_t *fill(size_t n, const uint64_t *mods, uint32_t limbs, uint32_t N) {
  uint64_t *p = (uint64_t *)malloc(n * 8);
  for (size_t i = 0; i < n; ++i) p[i] = rnd() % mods[(i / N) % limbs];
  return p;
}

int main(void) {
  /* hand-derived example: N = 4, q = 17, psi = 2 (smallest primitive 8th root) */
  CHECK(or_psi(17, 2) == 2);
  uint64_t e1[4] = {0, 1, 0, 0}, E1[4];
  or_dft_fwd(e1, E1, 2, 17, 2);
  CHECK(E1[0] == 2 && E1[1] == 15 && E1[2] == 8 && E1[3] == 9);
  uint64_t m17 = 17, x4[4] = {0, 1, 0, 0};
  CHECK(or_batch_ntt(x4, 1, 1, 2, &m17, +1, 1) == 0);
  CHECK(memcmp(x4, E1, sizeof E1) == 0);
  CHECK(or_batch_ntt(x4, 1, 1, 2, &m17, -1, 1) == 0);
  CHECK(memcmp(x4, e1, sizeof e1) == 0);
  /* primality and prime search */
  CHECK(or_is_prime(2) && or_is_prime(65537) && !or_is_prime(3215031751ull) && !or_is_prime(1));
  uint64_t mods[4];
  CHECK(or_gen_primes(50, 1ull << 12, 4, mods, 0) == 4);
  for (int i = 0; i < 4; ++i) CHECK(or_is_prime(mods[i]) && (mods[i] - 1) % (1ull << 12) == 0);
  /* definitions against the radix-2 algorithms, point evaluations, tables */
  const uint32_t ln = 6, N = 1u << ln;
  uint64_t psi = or_psi(mods[0], ln), fw[64], iv[64];
  or_psi_tables(mods[0], ln, psi, fw, iv);
  CHECK(fw[0] == 1 && or_mulmod(fw[1], fw[1], mods[0]) == mods[0] - 1);
  for (uint32_t k = 1; k < N; ++k) CHECK(or_mulmod(fw[k], iv[k], mods[0]) == 1);
  uint64_t *a = fill(N, mods, 1, N), D[64], R[64], back[64];
  or_dft_fwd(a, D, ln, mods[0], psi);
  memcpy(R, a, sizeof R);
  CHECK(or_batch_ntt(R, 1, 1, ln, mods, +1, 1) == 0);
  CHECK(memcmp(D, R, sizeof D) == 0);
  for (uint32_t k = 0; k < N; k += 7) CHECK(or_ntt_fwd_point(a, ln, mods[0], psi, k) == D[k]);
  or_dft_inv(D, back, ln, mods[0], psi);
  CHECK(memcmp(back, a, sizeof back) == 0);
  for (uint32_t i = 0; i < N; i += 5) CHECK(or_ntt_inv_point(D, ln, mods[0], psi, i) == a[i]);
  CHECK(or_bitrev(1, ln) == N / 2 && or_invmod(3, mods[0]) * 3 % mods[0] == 1);
  /* batched round trip, dyadic and tensor, polymul against the schoolbook */
  const uint32_t bl = 10, B = 3, L = 4, Nb = 1u << bl;
  const size_t W = (size_t)B * L * Nb;
  uint64_t *x = fill(W, mods, L, Nb), *y = (uint64_t *)malloc(W * 8), *z = fill(W, mods, L, Nb);
  memcpy(y, x, W * 8);
  CHECK(or_batch_ntt(y, B, L, bl, mods, +1, 2) == 0);
  CHECK(or_batch_ntt(y, B, L, bl, mods, -1, 2) == 0);
  CHECK(memcmp(x, y, W * 8) == 0);
  uint64_t *pm = (uint64_t *)malloc(W * 8), *sb = (uint64_t *)malloc(Nb * 8);
  CHECK(or_batch_polymul(x, z, pm, B, L, bl, mods, 2) == 0);
  for (uint32_t t = 0; t < B * L; t += 5) {
    or_negacyclic_schoolbook(x + (size_t)t * Nb, z + (size_t)t * Nb, sb, Nb, mods[t % L]);
    CHECK(memcmp(sb, pm + (size_t)t * Nb, Nb * 8) == 0);
    CHECK(or_negacyclic_point(x + (size_t)t * Nb, z + (size_t)t * Nb, Nb, mods[t % L], 17) == sb[17]);
  }
  uint64_t *dy = (uint64_t *)malloc(W * 8);
  or_batch_dyadic(x, z, dy, B, L, Nb, mods);
  CHECK(dy[5] == or_mulmod(x[5], z[5], mods[0]));
  /* ciphertext tensor: coefficient form against schoolbook products */
  const size_t Wc = (size_t)1 * 2 * L * Nb;
  uint64_t *c = fill(Wc, mods, L, Nb), *d = fill(Wc, mods, L, Nb);
  uint64_t *tc = (uint64_t *)malloc(3 * L * Nb * 8), *tn = (uint64_t *)malloc(3 * L * Nb * 8);
  CHECK(or_batch_ct_tensor_coeff(c, d, tc, 1, L, bl, mods, 1) == 0);
  or_negacyclic_schoolbook(c, d, sb, Nb, mods[0]);                      /* c0 d0, limb 0 */
  CHECK(memcmp(sb, tc, Nb * 8) == 0);
  or_batch_tensor(c, d, tn, 1, L, Nb, mods);
  CHECK(tn[3] == or_mulmod(c[3], d[3], mods[0]));
  /* rescale: exact rounded division by the last prime (two limbs) */
  uint64_t xr[2 * 4], outr[4];
  for (int i = 0; i < 4; ++i) {
    xr[i] = rnd() % mods[0];
    xr[4 + i] = rnd() % mods[1];
  }
  or_batch_rescale(xr, outr, 1, 2, 4, mods);
  for (int i = 0; i < 4; ++i) {
    /* CRT value x = x0 + q0 ((x1 - x0) q0^-1 mod q1); round(x / q1) mod q0 */
    unsigned __int128 t = (xr[4 + i] + mods[1] - xr[i] % mods[1]) % mods[1];
    t = t * or_invmod(mods[0] % mods[1], mods[1]) % mods[1];
    unsigned __int128 X = (unsigned __int128)xr[i] + (unsigned __int128)mods[0] * t;
    unsigned __int128 r = (X + (mods[1] - 1) / 2) / mods[1];
    CHECK(outr[i] == (uint64_t)(r % mods[0]));
  }
  /* matMul and relinearization: run every path (values pinned in the Python suite) */
  uint64_t *A = fill(2 * 2 * 2 * L * 64, mods, L, 64), *Bm = fill(2 * 3 * 2 * L * 64, mods, L, 64);
  uint64_t *C = fill(2 * 3 * 3 * L * 64, mods, L, 64);
  or_ct_matmul(A, Bm, C, 2, 3, 2, L, 64, mods);
  for (size_t i = 0; i < (size_t)2 * 3 * 3 * L * 64; ++i) CHECK(C[i] < mods[(i / 64) % L]);
  const uint32_t l = 3;
  uint64_t *cr = fill(2 * 3 * l * 64, mods, l, 64), *ksk = fill(l * 2 * (l + 1) * 64, mods, l + 1, 64);
  uint64_t *outl = (uint64_t *)malloc(2 * 2 * l * 64 * 8);
  CHECK(or_relin(cr, ksk, outl, 2, l, 6, mods, 1) == 0);
  for (size_t i = 0; i < (size_t)2 * 2 * l * 64; ++i) CHECK(outl[i] < mods[(i / 64) % l]);
  free(a); free(x); free(y); free(z); free(pm); free(sb); free(dy); free(c); free(d); free(tc); free(tn);
  free(A); free(Bm); free(C); free(cr); free(ksk); free(outl);
  printf(fails ? "FAIL %d\n" : "OK\n", fails);
  return fails ? 1 : 0;
}
