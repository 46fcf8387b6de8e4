/*
 * CPU oracle for the negacyclic NTT path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct reference for what the GPU library computes.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no source with the GPU library: every routine
 * here is written from the mathematics of the paper (arXiv 2109.14704, section
 * II-A "Basics of CKKS" and section II-B "Number Theoretic Transform and Residue
 * Number System") and of the radix-2 algorithms the paper cites there
 * (Longa-Naehrig), with exact unsigned 128-bit products and the C `%` operator.
 * No lazy reduction, no precomputed quotients, no blocking or fusion.
 *
 * Conventions (the paper is silent on them; these are the readings used):
 *   - psi is the smallest primitive 2N-th root of unity modulo q;
 *   - the forward transform writes its output in bit-reversed order:
 *       NTT(a)[k] = sum_i a_i * psi^(i*(2*brv(k)+1))  mod q,
 *     i.e. the paper's NTT of the psi-twisted vector (section II-B);
 *   - the inverse transform undoes it exactly, including N^-1 and the
 *     psi^-i untwist:  INTT(A)[i] = N^-1 * sum_k A_k * psi^(-i*(2*brv(k)+1));
 *   - every output is the canonical residue in [0, q).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* ---- scalar modular arithmetic ------------------------------------------ */

uint64_t or_mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
uint64_t or_addmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + b) % q); }
uint64_t or_submod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + q - (b % q)) % q); }

uint64_t or_powmod(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q, b = a % q;
  while (e) {
    if (e & 1) r = or_mulmod(r, b, q);
    b = or_mulmod(b, b, q);
    e >>= 1;
  }
  return r;
}

/* Inverse modulo a prime by Fermat's little theorem: a^(q-2). */
uint64_t or_invmod(uint64_t a, uint64_t q) { return or_powmod(a, q - 2, q); }

/* Deterministic Miller-Rabin: the first twelve primes as bases are exact for
 * every n < 3.3e24, hence for every 64-bit n. */
int or_is_prime(uint64_t n) {
  static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; ++i) {
    if (n == bases[i]) return 1;
    if (n % bases[i] == 0) return 0;
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (int i = 0; i < 12; ++i) {
    uint64_t x = or_powmod(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int witness = 1;
    for (int r = 1; r < s; ++r) {
      x = or_mulmod(x, x, n);
      if (x == n - 1) { witness = 0; break; }
    }
    if (witness) return 0;
  }
  return 1;
}

/* Largest primes below 2^bits that are 1 mod M, stepping down by M.
 * Skips any value already present in out[0..have).  Returns how many were
 * written (count unless the search space runs out). */
int or_gen_primes(uint32_t bits, uint64_t M, uint32_t count, uint64_t *out, uint32_t have) {
  uint64_t top = (bits >= 64) ? UINT64_MAX : ((uint64_t)1 << bits) - 1;
  uint64_t q = top - (top % M) + 1;           /* largest value <= top+1 that is 1 mod M */
  if (q > top) q -= M;
  uint32_t got = 0;
  while (got < count && q > M) {
    if (or_is_prime(q)) {
      int dup = 0;
      for (uint32_t i = 0; i < have + got; ++i) if (out[i] == q) dup = 1;
      if (!dup) out[have + got++] = q;
    }
    q -= M;
  }
  return (int)got;
}

uint32_t or_bitrev(uint32_t x, uint32_t bits) {
  uint32_t r = 0;
  for (uint32_t i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

/* Smallest primitive 2N-th root of unity mod prime q (requires q = 1 mod 2N).
 * A generator candidate c = x^((q-1)/2N) has order exactly 2N iff c^N = -1,
 * since 2N is a power of two.  The primitive 2N-th roots are then the odd
 * powers of c; the smallest of them is returned.  Returns 0 on failure. */
uint64_t or_psi(uint64_t q, uint32_t log_n) {
  uint64_t N = (uint64_t)1 << log_n, twoN = 2 * N;
  if ((q - 1) % twoN != 0) return 0;
  uint64_t c = 0;
  for (uint64_t x = 2; x < q && x < 100000; ++x) {
    uint64_t cand = or_powmod(x, (q - 1) / twoN, q);
    if (or_powmod(cand, N, q) == q - 1) { c = cand; break; }
  }
  if (!c) return 0;
  uint64_t best = c, c2 = or_mulmod(c, c, q), cur = c;
  for (uint64_t j = 3; j < twoN; j += 2) {
    cur = or_mulmod(cur, c2, q);
    if (cur < best) best = cur;
  }
  return best;
}

/* Twiddle tables in the order the radix-2 algorithms consume them:
 * psi_rev[k] = psi^brv(k), inv_psi_rev[k] = psi^-brv(k). */
void or_psi_tables(uint64_t q, uint32_t log_n, uint64_t psi, uint64_t *psi_rev, uint64_t *inv_psi_rev) {
  uint32_t N = 1u << log_n;
  uint64_t psi_inv = or_invmod(psi, q);
  for (uint32_t k = 0; k < N; ++k) {
    uint32_t e = or_bitrev(k, log_n);
    if (psi_rev) psi_rev[k] = or_powmod(psi, e, q);
    if (inv_psi_rev) inv_psi_rev[k] = or_powmod(psi_inv, e, q);
  }
}

/* ---- transforms by their definitions: O(N^2) --------------------------- */

/* Section II-B: NTT of the psi-twisted vector, output in bit-reversed order. */
void or_dft_fwd(const uint64_t *a, uint64_t *out, uint32_t log_n, uint64_t q, uint64_t psi) {
  uint32_t N = 1u << log_n;
  for (uint32_t k = 0; k < N; ++k) {
    uint64_t root = or_powmod(psi, 2 * (uint64_t)or_bitrev(k, log_n) + 1, q);
    uint64_t acc = 0, pw = 1;                      /* pw = root^i */
    for (uint32_t i = 0; i < N; ++i) {
      acc = or_addmod(acc, or_mulmod(a[i] % q, pw, q), q);
      pw = or_mulmod(pw, root, q);
    }
    out[k] = acc;
  }
}

/* Section II-B: inverse NTT followed by the psi^-i untwist, with N^-1. */
void or_dft_inv(const uint64_t *A, uint64_t *out, uint32_t log_n, uint64_t q, uint64_t psi) {
  uint32_t N = 1u << log_n;
  uint64_t psi_inv = or_invmod(psi, q), n_inv = or_invmod(N % q, q);
  for (uint32_t i = 0; i < N; ++i) {
    uint64_t acc = 0;
    for (uint32_t k = 0; k < N; ++k) {
      uint64_t e = (uint64_t)i * (2 * (uint64_t)or_bitrev(k, log_n) + 1) % (2 * (uint64_t)N);
      acc = or_addmod(acc, or_mulmod(A[k] % q, or_powmod(psi_inv, e, q), q), q);
    }
    out[i] = or_mulmod(acc, n_inv, q);
  }
}

/* One output of the forward definition, O(N): used to spot-check full-size runs. */
uint64_t or_ntt_fwd_point(const uint64_t *a, uint32_t log_n, uint64_t q, uint64_t psi, uint32_t k) {
  uint32_t N = 1u << log_n;
  uint64_t root = or_powmod(psi, 2 * (uint64_t)or_bitrev(k, log_n) + 1, q);
  uint64_t acc = 0, pw = 1;
  for (uint32_t i = 0; i < N; ++i) {
    acc = or_addmod(acc, or_mulmod(a[i], pw, q), q);
    pw = or_mulmod(pw, root, q);
  }
  return acc;
}

/* One output of the inverse definition, O(N). */
uint64_t or_ntt_inv_point(const uint64_t *A, uint32_t log_n, uint64_t q, uint64_t psi, uint32_t i) {
  uint32_t N = 1u << log_n;
  uint64_t psi_inv = or_invmod(psi, q), n_inv = or_invmod(N % q, q);
  uint64_t base = or_powmod(psi_inv, i, q);      /* psi^-i; term k needs base^(2 brv(k) + 1) */
  uint64_t base2 = or_mulmod(base, base, q);
  uint64_t acc = 0;
  for (uint32_t k = 0; k < N; ++k) {
    uint64_t e = or_bitrev(k, log_n);
    uint64_t w = or_mulmod(or_powmod(base2, e, q), base, q);
    acc = or_addmod(acc, or_mulmod(A[k], w, q), q);
  }
  return or_mulmod(acc, n_inv, q);
}

/* Section II-A: product in Z_q[x]/(x^N+1), written out term by term. */
void or_negacyclic_schoolbook(const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t N, uint64_t q) {
  for (uint32_t k = 0; k < N; ++k) out[k] = 0;
  for (uint32_t i = 0; i < N; ++i)
    for (uint32_t j = 0; j < N; ++j) {
      uint64_t p = or_mulmod(a[i], b[j], q);
      uint32_t k = i + j;
      if (k < N) out[k] = or_addmod(out[k], p, q);
      else out[k - N] = or_submod(out[k - N], p, q);   /* x^N = -1 */
    }
}

/* One coefficient of the negacyclic product, O(N). */
uint64_t or_negacyclic_point(const uint64_t *a, const uint64_t *b, uint32_t N, uint64_t q, uint32_t k) {
  uint64_t acc = 0;
  for (uint32_t i = 0; i < N; ++i) {
    if (i <= k) acc = or_addmod(acc, or_mulmod(a[i], b[k - i], q), q);
    else acc = or_submod(acc, or_mulmod(a[i], b[N + k - i], q), q);
  }
  return acc;
}

/* ---- radix-2 transforms (Longa-Naehrig, cited in section II-B) ----------- */

/* Cooley-Tukey, natural order in, bit-reversed order out.  Stage with m groups
 * pairs element j with j+t, t = N/(2m); group i uses psi_rev[m+i]. */
void or_ntt_fwd_r2(uint64_t *a, uint32_t log_n, uint64_t q, const uint64_t *psi_rev) {
  uint32_t N = 1u << log_n;
  for (uint32_t m = 1, t = N / 2; m < N; m *= 2, t /= 2) {
    for (uint32_t i = 0; i < m; ++i) {
      uint64_t S = psi_rev[m + i];
      for (uint32_t j = 2 * i * t; j < 2 * i * t + t; ++j) {
        uint64_t U = a[j], V = or_mulmod(a[j + t], S, q);
        a[j] = or_addmod(U, V, q);
        a[j + t] = or_submod(U, V, q);
      }
    }
  }
}

/* Gentleman-Sande, bit-reversed order in, natural order out, then N^-1.
 * Stage with h = m/2 groups pairs j with j+t, t = N/m; group i uses
 * inv_psi_rev[h+i]. */
void or_ntt_inv_r2(uint64_t *a, uint32_t log_n, uint64_t q, const uint64_t *inv_psi_rev) {
  uint32_t N = 1u << log_n;
  for (uint32_t m = N, t = 1; m > 1; m /= 2, t *= 2) {
    uint32_t h = m / 2;
    for (uint32_t i = 0; i < h; ++i) {
      uint64_t S = inv_psi_rev[h + i];
      for (uint32_t j = 2 * i * t; j < 2 * i * t + t; ++j) {
        uint64_t U = a[j], V = a[j + t];
        a[j] = or_addmod(U, V, q);
        a[j + t] = or_mulmod(or_submod(U, V, q), S, q);
      }
    }
  }
  uint64_t n_inv = or_invmod(N % q, q);
  for (uint32_t j = 0; j < N; ++j) a[j] = or_mulmod(a[j], n_inv, q);
}

/* ---- batched forms over [batch][limbs][N] --------------------------------- */

/* Per-limb tables for a modulus chain; caller frees. */
typedef struct { uint64_t q, psi; uint64_t *fwd, *inv; } or_limb;

static or_limb *make_limbs(uint32_t log_n, uint32_t limbs, const uint64_t *moduli) {
  uint32_t N = 1u << log_n;
  or_limb *t = (or_limb *)calloc(limbs, sizeof(or_limb));
  for (uint32_t l = 0; l < limbs; ++l) {
    t[l].q = moduli[l];
    t[l].psi = or_psi(moduli[l], log_n);
    t[l].fwd = (uint64_t *)malloc(sizeof(uint64_t) * N);
    t[l].inv = (uint64_t *)malloc(sizeof(uint64_t) * N);
    or_psi_tables(t[l].q, log_n, t[l].psi, t[l].fwd, t[l].inv);
  }
  return t;
}
static void free_limbs(or_limb *t, uint32_t limbs) {
  for (uint32_t l = 0; l < limbs; ++l) { free(t[l].fwd); free(t[l].inv); }
  free(t);
}

static void set_threads(int threads) {
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#else
  (void)threads;
#endif
}

int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* x[batch][limbs][N] in place; dir = +1 forward, -1 inverse. Returns 0 or -1. */
int or_batch_ntt(uint64_t *x, uint32_t batch, uint32_t limbs, uint32_t log_n, const uint64_t *moduli,
                 int dir, int threads) {
  uint32_t N = 1u << log_n;
  or_limb *t = make_limbs(log_n, limbs, moduli);
  for (uint32_t l = 0; l < limbs; ++l) if (!t[l].psi) { free_limbs(t, limbs); return -1; }
  set_threads(threads);
  long total = (long)batch * limbs;
#pragma omp parallel for schedule(dynamic)
  for (long bl = 0; bl < total; ++bl) {
    uint32_t l = (uint32_t)(bl % limbs);
    uint64_t *p = x + (size_t)bl * N;
    if (dir > 0) or_ntt_fwd_r2(p, log_n, t[l].q, t[l].fwd);
    else or_ntt_inv_r2(p, log_n, t[l].q, t[l].inv);
  }
  free_limbs(t, limbs);
  return 0;
}

/* out = a (.) b mod q per limb; [batch][limbs][N]. */
void or_batch_dyadic(const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t batch, uint32_t limbs,
                     uint32_t N, const uint64_t *moduli) {
  for (size_t bl = 0; bl < (size_t)batch * limbs; ++bl) {
    uint64_t q = moduli[bl % limbs];
    for (uint32_t k = 0; k < N; ++k) out[bl * N + k] = or_mulmod(a[bl * N + k], b[bl * N + k], q);
  }
}

/* Section II-A Mul on ciphertexts already in the NTT domain:
 * c, d [batch][2][limbs][N] -> out [batch][3][limbs][N] = (c0d0, c0d1+c1d0, c1d1). */
void or_batch_tensor(const uint64_t *c, const uint64_t *d, uint64_t *out, uint32_t batch, uint32_t limbs,
                     uint32_t N, const uint64_t *moduli) {
  size_t P = (size_t)limbs * N;
  for (uint32_t b = 0; b < batch; ++b) {
    const uint64_t *c0 = c + (size_t)b * 2 * P, *c1 = c0 + P;
    const uint64_t *d0 = d + (size_t)b * 2 * P, *d1 = d0 + P;
    uint64_t *o0 = out + (size_t)b * 3 * P, *o1 = o0 + P, *o2 = o1 + P;
    for (size_t e = 0; e < P; ++e) {
      uint64_t q = moduli[e / N];
      o0[e] = or_mulmod(c0[e], d0[e], q);
      o1[e] = or_addmod(or_mulmod(c0[e], d1[e], q), or_mulmod(c1[e], d0[e], q), q);
      o2[e] = or_mulmod(c1[e], d1[e], q);
    }
  }
}

/* Coefficient-domain negacyclic products through the transforms:
 * out = INTT(NTT(a) (.) NTT(b)), [batch][limbs][N]. */
int or_batch_polymul(const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t batch, uint32_t limbs,
                     uint32_t log_n, const uint64_t *moduli, int threads) {
  uint32_t N = 1u << log_n;
  size_t n = (size_t)batch * limbs * N;
  uint64_t *ta = (uint64_t *)malloc(n * 8), *tb = (uint64_t *)malloc(n * 8);
  memcpy(ta, a, n * 8); memcpy(tb, b, n * 8);
  int rc = or_batch_ntt(ta, batch, limbs, log_n, moduli, +1, threads);
  if (!rc) rc = or_batch_ntt(tb, batch, limbs, log_n, moduli, +1, threads);
  if (!rc) {
    or_batch_dyadic(ta, tb, out, batch, limbs, N, moduli);
    rc = or_batch_ntt(out, batch, limbs, log_n, moduli, -1, threads);
  }
  free(ta); free(tb);
  return rc;
}

/* Ciphertext tensor product in the coefficient domain:
 * forward transforms of c and d, tensor, inverse transforms of the 3 outputs. */
int or_batch_ct_tensor_coeff(const uint64_t *c, const uint64_t *d, uint64_t *out, uint32_t batch,
                             uint32_t limbs, uint32_t log_n, const uint64_t *moduli, int threads) {
  uint32_t N = 1u << log_n;
  size_t P = (size_t)limbs * N, n = (size_t)batch * 2 * P;
  uint64_t *tc = (uint64_t *)malloc(n * 8), *td = (uint64_t *)malloc(n * 8);
  memcpy(tc, c, n * 8); memcpy(td, d, n * 8);
  int rc = or_batch_ntt(tc, batch * 2, limbs, log_n, moduli, +1, threads);
  if (!rc) rc = or_batch_ntt(td, batch * 2, limbs, log_n, moduli, +1, threads);
  if (!rc) {
    or_batch_tensor(tc, td, out, batch, limbs, N, moduli);
    rc = or_batch_ntt(out, batch * 3, limbs, log_n, moduli, -1, threads);
  }
  free(tc); free(td);
  return rc;
}

/* Rescale RS_{l -> l-1} (section II-A): c' = round(c q_{l-1} / q_l) mod q_{l-1}.
 * In RNS, q_l = q_{l-1} * qL with qL the last prime of the level, so with x the
 * CRT value of a coefficient's residues x_0 .. x_L (L = limbs - 1):
 *   out_i = round(x / qL) mod q_i,  i < L.
 * Steps: qL is odd, so round(x / qL) = floor((x + h) / qL) with h = (qL - 1) / 2;
 * r = (x_L + h) mod qL is (x + h) mod qL, and x + h - r is divisible by qL:
 *   out_i = (x_i + h - r) * qL^-1  mod q_i.
 * x [batch][limbs][N] -> out [batch][limbs - 1][N], coefficient domain. */
void or_batch_rescale(const uint64_t *x, uint64_t *out, uint32_t batch, uint32_t limbs, uint32_t N,
                      const uint64_t *moduli) {
  const uint32_t L = limbs - 1;
  const uint64_t qL = moduli[L], h = (qL - 1) / 2;
  for (uint32_t b = 0; b < batch; ++b)
    for (uint32_t i = 0; i < L; ++i) {
      const uint64_t q = moduli[i], inv = or_invmod(qL % q, q);
      const uint64_t *xi = x + ((size_t)b * limbs + i) * N, *xL = x + ((size_t)b * limbs + L) * N;
      uint64_t *o = out + ((size_t)b * L + i) * N;
      for (uint32_t k = 0; k < N; ++k) {
        const uint64_t r = or_addmod(xL[k], h, qL);
        const uint64_t t = or_submod(or_addmod(xi[k], h % q, q), r % q, q);
        o[k] = or_mulmod(t, inv, q);
      }
    }
}

/* Encrypted element-wise polynomial matrix product (section IV-E), NTT domain:
 * C (m x n) += A (m x k) * B (k x n), every element a ciphertext and every
 * element product the Mul tensor of section II-A, accumulated over k:
 *   C_ij = C_ij + sum_l (a0 b0, a0 b1 + a1 b0, a1 b1),  a = A_il, b = B_lj.
 * A [m][k][2][limbs][N], B [k][n][2][limbs][N], C [m][n][3][limbs][N]. */
void or_ct_matmul(const uint64_t *A, const uint64_t *B, uint64_t *C, uint32_t m, uint32_t n, uint32_t k,
                  uint32_t limbs, uint32_t N, const uint64_t *moduli) {
  const size_t P = (size_t)limbs * N;
  for (uint32_t i = 0; i < m; ++i)
    for (uint32_t j = 0; j < n; ++j) {
      uint64_t *c0 = C + ((size_t)i * n + j) * 3 * P, *c1 = c0 + P, *c2 = c1 + P;
      for (uint32_t l = 0; l < k; ++l) {
        const uint64_t *a0 = A + ((size_t)i * k + l) * 2 * P, *a1 = a0 + P;
        const uint64_t *b0 = B + ((size_t)l * n + j) * 2 * P, *b1 = b0 + P;
        for (size_t e = 0; e < P; ++e) {
          const uint64_t q = moduli[e / N];
          c0[e] = or_addmod(c0[e], or_mulmod(a0[e], b0[e], q), q);
          c1[e] = or_addmod(c1[e], or_addmod(or_mulmod(a0[e], b1[e], q), or_mulmod(a1[e], b0[e], q), q), q);
          c2[e] = or_addmod(c2[e], or_mulmod(a1[e], b1[e], q), q);
        }
      }
    }
}

/* Relinearization Relin (section II-A): c' = (c0, c1) + round(P^-1 c2 evk)
 * mod q, with the RNS digit decomposition of c2 used by the key switch:
 *   c2 evk = sum_j [c2]_{q_j} evk_j   over the extended basis q_0..q_{l-1}, P.
 * Steps, in the NTT domain in and out (l = limbs of the ciphertext, moduli
 * holds l + 1 primes, the last one P):
 *   d_j = INTT_j(c2_j), integers in [0, q_j);
 *   acc_s[t] = sum_j NTT_t(d_j mod q_t) . ksk[j][s][t]  mod q_t,  t <= l, s = 0, 1;
 *   acc_s -> round(acc_s / P) over q_0..q_{l-1} (the rescale by P);
 *   out_s = c_s + acc_s.
 * c [batch][3][l][N], ksk [l][2][l + 1][N], out [batch][2][l][N]. */
int or_relin(const uint64_t *c, const uint64_t *ksk, uint64_t *out, uint32_t batch, uint32_t l, uint32_t log_n,
             const uint64_t *moduli, int threads) {
  const uint32_t N = 1u << log_n, L1 = l + 1;
  const size_t P = (size_t)l * N, PE = (size_t)L1 * N;
  uint64_t *d = (uint64_t *)malloc((size_t)batch * P * 8);
  uint64_t *e = (uint64_t *)malloc(PE * 8);
  uint64_t *acc = (uint64_t *)calloc((size_t)batch * 2 * PE, 8);
  uint64_t *lo = (uint64_t *)malloc((size_t)batch * 2 * P * 8);
  int rc = 0;
  for (uint32_t b = 0; b < batch; ++b) memcpy(d + b * P, c + ((size_t)b * 3 + 2) * P, P * 8);
  rc = or_batch_ntt(d, batch, l, log_n, moduli, -1, threads);
  for (uint32_t b = 0; b < batch && !rc; ++b)
    for (uint32_t j = 0; j < l && !rc; ++j) {
      const uint64_t *dj = d + b * P + (size_t)j * N;
      for (uint32_t t = 0; t < L1; ++t)
        for (uint32_t k = 0; k < N; ++k) e[(size_t)t * N + k] = dj[k] % moduli[t];
      rc = or_batch_ntt(e, 1, L1, log_n, moduli, +1, threads);
      for (uint32_t s = 0; s < 2 && !rc; ++s) {
        uint64_t *a = acc + ((size_t)b * 2 + s) * PE;
        const uint64_t *key = ksk + ((size_t)j * 2 + s) * PE;
        for (size_t x = 0; x < PE; ++x) {
          const uint64_t q = moduli[x / N];
          a[x] = or_addmod(a[x], or_mulmod(e[x], key[x], q), q);
        }
      }
    }
  if (!rc) rc = or_batch_ntt(acc, batch * 2, L1, log_n, moduli, -1, threads);
  if (!rc) {
    or_batch_rescale(acc, lo, batch * 2, L1, N, moduli);
    rc = or_batch_ntt(lo, batch * 2, l, log_n, moduli, +1, threads);
  }
  for (uint32_t b = 0; b < batch && !rc; ++b)
    for (uint32_t s = 0; s < 2; ++s) {
      const uint64_t *cs = c + ((size_t)b * 3 + s) * P;
      const uint64_t *ls = lo + ((size_t)b * 2 + s) * P;
      uint64_t *o = out + ((size_t)b * 2 + s) * P;
      for (size_t x = 0; x < P; ++x) o[x] = or_addmod(cs[x], ls[x], moduli[x / N]);
    }
  free(d); free(e); free(acc); free(lo);
  return rc;
}
