// Relinearization (Relin of section II-A) with the RNS digit key switch:
//   c' = (c0, c1) + round(P^-1 sum_j [c2]_{q_j} evk_j)  mod q,
// over the ciphertext primes q_0 .. q_{l-1} extended by a special prime P.
// The digits d_j = INTT_j(c2_j) are integers in [0, q_j).  For every target
// prime q_t (t <= l) each digit is reduced modulo q_t and forward-transformed
// (the reduction fused into the transform's first load), and the products
// with the key-switching key are accumulated in registers over the digits
// (fused into the transform's last stage):
//   acc_s[t] = sum_j NTT_t(d_j mod q_t) . ksk[j][s][t]   (s = 0, 1).
// The products are Montgomery products (R = 2^64) on the lazy transform
// outputs, summed lazily below 2 q_t; one Shoup product by R mod q_t per
// output word removes the common factor R^-1 before the store.  The same
// epilogue adds P c_s (s = 0, 1) for t < l: round((x + P c_s) / P) =
// c_s + round(x / P) exactly (x and x + P c_s agree mod P), so the rescale
// of rescale_kernels.hpp that divides by P with rounding also completes
// c' = (c0, c1) + round(P^-1 c2 evk).
#pragma once
#include "ntt_kernels.hpp"

namespace hentt {

struct KsLimb {     // per target prime q_t of one level
  uint64_t mu;      // floor(2^64 / q_t)
  uint64_t qinv;    // -q_t^-1 mod 2^64
  uint64_t r, rs;   // 2^64 mod q_t and its Shoup quotient
  uint64_t pm, pms; // P mod q_t and its Shoup quotient (t < l)
};

struct KsArgs {
  const uint64_t *d;    // [batch][l][N] digits, coefficient domain, canonical mod q_j
  const uint64_t *ksk;  // [l][2][l + 1][N] NTT domain
  uint64_t *e;          // [batch][l][l + 1][N] column-pass scratch (two-pass sizes)
  uint64_t *acc;        // [batch][2][l + 1][N]
  const uint64_t *c;    // [batch][3][l][N] NTT domain: (c0, c1) enter as P c_s
  const KsLimb *kc;     // [l + 1]
  uint32_t batch, l;
};

// A digit word x < q_j < 2^60 reduced modulo q_t into [0, 2 q_t) (the
// estimate floor(x mu / 2^64) of x / q_t is short by at most one): a valid
// lazy input of the forward transform.
__device__ __forceinline__ uint64_t ks_lift(uint64_t x, uint64_t mu, uint64_t q) { return x - mulhi64(x, mu) * q; }

// acc0 += v . key0 R^-1, acc1 += v . key1 R^-1 (mod q, accumulators kept
// in [0, 2q)) for the words of v (lazy forward outputs below 16q, so that
// v . key < 16 q^2 < q R) held in the (0, E) map of a 2^B block; key0 at k,
// key1 one prime-row further (`row` blocks of 2^B words).  The two products
// run one after the other (scheduling barrier) so that only one key array is
// live.
template <int B, int E>
__device__ __forceinline__ void ks_mac(const uint64_t (&v)[1 << E], const uint64_t *k, uint32_t row, uint32_t lp,
                                       uint64_t (&acc0)[1 << E], uint64_t (&acc1)[1 << E], const ModQ &m,
                                       uint64_t qinv) {
  uint64_t kv[1 << E];
  load_global<B, E, 0, E>(kv, k, lp);
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) acc0[s] = csubn(acc0[s] + mont_mul(v[s], kv[s], m.q, qinv), m.nq2);
  __builtin_amdgcn_sched_barrier(0);
  load_global<B, E, 0, E>(kv, k + ((uint64_t)row << B), lp);
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) acc1[s] = csubn(acc1[s] + mont_mul(v[s], kv[s], m.q, qinv), m.nq2);
}

// Accumulators (sums of Montgomery products, [0, 2q)) to canonical values:
// times R mod q by a Shoup product, plus P c_s when cs (c_s's words of the
// block, in the (0, E) map) is given; each Shoup product lies in [0, 4q).
template <int B, int E>
__device__ __forceinline__ void ks_finish(uint64_t (&acc)[1 << E], const KsLimb &kc, const ModQ &m,
                                          const uint64_t *cs, uint32_t lp) {
  if (cs) {
    uint64_t cv[1 << E];
    load_global<B, E, 0, E>(cv, cs, lp);
#pragma unroll
    for (int s = 0; s < (1 << E); ++s)
      acc[s] = reduce_8q(shoup(kc.r, kc.rs, acc[s], m.nq) + shoup(kc.pm, kc.pms, cv[s], m.nq), m);
  } else {
#pragma unroll
    for (int s = 0; s < (1 << E); ++s) acc[s] = reduce_4q(shoup(kc.r, kc.rs, acc[s], m.nq), m);
  }
}

// c_s's words (s = 0, 1) at block offset `off` of target prime t for batch
// entry b, or null for the special prime (t = l).
__device__ __forceinline__ const uint64_t *ks_cs(const KsArgs &a, uint32_t b, uint32_t s, uint32_t t, int logn,
                                                 uint32_t off) {
  return t < a.l ? a.c + ((((uint64_t)b * 3 + s) * a.l + t) << logn) + off : nullptr;
}

// Whole transforms (N <= 2^12, 256 lanes): one workgroup per (batch entry,
// target prime), looping over the digits.
template <int LOGN, int E>
__global__ __launch_bounds__(1 << (LOGN - E)) void k_ks_whole(KsArgs a, const Tw *__restrict__ tw,
                                                               const LimbConst *__restrict__ lc) {
  __shared__ uint64_t lds[LdsSize<LOGN>::value];
  const uint32_t L1 = a.l + 1;
  const uint32_t t = blockIdx.x / a.batch, b = blockIdx.x % a.batch;
  const LimbConst c = lc[t];
  const KsLimb kc = a.kc[t];
  const Tw *tt = tw + (size_t)t * 2 * (1u << LOGN);
  const uint32_t tid = threadIdx.x;
  using F = FwdFirst<LOGN, E>;
  using M0 = RoundMap<LOGN, E, 0, E>;
  uint64_t acc0[1 << E], acc1[1 << E];
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) acc0[s] = acc1[s] = 0;
#pragma unroll 1
  for (uint32_t j = 0; j < a.l; ++j) {
    if (j > 0) __syncthreads();  // the previous digit's last LDS reads are done
    uint64_t v[1 << E];
    load_global<LOGN, E, F::LO, F::R>(v, a.d + (((uint64_t)b * a.l + j) << LOGN),
                                       RoundMap<LOGN, E, F::LO, F::R>::lane_part(tid));
#pragma unroll
    for (int s = 0; s < (1 << E); ++s) v[s] = ks_lift(v[s], kc.mu, c.m.q);
    // an opaque copy of the table pointer per digit: the twiddles (the same
    // for every digit) are re-read from cache instead of held in VGPRs
    fwd_block_rounds<LOGN, E, F::LO, F::R>(v, LOGN, lds, tid, 0, opaque(tt), c.m);
    ks_mac<LOGN, E>(v, a.ksk + (((uint64_t)j * 2 * L1 + t) << LOGN), L1, M0::lane_part(tid), acc0, acc1, c.m,
                    kc.qinv);
  }
  ks_finish<LOGN, E>(acc0, kc, c.m, ks_cs(a, b, 0, t, LOGN, 0), M0::lane_part(tid));
  store_global_m0<LOGN, E>(acc0, a.acc + (((uint64_t)b * 2 * L1 + t) << LOGN), lds, tid);
  ks_finish<LOGN, E>(acc1, kc, c.m, ks_cs(a, b, 1, t, LOGN, 0), M0::lane_part(tid));
  store_global_m0<LOGN, E>(acc1, a.acc + (((uint64_t)(b * 2 + 1) * L1 + t) << LOGN), lds, tid);
}

// Two-pass sizes, pass 1: column pass of digit j modulo q_t into e.
template <int LOGN, int EC>
__global__ __launch_bounds__(256) void k_ks_cols(KsArgs a, const Tw *__restrict__ tw,
                                                 const LimbConst *__restrict__ lc) {
  constexpr uint32_t tiles = (1u << (LOGN - EC)) / 256;
  constexpr int LO = LOGN - EC;
  const uint32_t L1 = a.l + 1;
  uint32_t r = blockIdx.x / tiles;
  const uint32_t col = (blockIdx.x % tiles) * 256 + threadIdx.x;
  const uint32_t t = r % L1;
  r /= L1;
  const uint32_t j = r % a.l, b = r / a.l;
  const ModQ m = lc[t].m;
  const uint64_t mu = a.kc[t].mu;
  uint64_t v[1 << EC];
  load_global<LOGN, EC, LO, EC, true>(v, a.d + (((uint64_t)b * a.l + j) << LOGN), col);
#pragma unroll
  for (int s = 0; s < (1 << EC); ++s) v[s] = ks_lift(v[s], mu, m.q);
  fwd_round<LOGN, EC, LO, EC, 0>(v, LOGN, 0, col, tw + (size_t)t * 2 * (1u << LOGN), m);
  store_global<LOGN, EC, LO, EC, true>(v, a.e + ((((uint64_t)b * a.l + j) * L1 + t) << LOGN), col);
}

// Two-pass sizes, pass 2: per (batch entry, target prime, block), the block
// rounds of every digit, accumulated with the key in registers.
template <int LOGN, int B, int E>
__global__ __launch_bounds__(1 << (B - E)) void k_ks_blocks(KsArgs a, const Tw *__restrict__ tw,
                                                             const LimbConst *__restrict__ lc) {
  __shared__ uint64_t lds[LdsSize<B>::value];
  constexpr uint32_t tiles = 1u << (LOGN - B);
  const uint32_t L1 = a.l + 1;
  const uint32_t blockStart = (blockIdx.x % tiles) << B;
  const uint32_t r = blockIdx.x / tiles;
  const uint32_t t = r / a.batch, b = r % a.batch;
  const LimbConst c = lc[t];
  const KsLimb kc = a.kc[t];
  const Tw *tt = tw + (size_t)t * 2 * (1u << LOGN);
  const uint32_t tid = threadIdx.x;
  using F = FwdFirst<B, E>;
  using M0 = RoundMap<B, E, 0, E>;
  uint64_t acc0[1 << E], acc1[1 << E];
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) acc0[s] = acc1[s] = 0;
#pragma unroll 1
  for (uint32_t j = 0; j < a.l; ++j) {
    if (j > 0) __syncthreads();  // the previous digit's last LDS reads are done
    uint64_t v[1 << E];
    load_global<B, E, F::LO, F::R>(v, a.e + ((((uint64_t)b * a.l + j) * L1 + t) << LOGN) + blockStart,
                                   RoundMap<B, E, F::LO, F::R>::lane_part(tid));
    fwd_block_rounds<B, E, F::LO, F::R>(v, LOGN, lds, tid, blockStart, opaque(tt), c.m);
    ks_mac<B, E>(v, a.ksk + (((uint64_t)j * 2 * L1 + t) << LOGN) + blockStart, L1 << (LOGN - B),
                 M0::lane_part(tid), acc0, acc1, c.m, kc.qinv);
  }
  ks_finish<B, E>(acc0, kc, c.m, ks_cs(a, b, 0, t, LOGN, blockStart), M0::lane_part(tid));
  store_global_m0<B, E>(acc0, a.acc + (((uint64_t)b * 2 * L1 + t) << LOGN) + blockStart, lds, tid);
  ks_finish<B, E>(acc1, kc, c.m, ks_cs(a, b, 1, t, LOGN, blockStart), M0::lane_part(tid));
  store_global_m0<B, E>(acc1, a.acc + (((uint64_t)(b * 2 + 1) * L1 + t) << LOGN) + blockStart, lds, tid);
}

}  // namespace hentt
