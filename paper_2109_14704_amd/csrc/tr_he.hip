// Dispatch of the homomorphic routines built on the transforms: rescale (RS),
// relinearization with the RNS digit key switch (Relin) and the encrypted
// element-wise polynomial matrix product.
#include "host_tables.hpp"
#include "keyswitch_kernels.hpp"
#include "rescale_kernels.hpp"
#include "runtime.hpp"

namespace hentt_rt {
namespace {

// ---------------------------------------------------------------- rescale
// Constants of RS from a level of `level` limbs to level - 1 (section II-A):
// per remaining limb i, floor(2^64 / q_i), q_i - (h mod q_i) with
// h = (qL - 1) / 2, and qL^-1 mod q_i with its Shoup quotient.  Made once per
// (tables, level) with a synchronous upload, like the tables themselves.
int rs_constants(Storage *s, uint32_t level, const RsLimb **out) {
  std::lock_guard<std::mutex> lk(s->rs_mu);
  auto it = s->rs.find(level);
  if (it != s->rs.end()) {
    *out = it->second;
    return HENTT_OK;
  }
  const uint32_t L = level - 1;
  const uint64_t qL = s->moduli[L], h = (qL - 1) / 2;
  std::vector<RsLimb> host(L);
  for (uint32_t i = 0; i < L; ++i) {
    const uint64_t q = s->moduli[i];
    host[i].mu = (uint64_t)(((host::u128)1 << 64) / q);
    host[i].nh = q - h % q;
    host[i].w = host::pow(qL % q, q - 2, q);
    host[i].ws = host::shoup_quot(host[i].w, q);
  }
  RsLimb *d = nullptr;
  hipError_t e = hipMalloc(&d, L * sizeof(RsLimb));
  if (e == hipSuccess) e = hipMemcpy(d, host.data(), L * sizeof(RsLimb), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (d) (void)hipFree(d);
    return hip_fail(e);
  }
  s->rs[level] = d;
  *out = d;
  return HENTT_OK;
}

// Stage split of the rescale's forward transforms: the plain transform's
// default (whole up to 2^14; 5 column stages at 2^15 and 2^16, 4 at 2^17).
template <int LOGN> struct RsPlan {
  static constexpr bool WHOLE = LOGN <= 14;
  static constexpr int EC = LOGN == 15 ? 5 : LOGN == 16 ? 5 : LOGN == 17 ? 4 : (LOGN > 12 ? LOGN - 12 : 1);
  static constexpr int B = LOGN - EC;
};

template <int LOGN> void launch_rescale_ntt(const RsArgs &a, const Storage *s, hipStream_t st) {
  const uint32_t units = a.batch * a.L;
  using P = RsPlan<LOGN>;
  if constexpr (P::WHOLE) {
    LaunchTimer lt_("k_rs_whole", LOGN, st);
    hipLaunchKernelGGL((k_rs_whole<LOGN, 4>), dim3(units), dim3(1 << (LOGN - 4)), 0, st, a, s->d_tw, s->d_lc);
  } else {
    {
      LaunchTimer lt_("k_rs_cols", LOGN, st);
      hipLaunchKernelGGL((k_rs_cols<LOGN, P::EC>), dim3(units * ((1u << (LOGN - P::EC)) / 256)), dim3(256), 0, st, a,
                         s->d_tw, s->d_lc);
    }
    LaunchTimer lt_("k_rs_blocks", LOGN, st);
    hipLaunchKernelGGL((k_rs_blocks<LOGN, P::B, 4>), dim3(units << (LOGN - P::B)), dim3(1 << (P::B - 4)), 0, st, a,
                       s->d_tw, s->d_lc);
  }
}
typedef void (*rs_fn)(const RsArgs &, const Storage *, hipStream_t);
#define RS_ENTRY(n) launch_rescale_ntt<n>,
const rs_fn k_rs_table[] = {HENTT_SIZES(RS_ENTRY)};

// ------------------------------------------------------- relinearization
// Key-switching constants of the level with L1 limbs (the last one is P).
int ks_consts(Storage *s, uint32_t L1, const KsLimb **out) {
  std::lock_guard<std::mutex> lk(s->rs_mu);
  auto it = s->ks.find(L1);
  if (it != s->ks.end()) {
    *out = it->second;
    return HENTT_OK;
  }
  const uint64_t P = s->moduli[L1 - 1];
  std::vector<KsLimb> kc(L1);
  for (uint32_t t = 0; t < L1; ++t) {
    const uint64_t q = s->moduli[t];
    kc[t].mu = (uint64_t)(((host::u128)1 << 64) / q);
    kc[t].qinv = 0 - host::inv64(q);
    kc[t].r = (uint64_t)(((host::u128)1 << 64) % q);
    kc[t].rs = host::shoup_quot(kc[t].r, q);
    kc[t].pm = P % q;
    kc[t].pms = host::shoup_quot(kc[t].pm, q);
  }
  KsLimb *d = nullptr;
  hipError_t e = hipMalloc(&d, L1 * sizeof(KsLimb));
  if (e == hipSuccess) e = hipMemcpy(d, kc.data(), L1 * sizeof(KsLimb), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (d) (void)hipFree(d);
    return hip_fail(e);
  }
  s->ks[L1] = d;
  *out = d;
  return HENTT_OK;
}

// Key-switch split: the digit loop holds two accumulator arrays, so whole
// transforms only up to 2^12 (256 lanes); above, a column pass of EC stages
// and blocks of at most 2^12.
template <int LOGN> struct KsPlan {
  static constexpr bool WHOLE = LOGN <= 12;
  static constexpr int EC = LOGN <= 12 ? 0 : (LOGN == 15 || LOGN == 16 || LOGN == 17) ? 5 : LOGN - 12;
  static constexpr int B = LOGN - EC;
  static constexpr int E = 3;  // words per lane in the block kernel (3: occupancy over radix)
};

template <int LOGN> void launch_keyswitch(const KsArgs &a, const Storage *s, hipStream_t st) {
  const uint32_t L1 = a.l + 1;
  using P = KsPlan<LOGN>;
  if constexpr (P::WHOLE) {
    LaunchTimer lt_("k_ks_whole", LOGN, st);
    hipLaunchKernelGGL((k_ks_whole<LOGN, 4>), dim3(a.batch * L1), dim3(1 << (LOGN - 4)), 0, st, a, s->d_tw, s->d_lc);
  } else {
    {
      LaunchTimer lt_("k_ks_cols", LOGN, st);
      hipLaunchKernelGGL((k_ks_cols<LOGN, P::EC>), dim3(a.batch * a.l * L1 * ((1u << (LOGN - P::EC)) / 256)),
                         dim3(256), 0, st, a, s->d_tw, s->d_lc);
    }
    LaunchTimer lt_("k_ks_blocks", LOGN, st);
    hipLaunchKernelGGL((k_ks_blocks<LOGN, P::B, P::E>), dim3((a.batch * L1) << (LOGN - P::B)), dim3(1 << (P::B - P::E)), 0,
                       st, a, s->d_tw, s->d_lc);
  }
}
typedef void (*ks_fn)(const KsArgs &, const Storage *, hipStream_t);
#define KS_ENTRY(n) launch_keyswitch<n>,
const ks_fn k_ks_table[] = {HENTT_SIZES(KS_ENTRY)};

}  // namespace

int run_rescale(const hentt_tables *t, const uint64_t *c, uint64_t *out, uint32_t batch, bool ntt, hipStream_t st) {
  Storage *s = t->s;
  const uint32_t ln = s->log_n, level = t->limbs, L = level - 1;
  const uint64_t N = 1ull << ln;
  const RsLimb *rs = nullptr;
  int rc = rs_constants(s, level, &rs);
  if (rc) return rc;
  RsArgs a{};
  a.c = c;
  a.out = out;
  a.rs = rs;
  a.qL = s->moduli[L];
  a.h = (a.qL - 1) / 2;
  a.batch = batch;
  a.L = L;
  if (!ntt) {
    const uint32_t tiles = (uint32_t)((N + 2047) / 2048);
    LaunchTimer lt_("k_rs_coeff", (int)ln, st);
    hipLaunchKernelGGL(k_rs_coeff, dim3(batch * L * tiles), dim3(256), 0, st, a, s->d_lc, ln, tiles);
    HIPCHK(hipGetLastError());
    return HENTT_OK;
  }
  // the last limb of every batch entry, inverse-transformed modulo qL
  void *tl = nullptr;
  rc = pool_get((size_t)batch * N * 8, st, &tl);
  if (rc) return rc;
  hipError_t e = hipMemcpy2DAsync(tl, N * 8, c + (size_t)L * N, (size_t)level * N * 8, N * 8, batch,
                                  hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) {
    Storage last;  // limb L's tables alone (a view: owns nothing)
    last.log_n = ln;
    last.limbs = 1;
    last.d_tw = s->d_tw + (size_t)L * 2 * N;
    last.d_lc = s->d_lc + L;
    last.d_lcm = s->d_lcm + L;
    last.d_mont = s->d_mont + L;
    last.device = s->device;
    const hentt_tables lv{&last, 1};
    rc = run_transform(&lv, (uint64_t *)tl, batch, st, true);
    if (!rc) {
      a.tl = (const uint64_t *)tl;
      k_rs_table[ln - HENTT_LOG_N_MIN](a, s, st);
      e = hipGetLastError();
    }
  }
  pool_put(tl);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e);
  return HENTT_OK;
}

int run_relin(const hentt_tables *t, const uint64_t *c, const uint64_t *ksk, uint64_t *out, uint32_t batch,
              hipStream_t st) {
  Storage *s = t->s;
  const uint32_t ln = s->log_n, L1 = t->limbs, l = L1 - 1;
  const uint64_t N = 1ull << ln, P = (uint64_t)l * N;
  const KsLimb *kc = nullptr;
  int rc = ks_consts(s, L1, &kc);
  if (rc) return rc;
  const bool two_pass = ln > 12;  // KsPlan<>::WHOLE
  const size_t d_bytes = (size_t)batch * P * 8, acc_bytes = (size_t)batch * 2 * L1 * N * 8;
  const size_t e_bytes = two_pass ? (size_t)batch * l * L1 * N * 8 : 0;
  void *buf = nullptr;
  rc = pool_get(d_bytes + acc_bytes + e_bytes, st, &buf);
  if (rc) return rc;
  uint64_t *d = (uint64_t *)buf, *acc = d + batch * P, *e = acc + (size_t)batch * 2 * L1 * N;
  // digits: c2 in the coefficient domain, modulo its own primes
  hipError_t he = hipMemcpy2DAsync(d, P * 8, c + 2 * P, 3 * P * 8, P * 8, batch, hipMemcpyDeviceToDevice, st);
  const hentt_tables lv{s, l};
  if (he == hipSuccess) rc = run_transform(&lv, d, batch, st, true);
  if (he == hipSuccess && !rc) {
    KsArgs a{};
    a.d = d;
    a.ksk = ksk;
    a.e = two_pass ? e : nullptr;
    a.acc = acc;
    a.c = c;
    a.kc = kc;
    a.batch = batch;
    a.l = l;
    k_ks_table[ln - HENTT_LOG_N_MIN](a, s, st);
    he = hipGetLastError();
    // divide by P with rounding, over q_0 .. q_{l-1}: [batch][2][l+1] -> [batch][2][l];
    // the accumulators already hold P c_s, so this yields (c0, c1) + round(P^-1 c2 evk)
    if (he == hipSuccess) rc = run_rescale(t, acc, out, batch * 2, true, st);
  }
  pool_put(buf);
  if (rc) return rc;
  if (he != hipSuccess) return hip_fail(he);
  return HENTT_OK;
}


// ------------------------------------------------------------ matMul
int run_matmul(const hentt_tables *t, const uint64_t *A, const uint64_t *B, uint64_t *C, uint32_t m, uint32_t n,
               uint32_t k, hipStream_t st) {
  const uint64_t N = 1ull << t->s->log_n;
  const uint32_t tiles = (uint32_t)((N + 2047) / 2048);
  const uint64_t grid = (uint64_t)m * n * t->limbs * tiles;
  if (grid > 0x7fffffffu) return HENTT_EINVAL;
  LaunchTimer lt_("k_ct_matmul", (int)t->s->log_n, st);
  const bool full = N >= 2048, mont = k >= 3;  // Montgomery accumulation pays from k = 3 on
  auto kern = full ? (mont ? k_ct_matmul<true, true> : k_ct_matmul<true, false>)
                   : (mont ? k_ct_matmul<false, true> : k_ct_matmul<false, false>);
  hipLaunchKernelGGL(kern, dim3((uint32_t)grid), dim3(256), 0, st, A, B, C, t->s->d_lc, t->s->d_mont, m, n, k,
                     t->limbs, t->s->log_n, tiles);
  HIPCHK(hipGetLastError());
  return HENTT_OK;
}

}  // namespace hentt_rt
