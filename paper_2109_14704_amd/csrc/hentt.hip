// libhentt: C ABI, twiddle tables, argument checks and kernel dispatch.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/hentt.h"
#include "ntt_kernels.hpp"
#include "batch_kernels.hpp"
#include "rescale_kernels.hpp"
#include "keyswitch_kernels.hpp"

using namespace hentt;

namespace {

thread_local int g_last_hip = 0;

inline int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return HENTT_EHIP;
}
#define HIPCHK(x)                            \
  do {                                       \
    hipError_t e_ = (x);                     \
    if (e_ != hipSuccess) return hip_fail(e_); \
  } while (0)

typedef unsigned __int128 u128;

// ------------------------------------------------------------ host number theory
uint64_t h_mul(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }
uint64_t h_pow(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1;
  b %= m;
  for (; e; e >>= 1, b = h_mul(b, b, m))
    if (e & 1) r = h_mul(r, b, m);
  return r;
}

// Miller-Rabin with the witness set {2, 325, 9375, 28178, 450775, 9780504,
// 1795265022} (Jim Sinclair), deterministic for all n < 2^64.
bool h_is_prime(uint64_t n) {
  if (n < 2) return false;
  for (uint64_t p : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull})
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = __builtin_ctzll(d);
  d >>= s;
  for (uint64_t a : {2ull, 325ull, 9375ull, 28178ull, 450775ull, 9780504ull, 1795265022ull}) {
    a %= n;
    if (a == 0) continue;
    uint64_t x = h_pow(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s && comp; ++r) {
      x = h_mul(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

uint32_t h_brv(uint32_t x, int bits) { return __builtin_bitreverse32(x) >> (32 - bits); }

// Smallest primitive 2N-th root: take any root g of order 2N (a residue r
// with r^N = -1 gives g = r^((q-1)/2N)... found by testing small bases), then
// scan its odd powers g, g^3, ... for the minimum.
uint64_t h_psi(uint64_t q, int log_n) {
  const uint64_t two_n = 2ull << log_n;
  const uint64_t e = (q - 1) / two_n;
  uint64_t g = 0;
  for (uint64_t r = 2; r < 1000000 && r < q; ++r) {
    uint64_t c = h_pow(r, e, q);
    if (h_pow(c, two_n / 2, q) == q - 1) {
      g = c;
      break;
    }
  }
  if (!g) return 0;
  const uint64_t g2 = h_mul(g, g, q);
  uint64_t best = g, cur = g;
  for (uint64_t j = 1; j < two_n / 2; ++j) {
    cur = h_mul(cur, g2, q);
    if (cur < best) best = cur;
  }
  return best;
}

int bit_length(uint64_t v) { return 64 - __builtin_clzll(v); }

int check_modulus(uint64_t q, int log_n) {
  if (q <= (1ull << 7) || q >= (1ull << 60)) return HENTT_EMODULUS;
  if ((q - 1) % (2ull << log_n) != 0) return HENTT_EMODULUS;
  if (!h_is_prime(q)) return HENTT_EMODULUS;
  return HENTT_OK;
}

inline uint64_t shoup_quot(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

// ------------------------------------------------------------ table storage
struct Storage {
  std::atomic<int> refs{1};
  uint32_t log_n = 0, limbs = 0;
  Tw *d_tw = nullptr;          // [limbs][2][N]
  LimbConst *d_lc = nullptr;   // [limbs]
  LimbConst *d_lcm = nullptr;  // [limbs] the same with N^-1 R mod q for N^-1 (after Montgomery products)
  MontLimb *d_mont = nullptr;  // [limbs] Montgomery constants
  std::vector<uint64_t> moduli;
  int device = 0;
  std::mutex rs_mu;            // rescale constants per level (limb count), made on first use
  std::map<uint32_t, RsLimb *> rs;
  std::map<uint32_t, KsLimb *> ks;  // key-switching constants per level (limb count), made on first use
};

void release(Storage *s) {
  if (s->refs.fetch_sub(1) == 1) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(s->device);
    if (s->d_tw) (void)hipFree(s->d_tw);
    if (s->d_lc) (void)hipFree(s->d_lc);
    if (s->d_lcm) (void)hipFree(s->d_lcm);
    if (s->d_mont) (void)hipFree(s->d_mont);
    for (auto &kv : s->rs) (void)hipFree(kv.second);
    for (auto &kv : s->ks) (void)hipFree(kv.second);
    (void)hipSetDevice(cur);
    delete s;
  }
}

// ------------------------------------------------------------ workspace pool
// Device buffers reused by capacity: a request takes the smallest free buffer
// that is large enough, else allocates (the memory cache of section III-C-1).
// A buffer handed out stays with its stream's queued work; it is returned to
// the pool right after the launches are enqueued, which is safe because all
// users of one pool entry enqueue on streams that the caller serialises, and
// the stream ordering of the same stream keeps reuse after completion.
struct PoolEntry {
  void *ptr;
  size_t bytes;
  int device;
  hipStream_t stream;
  bool busy;
};
std::mutex g_pool_mu;
std::vector<PoolEntry> g_pool;

int pool_get(size_t bytes, hipStream_t stream, void **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_pool_mu);
  int best = -1;
  for (size_t i = 0; i < g_pool.size(); ++i) {
    PoolEntry &e = g_pool[i];
    if (e.busy || e.device != dev || e.bytes < bytes) continue;
    if (e.stream != stream) continue;  // reuse only in the stream order that last used it
    if (best < 0 || e.bytes < g_pool[best].bytes) best = (int)i;
  }
  if (best >= 0) {
    g_pool[best].busy = true;
    *out = g_pool[best].ptr;
    return HENTT_OK;
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    return HENTT_ENOMEM;
  }
  g_pool.push_back({p, bytes, dev, stream, true});
  *out = p;
  return HENTT_OK;
}
void pool_put(void *p) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  for (auto &e : g_pool)
    if (e.ptr == p) e.busy = false;
}


// ------------------------------------------------------------ launch timing
// Optional per-kernel timing with HIP events recorded on the launching stream
// around each kernel (hentt_prof_enable); read back with hentt_prof_get.
struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
struct ProfAgg {
  std::string name;
  double ms;
  uint32_t n;
};
std::vector<ProfAgg> g_prof_agg;

struct LaunchTimer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t st;
  const char *name;
  int ln;
  LaunchTimer(const char *nm, int log_n, hipStream_t s) : st(s), name(nm), ln(log_n) {
    if (g_prof_on && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) (void)hipEventRecord(a, st);
  }
  ~LaunchTimer() {
    if (a && b) {
      (void)hipEventRecord(b, st);
      std::lock_guard<std::mutex> lk(g_prof_mu);
      g_prof.push_back({std::string(name) + "<" + std::to_string(ln) + ">", a, b});
    }
  }
};
}  // namespace

struct hentt_tables {
  Storage *s;
  uint32_t limbs;  // <= s->limbs
};

// ------------------------------------------------------------ dispatch
namespace {

// Stage split per N: transforms with N <= 2^14 run whole in one workgroup
// (one HBM round trip); larger N run a column pass of EC stages then blocks
// of 2^(log_n - EC) coefficients.
#ifndef HENTT_EC15
#define HENTT_EC15 5
#endif
#ifndef HENTT_EC16
#define HENTT_EC16 5
#endif
#ifndef HENTT_PEC15
#define HENTT_PEC15 5
#endif
#ifndef HENTT_PEC16
#define HENTT_PEC16 5
#endif
// Stage split (measured): the column pass is HBM-bound with idle ALU, so it
// takes 5 stages at N = 2^15 and 2^16, leaving 2^10 / 2^11 blocks to the
// ALU-bound block and fused kernels (the 5-stage split was 10% faster on the
// CKKS-level batch and 19% on the ciphertext tensor than 3 / 4 stages).
constexpr uint32_t kWholeMaxLogN = 14;  // largest transform done whole by one workgroup
template <int LOGN> struct Plan {
  static constexpr bool WHOLE = LOGN <= (int)kWholeMaxLogN;
  static constexpr int EC = LOGN == 15 ? HENTT_EC15 : LOGN == 16 ? HENTT_EC16 : LOGN == 17 ? 4 : (LOGN > 12 ? LOGN - 12 : 1);
  static constexpr int B = LOGN - EC;
  // fused products: one kernel up to 2^12, else a column pass of PEC stages
  // and blocks of 2^(LOGN - PEC) coefficients
  static constexpr bool PROD_WHOLE = LOGN <= 12;
  static constexpr int PEC = LOGN == 15 ? HENTT_PEC15 : LOGN == 16 ? HENTT_PEC16 : (LOGN > 12 ? LOGN - 12 : 1);
};
// Elements per lane (2^E) in the fused product kernels: the tensor keeps four
// transformed inputs live, so it uses 8 per lane to stay within the VGPRs.
template <int MODE> struct ProdE { static constexpr int E = MODE == PROD_MUL ? 4 : 3; };

ColArgs col_args(uint64_t *x, uint64_t sb) {
  ColArgs a{};
  a.src[0] = x;
  a.dst[0] = x;
  a.src_sb = a.dst_sb = sb;
  return a;
}

template <int LOGN>
void launch_fwd(const hentt_tables *t, uint64_t *x, uint32_t batch, hipStream_t st) {
  const Tw *tw = t->s->d_tw;
  const LimbConst *lc = t->s->d_lc;
  const uint32_t L = t->limbs;
  const uint32_t units = batch * L;
  using P = Plan<LOGN>;
  if constexpr (P::WHOLE) {
    { LaunchTimer lt_("k_fwd_whole", LOGN, st); hipLaunchKernelGGL((k_fwd_whole<LOGN, 4>), dim3(units), dim3(1 << (LOGN - 4)), 0, st, x, tw, lc, batch, L); }
  } else {
    { LaunchTimer lt_("k_cols_fwd", LOGN, st); hipLaunchKernelGGL((k_cols<LOGN, P::EC, false>), dim3(units * ((1u << (LOGN - P::EC)) / (256 * ColCpl<P::EC>::value))), dim3(256), 0, st,
                       col_args(x, (uint64_t)L << LOGN), tw, lc, batch, L); }
    { LaunchTimer lt_("k_fwd_blocks", LOGN, st); hipLaunchKernelGGL((k_fwd_blocks<LOGN, P::B, 4>), dim3(units << (LOGN - P::B)), dim3(1 << (P::B - 4)), 0, st, x,
                       tw, lc, batch, L); }
  }
}

template <int LOGN>
void launch_inv(const hentt_tables *t, uint64_t *x, uint32_t batch, hipStream_t st) {
  const Tw *tw = t->s->d_tw;
  const LimbConst *lc = t->s->d_lc;
  const uint32_t L = t->limbs;
  const uint32_t units = batch * L;
  using P = Plan<LOGN>;
  if constexpr (P::WHOLE) {
    { LaunchTimer lt_("k_inv_whole", LOGN, st); hipLaunchKernelGGL((k_inv_whole<LOGN, 4>), dim3(units), dim3(1 << (LOGN - 4)), 0, st, x, tw, lc, batch, L); }
  } else {
    { LaunchTimer lt_("k_inv_blocks", LOGN, st); hipLaunchKernelGGL((k_inv_blocks<LOGN, P::B, 4>), dim3(units << (LOGN - P::B)), dim3(1 << (P::B - 4)), 0, st, x,
                       tw, lc, batch, L); }
    { LaunchTimer lt_("k_cols_inv", LOGN, st); hipLaunchKernelGGL((k_cols<LOGN, P::EC, true>), dim3(units * ((1u << (LOGN - P::EC)) / (256 * ColCpl<P::EC>::value))), dim3(256), 0, st,
                       col_args(x, (uint64_t)L << LOGN), tw, lc, batch, L); }
  }
}

// Products: in/out component pointers with their batch strides.  in_coeff:
// inputs are coefficient-domain (forward transforms applied); out_coeff:
// outputs go back to the coefficient domain.  ws: workspace for the forward
// column pass output when the product is not one kernel (NIN components of
// batch * limbs * N words), may be null otherwise.
// HENTT_PROD_LDS: extra dynamic LDS bytes per fused-product workgroup (caps
// its occupancy so other kernels' waves can share the CU; tuning knob).
int g_prod_lds = -1;
uint32_t prod_lds_pad() {
  if (g_prod_lds < 0) {
    const char *e = getenv("HENTT_PROD_LDS");
    g_prod_lds = e ? atoi(e) : 0;
  }
  return (uint32_t)g_prod_lds;
}

template <int LOGN, int MODE>
void launch_prod(const hentt_tables *t, const ProdArgs &pa, uint32_t batch, bool in_coeff, bool out_coeff,
                 uint64_t *ws, hipStream_t st) {
  const Tw *tw = t->s->d_tw;
  // outputs going back to the coefficient domain take Montgomery products,
  // whose R^-1 the inverse transform's folded N^-1 R scaling cancels
  const LimbConst *lc = out_coeff ? t->s->d_lcm : t->s->d_lc;
  const MontLimb *mont = t->s->d_mont;
  const uint32_t L = t->limbs;
  const uint32_t units = batch * L;
  constexpr int NIN = ProdShape<MODE>::NIN, NOUT = ProdShape<MODE>::NOUT;
  using P = Plan<LOGN>;
  if (!in_coeff && !out_coeff) {
    const uint32_t tiles = LOGN > 11 ? (1u << (LOGN - 11)) : 1u;
    { LaunchTimer lt_(MODE == PROD_MUL ? "k_elem_mul" : "k_elem_tensor", LOGN, st); hipLaunchKernelGGL((k_elem<MODE>), dim3(units * tiles), dim3(256), 0, st, pa, lc, batch, L, (uint32_t)LOGN, tiles); }
    return;
  }
  constexpr int PE = ProdE<MODE>::E;
  if constexpr (P::PROD_WHOLE) {
    const dim3 g(units), blk(1 << (LOGN - PE));
    if (in_coeff && out_coeff) { LaunchTimer lt_(MODE == PROD_MUL ? "k_prod_mul" : "k_prod_tensor", LOGN, st); hipLaunchKernelGGL((k_prod<LOGN, LOGN, PE, MODE, true, true>), g, blk, prod_lds_pad(), st, pa, tw, lc, mont, batch, L); }
    else if (in_coeff) { LaunchTimer lt_(MODE == PROD_MUL ? "k_prod_mul" : "k_prod_tensor", LOGN, st); hipLaunchKernelGGL((k_prod<LOGN, LOGN, PE, MODE, true, false>), g, blk, prod_lds_pad(), st, pa, tw, lc, mont, batch, L); }
    else { LaunchTimer lt_(MODE == PROD_MUL ? "k_prod_mul" : "k_prod_tensor", LOGN, st); hipLaunchKernelGGL((k_prod<LOGN, LOGN, PE, MODE, false, true>), g, blk, prod_lds_pad(), st, pa, tw, lc, mont, batch, L); }
  } else {
    constexpr int EC = P::PEC, B = LOGN - P::PEC;
    const uint64_t NL = (uint64_t)L << LOGN;
    ProdArgs pb = pa;
    if (in_coeff) {
      // forward column pass of every input into the workspace ([NIN][batch][L][N])
      ColArgs ca{};
      for (int p = 0; p < NIN; ++p) {
        ca.src[p] = pa.in[p];
        ca.dst[p] = ws + (uint64_t)p * batch * NL;
        pb.in[p] = ca.dst[p];
      }
      ca.src_sb = pa.in_sb;
      ca.dst_sb = NL;
      pb.in_sb = NL;
      { LaunchTimer lt_("k_cols_fwd", LOGN, st); hipLaunchKernelGGL((k_cols<LOGN, EC, false>), dim3(NIN * units * ((1u << (LOGN - EC)) / (256 * ColCpl<EC>::value))), dim3(256), 0, st,
                         ca, tw, lc, batch, L); }
    }
    const dim3 g(units << (LOGN - B)), blk(1 << (B - PE));
    if (in_coeff && out_coeff) { LaunchTimer lt_(MODE == PROD_MUL ? "k_prod_mul" : "k_prod_tensor", LOGN, st); hipLaunchKernelGGL((k_prod<LOGN, B, PE, MODE, true, true>), g, blk, prod_lds_pad(), st, pb, tw, lc, mont, batch, L); }
    else if (in_coeff) { LaunchTimer lt_(MODE == PROD_MUL ? "k_prod_mul" : "k_prod_tensor", LOGN, st); hipLaunchKernelGGL((k_prod<LOGN, B, PE, MODE, true, false>), g, blk, prod_lds_pad(), st, pb, tw, lc, mont, batch, L); }
    else { LaunchTimer lt_(MODE == PROD_MUL ? "k_prod_mul" : "k_prod_tensor", LOGN, st); hipLaunchKernelGGL((k_prod<LOGN, B, PE, MODE, false, true>), g, blk, prod_lds_pad(), st, pb, tw, lc, mont, batch, L); }
    if (out_coeff) {
      ColArgs ca{};
      for (int o = 0; o < NOUT; ++o) ca.src[o] = ca.dst[o] = pa.out[o];
      ca.src_sb = ca.dst_sb = pa.out_sb;
      { LaunchTimer lt_("k_cols_inv", LOGN, st); hipLaunchKernelGGL((k_cols<LOGN, EC, true>), dim3(NOUT * units * ((1u << (LOGN - EC)) / (256 * ColCpl<EC>::value))), dim3(256), 0, st,
                         ca, tw, lc, batch, L); }
    }
  }
}

template <int LOGN> constexpr bool needs_ws() { return !Plan<LOGN>::PROD_WHOLE; }

typedef void (*launch_fn)(const hentt_tables *, uint64_t *, uint32_t, hipStream_t);
typedef void (*prod_fn)(const hentt_tables *, const ProdArgs &, uint32_t, bool, bool, uint64_t *, hipStream_t);

#define HENTT_SIZES(M) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15) M(16) M(17)
#define FWD_ENTRY(n) launch_fwd<n>,
#define INV_ENTRY(n) launch_inv<n>,
#define MUL_ENTRY(n) launch_prod<n, PROD_MUL>,
#define TEN_ENTRY(n) launch_prod<n, PROD_TENSOR>,
#define WS_ENTRY(n) needs_ws<n>(),
const launch_fn k_fwd_table[] = {HENTT_SIZES(FWD_ENTRY)};
const launch_fn k_inv_table[] = {HENTT_SIZES(INV_ENTRY)};
const prod_fn k_mul_table[] = {HENTT_SIZES(MUL_ENTRY)};
const prod_fn k_ten_table[] = {HENTT_SIZES(TEN_ENTRY)};
const bool k_ws_table[] = {HENTT_SIZES(WS_ENTRY)};

// Two library streams per device (default priority) and a ring of events.
// A large two-pass call is split into batch chunks alternating between the
// two streams, so one chunk's HBM-bound column pass overlaps another chunk's
// ALU-bound block kernel.  fork/join keep the caller's stream order: the
// chunks wait on an event recorded on the caller's stream, and the caller's
// stream waits on both library streams afterwards (no host synchronisation).
struct DevStreams {
  int device = -1;
  hipStream_t s[2] = {nullptr, nullptr};
  hipEvent_t ev[64] = {};
  uint32_t next = 0;
};
std::mutex g_ds_mu;
std::vector<DevStreams *> g_ds;

DevStreams *dev_streams() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_ds_mu);
  for (auto *d : g_ds)
    if (d->device == dev) return d;
  DevStreams *d = new (std::nothrow) DevStreams();
  if (!d) return nullptr;
  d->device = dev;
  for (auto &x : d->s)
    if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) return nullptr;
  for (auto &e : d->ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  g_ds.push_back(d);
  return d;
}

hipEvent_t next_event(DevStreams *d) {
  std::lock_guard<std::mutex> lk(g_ds_mu);
  return d->ev[d->next++ % 64];
}

// Number of chunks for a two-pass call over batch x limbs (polynomial, limb)
// pairs; HENTT_CHUNKS overrides it (tuning).
int g_chunks_env = -2;
uint32_t chunks_for(uint32_t batch, uint32_t limbs) {
  if (g_chunks_env == -2) {
    const char *e = getenv("HENTT_CHUNKS");
    g_chunks_env = e ? atoi(e) : -1;
  }
  const uint64_t units = (uint64_t)batch * limbs;
  uint32_t n = 1;  // chunking measured at most 2-5% faster: off unless requested
  (void)units;
  if (g_chunks_env > 0) n = (uint32_t)g_chunks_env;
  return n > batch ? batch : n;
}
int g_streams_env = -2;
int stream_count() {
  if (g_streams_env == -2) {
    const char *e = getenv("HENTT_STREAMS");
    g_streams_env = e ? atoi(e) : 2;
  }
  return g_streams_env == 1 ? 1 : 2;
}

int fork_streams(DevStreams *d, hipStream_t caller) {
  hipEvent_t e = next_event(d);
  HIPCHK(hipEventRecord(e, caller));
  HIPCHK(hipStreamWaitEvent(d->s[0], e, 0));
  HIPCHK(hipStreamWaitEvent(d->s[1], e, 0));
  return HENTT_OK;
}

int join_streams(DevStreams *d, hipStream_t caller) {
  for (int k = 0; k < 2; ++k) {
    hipEvent_t e = next_event(d);
    HIPCHK(hipEventRecord(e, d->s[k]));
    HIPCHK(hipStreamWaitEvent(caller, e, 0));
  }
  return HENTT_OK;
}

int run_transform(const hentt_tables *t, uint64_t *x, uint32_t batch, hipStream_t st, bool inv) {
  const int ln = (int)t->s->log_n;
  launch_fn fn = (inv ? k_inv_table : k_fwd_table)[ln - HENTT_LOG_N_MIN];
  const uint32_t nch = ln > 14 ? chunks_for(batch, t->limbs) : 1;
  DevStreams *d = nch > 1 ? dev_streams() : nullptr;
  if (!d) {
    fn(t, x, batch, st);
    HIPCHK(hipGetLastError());
    return HENTT_OK;
  }
  int rc = fork_streams(d, st);
  if (rc) return rc;
  const uint64_t NL = (uint64_t)t->limbs << ln;
  for (uint32_t c = 0, b0 = 0; c < nch; ++c) {
    const uint32_t b1 = (uint32_t)((uint64_t)batch * (c + 1) / nch);
    fn(t, x + (uint64_t)b0 * NL, b1 - b0, d->s[stream_count() == 1 ? 0 : (c & 1)]);
    b0 = b1;
  }
  HIPCHK(hipGetLastError());
  return join_streams(d, st);
}

// Design-ladder variants of the forward transform (section III-B): the naive
// radix-2 baseline; staged radix-2 (four naive global stages, then LDS blocks
// of 2048 words with radix-2 rounds, one stage per LDS exchange); and staged
// transforms whose LDS rounds are radix-4, -8 or -16 on blocks of 4096 words
// (the paper's work-group tile) after one radix-8 column pass.
void launch_naive_stages(const hentt_tables *t, uint64_t *x, uint64_t units, uint32_t s0, uint32_t s1,
                         hipStream_t st) {
  const uint32_t ln = t->s->log_n;
  const uint64_t grid = ((units << (ln - 1)) + 255) / 256;
  for (uint32_t s = s0; s < s1; ++s) {
    LaunchTimer lt_("k_naive_stage", (int)ln, st);
    hipLaunchKernelGGL(k_naive_stage, dim3((uint32_t)grid), dim3(256), 0, st, x, t->s->d_tw, t->s->d_lc,
                       (uint32_t)units, t->limbs, ln, s);
  }
}

template <int E> void launch_staged15(const hentt_tables *t, uint64_t *x, uint32_t batch, hipStream_t st) {
  const uint32_t L = t->limbs, units = batch * L;
  const char *name = E == 2 ? "k_fwd_blocks_r4" : E == 3 ? "k_fwd_blocks_r8" : "k_fwd_blocks_r16";
  { LaunchTimer lt_("k_cols_fwd_r8", 15, st); hipLaunchKernelGGL((k_cols<15, 3, false>), dim3(units * ((1u << 12) / (256 * ColCpl<3>::value))), dim3(256), 0, st, col_args(x, (uint64_t)L << 15), t->s->d_tw, t->s->d_lc, batch, L); }
  { LaunchTimer lt_(name, 15, st); hipLaunchKernelGGL((k_fwd_blocks<15, 12, E>), dim3(units << 3), dim3(1 << (12 - E)), 0, st, x, t->s->d_tw, t->s->d_lc, batch, L); }
}

int run_fwd_variant(const hentt_tables *t, uint64_t *x, uint32_t batch, int variant, hipStream_t st) {
  const uint32_t ln = t->s->log_n, L = t->limbs;
  const uint64_t units = (uint64_t)batch * L;
  switch (variant) {
    case HENTT_VARIANT_LIBRARY:
      return run_transform(t, x, batch, st, false);
    case HENTT_VARIANT_NAIVE: {
      const uint64_t grid = ((units << (ln - 1)) + 255) / 256, words = units << ln;
      if (grid > 0x7fffffffu || (words + 255) / 256 > 0x7fffffffu || units > 0xffffffffu) return HENTT_EINVAL;
      launch_naive_stages(t, x, units, 0, ln, st);
      {
        LaunchTimer lt_("k_reduce8q", (int)ln, st);
        hipLaunchKernelGGL(k_reduce8q, dim3((uint32_t)((words + 255) / 256)), dim3(256), 0, st, x, t->s->d_lc, words, L,
                           ln);
      }
      break;
    }
    case HENTT_VARIANT_STAGED_R2:
      if (ln != 15 || ((units << 14) + 255) / 256 > 0x7fffffffu) return HENTT_EINVAL;
      launch_naive_stages(t, x, units, 0, 4, st);
      {
        LaunchTimer lt_("k_fwd_blocks_r2", 15, st);
        hipLaunchKernelGGL((k_fwd_blocks<15, 11, 1>), dim3((uint32_t)(units << 4)), dim3(1 << 10), 0, st, x,
                           t->s->d_tw, t->s->d_lc, batch, L);
      }
      break;
    case HENTT_VARIANT_STAGED_R4:
    case HENTT_VARIANT_STAGED_R8:
    case HENTT_VARIANT_STAGED_R16:
      if (ln != 15) return HENTT_EINVAL;
      if (variant == HENTT_VARIANT_STAGED_R4) launch_staged15<2>(t, x, batch, st);
      else if (variant == HENTT_VARIANT_STAGED_R8) launch_staged15<3>(t, x, batch, st);
      else launch_staged15<4>(t, x, batch, st);
      break;
    default:
      return HENTT_EINVAL;
  }
  HIPCHK(hipGetLastError());
  return HENTT_OK;
}

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
    host[i].mu = (uint64_t)(((u128)1 << 64) / q);
    host[i].nh = q - h % q;
    host[i].w = h_pow(qL % q, q - 2, q);
    host[i].ws = shoup_quot(host[i].w, q);
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

template <int LOGN> void launch_rescale_ntt(const RsArgs &a, const Storage *s, hipStream_t st) {
  const uint32_t units = a.batch * a.L;
  using P = Plan<LOGN>;
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
    uint64_t qi = q;  // q^-1 mod 2^64 by Newton's iteration
    for (int i = 0; i < 5; ++i) qi *= 2 - q * qi;
    kc[t].mu = (uint64_t)(((u128)1 << 64) / q);
    kc[t].qinv = 0 - qi;
    kc[t].r = (uint64_t)(((u128)1 << 64) % q);
    kc[t].rs = shoup_quot(kc[t].r, q);
    kc[t].pm = P % q;
    kc[t].pms = shoup_quot(kc[t].pm, q);
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

int run_prod(const hentt_tables *t, int mode, const ProdArgs &pa, uint32_t batch, bool in_coeff, bool out_coeff,
             hipStream_t st) {
  const int ln = (int)t->s->log_n;
  const int nin = mode == PROD_MUL ? 2 : 4;
  const uint64_t NL = (uint64_t)t->limbs << ln;
  void *ws = nullptr;
  if (in_coeff && k_ws_table[ln - HENTT_LOG_N_MIN]) {
    int rc = pool_get((size_t)nin * batch * NL * 8ull, st, &ws);
    if (rc) return rc;
  }
  prod_fn fn = (mode == PROD_MUL ? k_mul_table : k_ten_table)[ln - HENTT_LOG_N_MIN];
  const bool two_pass = k_ws_table[ln - HENTT_LOG_N_MIN] && (in_coeff || out_coeff);
  const uint32_t nch = two_pass ? chunks_for(batch, t->limbs) : 1;
  DevStreams *d = nch > 1 ? dev_streams() : nullptr;
  int rc = HENTT_OK;
  if (!d) {
    fn(t, pa, batch, in_coeff, out_coeff, (uint64_t *)ws, st);
  } else {
    rc = fork_streams(d, st);
    for (uint32_t c = 0, b0 = 0; c < nch && !rc; ++c) {
      const uint32_t b1 = (uint32_t)((uint64_t)batch * (c + 1) / nch);
      ProdArgs pc = pa;
      for (int p = 0; p < nin; ++p) pc.in[p] = pa.in[p] + (uint64_t)b0 * pa.in_sb;
      for (int o = 0; o < 3; ++o)
        if (pa.out[o]) pc.out[o] = pa.out[o] + (uint64_t)b0 * pa.out_sb;
      // each chunk owns the slice [chunk][batch entries][limbs][N] of the workspace
      uint64_t *wc = ws ? (uint64_t *)ws + (uint64_t)nin * b0 * NL : nullptr;
      fn(t, pc, b1 - b0, in_coeff, out_coeff, wc, d->s[stream_count() == 1 ? 0 : (c & 1)]);
      b0 = b1;
    }
    if (!rc) rc = join_streams(d, st);
  }
  hipError_t e = hipGetLastError();
  if (ws) pool_put(ws);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e);
  return HENTT_OK;
}

}  // namespace

namespace {
template <int LOGN> void split_of(uint32_t *ec, uint32_t *pec) {
  *ec = Plan<LOGN>::WHOLE ? 0u : (uint32_t)Plan<LOGN>::EC;
  *pec = Plan<LOGN>::PROD_WHOLE ? 0u : (uint32_t)Plan<LOGN>::PEC;
}
typedef void (*split_fn)(uint32_t *, uint32_t *);
#define SPLIT_ENTRY(n) split_of<n>,
const split_fn k_split_table[] = {HENTT_SIZES(SPLIT_ENTRY)};
}  // namespace

// ================================================================== C ABI
extern "C" {

const char *hentt_status_str(int s) {
  switch (s) {
    case HENTT_OK: return "ok";
    case HENTT_EINVAL: return "invalid argument";
    case HENTT_EMODULUS: return "bad modulus (must be prime, 1 mod 2N, 2^7 < q < 2^60)";
    case HENTT_ENOMEM: return "out of memory";
    case HENTT_EHIP: return "HIP runtime error";
    case HENTT_ETIMEOUT: return "a batch tile waited past its spin limit (results incomplete)";
    default: return "unknown status";
  }
}

int hentt_last_hip_error(void) { return g_last_hip; }

int hentt_stage_split(uint32_t log_n, uint32_t *transform_cols, uint32_t *product_cols) {
  if (!transform_cols || !product_cols || log_n < HENTT_LOG_N_MIN || log_n > HENTT_LOG_N_MAX) return HENTT_EINVAL;
  k_split_table[log_n - HENTT_LOG_N_MIN](transform_cols, product_cols);
  return HENTT_OK;
}

int hentt_psi(uint64_t q, uint32_t log_n, uint64_t *psi) {
  if (!psi || log_n < 1 || log_n > 30) return HENTT_EINVAL;
  if (q < 3 || (q - 1) % (2ull << log_n) != 0 || !h_is_prime(q)) return HENTT_EMODULUS;
  uint64_t p = h_psi(q, (int)log_n);
  if (!p) return HENTT_EMODULUS;
  *psi = p;
  return HENTT_OK;
}

int hentt_tables_create(uint32_t log_n, uint32_t limbs, const uint64_t *moduli_host, void *stream,
                        hentt_tables **out) {
  if (!out || !moduli_host || limbs == 0 || limbs > HENTT_LIMBS_MAX) return HENTT_EINVAL;
  if (log_n < HENTT_LOG_N_MIN || log_n > HENTT_LOG_N_MAX) return HENTT_EINVAL;
  *out = nullptr;
  for (uint32_t l = 0; l < limbs; ++l) {
    int rc = check_modulus(moduli_host[l], (int)log_n);
    if (rc) return rc;
  }
  const uint32_t N = 1u << log_n;
  std::vector<Tw> tw((size_t)limbs * 2 * N);
  std::vector<LimbConst> lc(limbs), lcm(limbs);
  std::vector<MontLimb> mont(limbs);
  std::vector<uint64_t> pw(N), ipw(N);
  for (uint32_t l = 0; l < limbs; ++l) {
    const uint64_t q = moduli_host[l];
    const uint64_t psi = h_psi(q, (int)log_n);
    if (!psi) return HENTT_EMODULUS;
    const uint64_t psi_inv = h_pow(psi, q - 2, q);
    pw[0] = ipw[0] = 1;
    for (uint32_t i = 1; i < N; ++i) {
      pw[i] = h_mul(pw[i - 1], psi, q);
      ipw[i] = h_mul(ipw[i - 1], psi_inv, q);
    }
    Tw *f = &tw[(size_t)l * 2 * N], *iv = f + N;
    for (uint32_t k = 0; k < N; ++k) {
      const uint32_t r = h_brv(k, (int)log_n);
      f[k] = {pw[r], shoup_quot(pw[r], q)};
      iv[k] = {ipw[r], shoup_quot(ipw[r], q)};
    }
    LimbConst &c = lc[l];
    memset(&c, 0, sizeof(c));
    c.m.q = q;
    c.m.nq = 0 - q;
    c.m.q2 = 2 * q;
    c.m.nq2 = 0 - 2 * q;
    c.m.q4 = 4 * q;
    c.m.nq4 = 0 - 4 * q;
    c.ninv = h_pow(N % q, q - 2, q);
    c.ninv_s = shoup_quot(c.ninv, q);
    c.ninvw = h_mul(c.ninv, iv[1].w, q);
    c.ninvw_s = shoup_quot(c.ninvw, q);
    c.k = (uint32_t)bit_length(q);
    c.mu = (uint64_t)(((u128)1 << (2 * c.k)) / q);
    uint64_t qi = q;  // q^-1 mod 2^64 by Newton's iteration (3 -> 96 bits)
    for (int i = 0; i < 5; ++i) qi *= 2 - q * qi;
    const uint64_t r = (uint64_t)(((u128)1 << 64) % q);
    mont[l] = MontLimb{0 - qi, r, shoup_quot(r, q), 0};
    LimbConst &cm = lcm[l];
    cm = c;
    cm.ninv = h_mul(c.ninv, r, q);
    cm.ninv_s = shoup_quot(cm.ninv, q);
    cm.ninvw = h_mul(c.ninvw, r, q);
    cm.ninvw_s = shoup_quot(cm.ninvw, q);
  }
  Storage *s = new (std::nothrow) Storage();
  if (!s) return HENTT_ENOMEM;
  s->log_n = log_n;
  s->limbs = limbs;
  s->moduli.assign(moduli_host, moduli_host + limbs);
  (void)hipGetDevice(&s->device);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMalloc(&s->d_tw, tw.size() * sizeof(Tw));
  if (e == hipSuccess) e = hipMalloc(&s->d_lc, lc.size() * sizeof(LimbConst));
  if (e == hipSuccess) e = hipMemcpyAsync(s->d_tw, tw.data(), tw.size() * sizeof(Tw), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMalloc(&s->d_lcm, lcm.size() * sizeof(LimbConst));
  if (e == hipSuccess) e = hipMalloc(&s->d_mont, mont.size() * sizeof(MontLimb));
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_lc, lc.data(), lc.size() * sizeof(LimbConst), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_lcm, lcm.data(), lcm.size() * sizeof(LimbConst), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_mont, mont.data(), mont.size() * sizeof(MontLimb), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    release(s);
    g_last_hip = (int)e;
    return e == hipErrorOutOfMemory ? HENTT_ENOMEM : HENTT_EHIP;
  }
  hentt_tables *h = new (std::nothrow) hentt_tables{s, limbs};
  if (!h) {
    release(s);
    return HENTT_ENOMEM;
  }
  *out = h;
  return HENTT_OK;
}

int hentt_tables_destroy(hentt_tables *t) {
  if (!t) return HENTT_EINVAL;
  release(t->s);
  delete t;
  return HENTT_OK;
}

int hentt_tables_view(const hentt_tables *t, uint32_t limbs, hentt_tables **view) {
  if (!t || !view || limbs == 0 || limbs > t->limbs) return HENTT_EINVAL;
  hentt_tables *h = new (std::nothrow) hentt_tables{t->s, limbs};
  if (!h) return HENTT_ENOMEM;
  t->s->refs.fetch_add(1);
  *view = h;
  return HENTT_OK;
}

int hentt_tables_info(const hentt_tables *t, uint32_t *log_n, uint32_t *limbs) {
  if (!t) return HENTT_EINVAL;
  if (log_n) *log_n = t->s->log_n;
  if (limbs) *limbs = t->limbs;
  return HENTT_OK;
}

int hentt_tables_device_ptrs(const hentt_tables *t, const uint64_t **fwd, const uint64_t **inv,
                             const uint64_t **moduli) {
  if (!t) return HENTT_EINVAL;
  const size_t N = 1u << t->s->log_n;
  // per limb: fwd pairs then inv pairs; callers index limb l at l * 2N pairs
  if (fwd) *fwd = (const uint64_t *)t->s->d_tw;
  if (inv) *inv = (const uint64_t *)(t->s->d_tw + N);
  if (moduli) *moduli = (const uint64_t *)t->s->d_lc;
  return HENTT_OK;
}

int hentt_ntt_fwd(const hentt_tables *t, uint64_t *x, uint32_t batch, void *stream) {
  if (!t || !x || batch == 0) return HENTT_EINVAL;
  return run_transform(t, x, batch, (hipStream_t)stream, false);
}

int hentt_ntt_fwd_variant(const hentt_tables *t, uint64_t *x, uint32_t batch, int variant, void *stream) {
  if (!t || !x || batch == 0) return HENTT_EINVAL;
  return run_fwd_variant(t, x, batch, variant, (hipStream_t)stream);
}

int hentt_rescale(const hentt_tables *t, const uint64_t *c, uint64_t *out, uint32_t batch, uint32_t flags,
                  void *stream) {
  if (!t || !c || !out || batch == 0 || t->limbs < 2) return HENTT_EINVAL;
  const bool ntt = flags == (HENTT_IN_NTT | HENTT_OUT_NTT);
  if (!ntt && flags != 0) return HENTT_EINVAL;
  const uint64_t N = 1ull << t->s->log_n;
  const uintptr_t c0 = (uintptr_t)c, c1 = c0 + (uintptr_t)(batch * (uint64_t)t->limbs * N * 8);
  const uintptr_t o0 = (uintptr_t)out, o1 = o0 + (uintptr_t)(batch * (uint64_t)(t->limbs - 1) * N * 8);
  if (o0 < c1 && c0 < o1) return HENTT_EINVAL;  // out overlaps c
  return run_rescale(t, c, out, batch, ntt, (hipStream_t)stream);
}

int hentt_ct_matmul(const hentt_tables *t, const uint64_t *A, const uint64_t *B, uint64_t *C, uint32_t m, uint32_t n,
                    uint32_t k, void *stream) {
  if (!t || !A || !B || !C || m == 0 || n == 0 || k == 0) return HENTT_EINVAL;
  const uint64_t N = 1ull << t->s->log_n, P = (uint64_t)t->limbs * N;
  const uintptr_t c0 = (uintptr_t)C, c1 = c0 + (uintptr_t)((uint64_t)m * n * 3 * P * 8);
  const uintptr_t a0 = (uintptr_t)A, a1 = a0 + (uintptr_t)((uint64_t)m * k * 2 * P * 8);
  const uintptr_t b0 = (uintptr_t)B, b1 = b0 + (uintptr_t)((uint64_t)k * n * 2 * P * 8);
  if ((c0 < a1 && a0 < c1) || (c0 < b1 && b0 < c1)) return HENTT_EINVAL;  // C overlaps an input
  const uint32_t tiles = (uint32_t)((N + 2047) / 2048);
  const uint64_t grid = (uint64_t)m * n * t->limbs * tiles;
  if (grid > 0x7fffffffu) return HENTT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  LaunchTimer lt_("k_ct_matmul", (int)t->s->log_n, st);
  const bool full = N >= 2048, mont = k >= 3;  // Montgomery accumulation pays from k = 3 on
  auto kern = full ? (mont ? k_ct_matmul<true, true> : k_ct_matmul<true, false>)
                   : (mont ? k_ct_matmul<false, true> : k_ct_matmul<false, false>);
  hipLaunchKernelGGL(kern, dim3((uint32_t)grid), dim3(256), 0, st, A, B, C, t->s->d_lc, t->s->d_mont, m, n, k,
                     t->limbs, t->s->log_n, tiles);
  HIPCHK(hipGetLastError());
  return HENTT_OK;
}

int hentt_relin(const hentt_tables *t, const uint64_t *c, const uint64_t *ksk, uint64_t *out, uint32_t batch,
                void *stream) {
  if (!t || !c || !ksk || !out || batch == 0 || t->limbs < 2) return HENTT_EINVAL;
  const uint64_t N = 1ull << t->s->log_n, l = t->limbs - 1;
  const uintptr_t o0 = (uintptr_t)out, o1 = o0 + (uintptr_t)(batch * 2 * l * N * 8);
  const uintptr_t c0 = (uintptr_t)c, c1 = c0 + (uintptr_t)(batch * 3 * l * N * 8);
  const uintptr_t k0 = (uintptr_t)ksk, k1 = k0 + (uintptr_t)(l * 2 * (l + 1) * N * 8);
  if ((o0 < c1 && c0 < o1) || (o0 < k1 && k0 < o1)) return HENTT_EINVAL;  // out overlaps an input
  return run_relin(t, c, ksk, out, batch, (hipStream_t)stream);
}

int hentt_ntt_inv(const hentt_tables *t, uint64_t *x, uint32_t batch, void *stream) {
  if (!t || !x || batch == 0) return HENTT_EINVAL;
  return run_transform(t, x, batch, (hipStream_t)stream, true);
}

int hentt_dyadic_mul(const hentt_tables *t, const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t batch,
                     void *stream) {
  if (!t || !a || !b || !out || batch == 0) return HENTT_EINVAL;
  ProdArgs pa{};
  pa.in[0] = a;
  pa.in[1] = b;
  pa.out[0] = out;
  pa.in_sb = pa.out_sb = (uint64_t)t->limbs << t->s->log_n;
  return run_prod(t, PROD_MUL, pa, batch, false, false, (hipStream_t)stream);
}

int hentt_polymul(const hentt_tables *t, const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t batch,
                  void *stream) {
  if (!t || !a || !b || !out || batch == 0) return HENTT_EINVAL;
  ProdArgs pa{};
  pa.in[0] = a;
  pa.in[1] = b;
  pa.out[0] = out;
  pa.in_sb = pa.out_sb = (uint64_t)t->limbs << t->s->log_n;
  return run_prod(t, PROD_MUL, pa, batch, true, true, (hipStream_t)stream);
}

int hentt_ct_tensor(const hentt_tables *t, const uint64_t *c, const uint64_t *d, uint64_t *out, uint32_t batch,
                    uint32_t flags, void *stream) {
  if (!t || !c || !d || !out || batch == 0 || (flags & ~3u)) return HENTT_EINVAL;
  const uint64_t NL = (uint64_t)t->limbs << t->s->log_n;
  ProdArgs pa{};
  pa.in[0] = c;
  pa.in[1] = c + NL;
  pa.in[2] = d;
  pa.in[3] = d + NL;
  for (int o = 0; o < 3; ++o) pa.out[o] = out + o * NL;
  pa.in_sb = 2 * NL;
  pa.out_sb = 3 * NL;
  return run_prod(t, PROD_TENSOR, pa, batch, !(flags & HENTT_IN_NTT), !(flags & HENTT_OUT_NTT), (hipStream_t)stream);
}

// ------------------------------------------------------------ uneven batches
}  // extern "C"

struct hentt_batch_plan {
  int dir = 1;
  int device = 0;
  uint32_t nunits = 0, ntiles = 0, grid = 0, nq = 0;
  std::vector<BatchUnit> units;          // host copy (queues are rebuilt when the grid changes)
  BatchUnit *d_units = nullptr;
  BatchTile *d_tiles = nullptr;
  uint32_t *d_qoff = nullptr;            // BATCH_NQ + 1 tile offsets
  uint32_t *d_qmap = nullptr;            // 16 entries: XCC_ID -> queue (or ~0)
  uint32_t *d_ctl = nullptr;             // BATCH_NQ + 1 + nunits words
  std::vector<uint32_t> qlen;
  std::vector<hentt_job> small;          // jobs with N < 2^12: ordinary launches
  std::vector<hentt_tables> small_views;
  hipEvent_t done = nullptr;
};

struct hentt_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

const uint32_t kSpinLimit = 1u << 22;   // bounded wait of a pass-2 tile (s_sleep 4 per try)

int default_grid() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus * 2;  // the persistent kernel holds many VGPRs: 2 workgroups of 256 lanes per CU
}

void plan_free(hentt_batch_plan *p) {
  if (p->done) (void)hipEventSynchronize(p->done), (void)hipEventDestroy(p->done);
  for (void *d : {(void *)p->d_units, (void *)p->d_tiles, (void *)p->d_qoff, (void *)p->d_qmap, (void *)p->d_ctl})
    if (d) (void)hipFree(d);
  delete p;
}

uint32_t pass1_tiles(uint32_t ln, int dir) {
  if (ln == BATCH_B) return 0;
  return dir > 0 ? batch_col_tiles(ln) : (1u << (ln - BATCH_B));
}
uint32_t pass2_tiles(uint32_t ln, int dir) {
  if (ln == BATCH_B) return 0;
  return dir > 0 ? (1u << (ln - BATCH_B)) : batch_col_tiles(ln);
}

// Places the plan's workgroups (probe kernel), maps XCDs to queues, spreads
// the units over the queues (largest first, least-loaded queue) and orders
// each queue.  A queue is two streams merged: pass-1 (and whole) tiles in
// unit order, and pass-2 tiles in unit order.  A pass-2 tile is placed at
// least LOOK tiles after the last pass-1 tile of its unit, where LOOK is
// twice the number of workgroups serving the queue: by the time a workgroup
// takes the pass-2 tile, the workgroups that took those pass-1 tiles have
// most likely finished them, so the dependency wait is rarely taken.
int plan_queues(hentt_batch_plan *p) {
  const uint32_t grid = std::max(1u, p->grid);
  uint32_t *d_probe = nullptr;
  HIPCHK(hipMalloc(&d_probe, grid * sizeof(uint32_t)));
  hipLaunchKernelGGL(k_xcc_probe, dim3(grid), dim3(64), 0, 0, d_probe);
  std::vector<uint32_t> where(grid);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpy(where.data(), d_probe, grid * sizeof(uint32_t), hipMemcpyDeviceToHost);
  (void)hipFree(d_probe);
  if (e != hipSuccess) return hip_fail(e);
  uint32_t qmap[16];
  for (auto &m : qmap) m = ~0u;
  uint32_t nq = 0;
  for (uint32_t x : where)
    if (qmap[x & 15] == ~0u && nq < BATCH_NQ) qmap[x & 15] = nq++;
  p->nq = nq;
  std::vector<uint32_t> served(BATCH_NQ, 0);  // workgroups serving each queue
  for (uint32_t x : where)
    if (qmap[x & 15] < BATCH_NQ) ++served[qmap[x & 15]];
  // Units that share a twiddle table (same limb, size and direction) go to
  // one queue back to back, so that the table is read into that XCD's L2 once
  // rather than from memory per unit: the block pass of an N = 2^17
  // transform reads about as many twiddle bytes as data bytes.  Groups are cut
  // into pieces of at most half a fair share (cost ~ N log N per unit) and the
  // pieces placed largest first on the least-loaded queue; each queue then
  // runs its pieces largest N first.
  auto cost = [&](uint32_t i) { return (double)(1u << p->units[i].logn) * p->units[i].logn; };
  std::map<const Tw *, std::vector<uint32_t>> by_table;
  double total = 0;
  for (uint32_t i = 0; i < p->units.size(); ++i) {
    by_table[p->units[i].tw].push_back(i);
    total += cost(i);
  }
  const double cap = std::max(total / nq / 2, 1.0);
  std::vector<std::vector<uint32_t>> pieces;
  for (auto &g : by_table) {
    std::vector<uint32_t> cur;
    double c = 0;
    for (uint32_t i : g.second) {
      if (!cur.empty() && c + cost(i) > cap) {
        pieces.push_back(cur);
        cur.clear();
        c = 0;
      }
      cur.push_back(i);
      c += cost(i);
    }
    if (!cur.empty()) pieces.push_back(cur);
  }
  auto piece_cost = [&](const std::vector<uint32_t> &pc) { return cost(pc[0]) * pc.size(); };
  std::stable_sort(pieces.begin(), pieces.end(),
                   [&](const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) { return piece_cost(a) > piece_cost(b); });
  std::vector<std::vector<const std::vector<uint32_t> *>> qpieces(nq);
  std::vector<double> load(nq, 0.0);
  for (const auto &pc : pieces) {
    uint32_t best = 0;
    for (uint32_t k = 1; k < nq; ++k)
      if (load[k] < load[best]) best = k;
    qpieces[best].push_back(&pc);
    load[best] += piece_cost(pc);
  }
  std::vector<std::vector<uint32_t>> qunits(nq);
  for (uint32_t k = 0; k < nq; ++k) {
    std::stable_sort(qpieces[k].begin(), qpieces[k].end(), [&](const std::vector<uint32_t> *a, const std::vector<uint32_t> *b) {
      return p->units[(*a)[0]].logn > p->units[(*b)[0]].logn;
    });
    for (const auto *pc : qpieces[k]) qunits[k].insert(qunits[k].end(), pc->begin(), pc->end());
  }
  std::vector<BatchTile> tiles;
  std::vector<uint32_t> qoff(BATCH_NQ + 1, 0);
  std::vector<size_t> ready(p->units.size(), 0);  // queue position after a unit's last pass-1 tile
  for (uint32_t k = 0; k < BATCH_NQ; ++k) {
    qoff[k] = (uint32_t)tiles.size();
    if (k >= nq) continue;
    const size_t look = 2 * (size_t)served[k];
    const std::vector<uint32_t> &us = qunits[k];
    std::vector<BatchTile> first;  // whole and pass-1 tiles, unit order
    for (uint32_t i : us) {
      const BatchUnit &u = p->units[i];
      if (u.logn == BATCH_B) first.push_back({i, (uint32_t)BT_WHOLE << 16});
      for (uint32_t t = 0; t < u.pass1; ++t) first.push_back({i, ((uint32_t)BT_PASS1 << 16) | t});
    }
    size_t next = 0;
    auto emit_first = [&]() {
      const BatchTile bt = first[next++];
      tiles.push_back(bt);
      if ((bt.kind_idx >> 16) == BT_PASS1 && (bt.kind_idx & 0xffffu) + 1 == p->units[bt.unit].pass1)
        ready[bt.unit] = tiles.size();
    };
    for (uint32_t i : us) {
      const uint32_t n2 = pass2_tiles(p->units[i].logn, p->dir);
      if (n2 == 0) continue;
      // every pass-1 tile of unit i is queued, and LOOK more tiles after it
      while (next < first.size() && (ready[i] == 0 || tiles.size() < ready[i] + look)) emit_first();
      for (uint32_t t = 0; t < n2; ++t) tiles.push_back({i, ((uint32_t)BT_PASS2 << 16) | t});
    }
    while (next < first.size()) emit_first();
  }
  qoff[BATCH_NQ] = (uint32_t)tiles.size();
  p->ntiles = (uint32_t)tiles.size();
  p->qlen.assign(BATCH_NQ, 0);
  for (uint32_t k = 0; k < BATCH_NQ; ++k) p->qlen[k] = qoff[k + 1] - qoff[k];
  if (p->d_tiles) (void)hipFree(p->d_tiles);
  p->d_tiles = nullptr;
  e = hipMalloc(&p->d_tiles, std::max<size_t>(1, tiles.size()) * sizeof(BatchTile));
  if (e == hipSuccess && !tiles.empty())
    e = hipMemcpy(p->d_tiles, tiles.data(), tiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_qoff, qoff.data(), qoff.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_qmap, qmap, sizeof(qmap), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e);
  return HENTT_OK;
}

int plan_build(const hentt_job *jobs, uint32_t njobs, int dir, hentt_batch_plan **out) {
  if (!jobs || njobs == 0 || !out || (dir != 1 && dir != -1)) return HENTT_EINVAL;
  for (uint32_t j = 0; j < njobs; ++j) {
    const hentt_job &jb = jobs[j];
    if (!jb.data || !jb.t || jb.batch == 0 || jb.limbs == 0 || jb.limbs > jb.t->limbs) return HENTT_EINVAL;
  }
  hentt_batch_plan *p = new (std::nothrow) hentt_batch_plan();
  if (!p) return HENTT_ENOMEM;
  p->dir = dir;
  (void)hipGetDevice(&p->device);
  for (uint32_t j = 0; j < njobs; ++j) {
    const hentt_job &jb = jobs[j];
    const uint32_t ln = jb.t->s->log_n;
    const uint64_t N = 1ull << ln;
    if (ln < BATCH_B) {
      p->small.push_back(jb);
      continue;
    }
    for (uint32_t b = 0; b < jb.batch; ++b)
      for (uint32_t l = 0; l < jb.limbs; ++l) {
        BatchUnit u;
        u.data = jb.data + ((uint64_t)b * jb.limbs + l) * N;
        u.tw = jb.t->s->d_tw + ((size_t)l * 2 + (dir < 0 ? 1 : 0)) * N;
        u.lc = jb.t->s->d_lc + l;
        u.logn = ln;
        u.pass1 = pass1_tiles(ln, dir);
        p->units.push_back(u);
      }
  }
  for (auto &sj : p->small) p->small_views.push_back(hentt_tables{sj.t->s, sj.limbs});
  p->nunits = (uint32_t)p->units.size();
  p->grid = (uint32_t)default_grid();
  hipError_t e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
  if (p->nunits && e == hipSuccess) {
    e = hipMalloc(&p->d_units, p->units.size() * sizeof(BatchUnit));
    if (e == hipSuccess) e = hipMalloc(&p->d_qoff, (BATCH_NQ + 1) * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&p->d_qmap, 16 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&p->d_ctl, (BATCH_NQ + 1 + p->units.size()) * sizeof(uint32_t));
    if (e == hipSuccess)
      e = hipMemcpy(p->d_units, p->units.data(), p->units.size() * sizeof(BatchUnit), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    plan_free(p);
    g_last_hip = (int)e;
    return e == hipErrorOutOfMemory ? HENTT_ENOMEM : HENTT_EHIP;
  }
  if (p->nunits) {
    int rc = plan_queues(p);
    if (rc) {
      plan_free(p);
      return rc;
    }
  }
  *out = p;
  return HENTT_OK;
}

int plan_launch(hentt_batch_plan *p, hipStream_t st) {
  const int LOGN = 0;  // timer label
  if (p->nunits) {
    const uint32_t n = BATCH_NQ + 1 + p->nunits;
    hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024), dim3(256), 0, st, p->d_ctl, n, 0u);
    HIPCHK(hipGetLastError());
    const uint32_t grid = p->grid;  // every workgroup of the probed placement (idle ones exit at once)
    if (p->dir > 0) { LaunchTimer lt_("k_batch_fwd", LOGN, st); hipLaunchKernelGGL(k_batch<false>, dim3(grid), dim3(BATCH_LANES), 0, st, p->d_units, p->d_tiles, p->d_qoff, p->d_qmap, p->d_ctl, kSpinLimit); }
    else { LaunchTimer lt_("k_batch_inv", LOGN, st); hipLaunchKernelGGL(k_batch<true>, dim3(grid), dim3(BATCH_LANES), 0, st, p->d_units, p->d_tiles, p->d_qoff, p->d_qmap, p->d_ctl, kSpinLimit); }
    HIPCHK(hipGetLastError());
  }
  for (size_t i = 0; i < p->small.size(); ++i) {
    int rc = run_transform(&p->small_views[i], p->small[i].data, p->small[i].batch, st, p->dir < 0);
    if (rc) return rc;
  }
  return HENTT_OK;
}

// Plans made by hentt_ntt_batch, keyed by the job list (bounded cache).
std::mutex g_plan_mu;
std::map<std::vector<uint64_t>, hentt_batch_plan *> g_plans;

}  // namespace

extern "C" {

int hentt_batch_plan_create(const hentt_job *jobs, uint32_t njobs, int dir, hentt_batch_plan **out) {
  return plan_build(jobs, njobs, dir, out);
}

int hentt_batch_plan_set_grid(hentt_batch_plan *p, uint32_t workgroups) {
  if (!p) return HENTT_EINVAL;
  if (p->done) HIPCHK(hipEventSynchronize(p->done));
  p->grid = workgroups ? workgroups : (uint32_t)default_grid();
  return p->nunits ? plan_queues(p) : HENTT_OK;
}

int hentt_batch_plan_info(const hentt_batch_plan *p, uint32_t *units, uint32_t *tiles, uint32_t *grid) {
  if (!p) return HENTT_EINVAL;
  if (units) *units = p->nunits;
  if (tiles) *tiles = p->ntiles;
  if (grid) *grid = p->grid;
  return HENTT_OK;
}

int hentt_batch_plan_run(hentt_batch_plan *p, void *stream) {
  if (!p) return HENTT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  int rc = plan_launch(p, st);
  if (rc) return rc;
  HIPCHK(hipEventRecord(p->done, st));
  return HENTT_OK;
}

int hentt_batch_plan_status(hentt_batch_plan *p) {
  if (!p) return HENTT_EINVAL;
  if (!p->nunits) return HENTT_OK;
  HIPCHK(hipEventSynchronize(p->done));
  uint32_t h[BATCH_NQ + 1];
  HIPCHK(hipMemcpy(h, p->d_ctl, sizeof(h), hipMemcpyDeviceToHost));
  if (h[BATCH_NQ]) return HENTT_ETIMEOUT;
  for (uint32_t k = 0; k < BATCH_NQ; ++k)
    if (h[k] < p->qlen[k]) return HENTT_ETIMEOUT;  // a queue no workgroup served
  return HENTT_OK;
}

int hentt_batch_plan_destroy(hentt_batch_plan *p) {
  if (!p) return HENTT_EINVAL;
  plan_free(p);
  return HENTT_OK;
}

int hentt_batch_graph_create(hentt_batch_plan *p, hentt_graph **out) {
  if (!p || !out) return HENTT_EINVAL;
  hipStream_t cs = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hentt_graph *g = new (std::nothrow) hentt_graph();
  if (!g) {
    (void)hipStreamDestroy(cs);
    return HENTT_ENOMEM;
  }
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  int rc = HENTT_OK;
  if (e == hipSuccess) rc = plan_launch(p, cs);
  hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess && !rc) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess || rc) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    if (rc) return rc;
    return hip_fail(e);
  }
  *out = g;
  return HENTT_OK;
}

int hentt_graph_launch(hentt_graph *g, void *stream) {
  if (!g) return HENTT_EINVAL;
  HIPCHK(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return HENTT_OK;
}

int hentt_graph_destroy(hentt_graph *g) {
  if (!g) return HENTT_EINVAL;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return HENTT_OK;
}

int hentt_ntt_batch(const hentt_job *jobs, uint32_t njobs, int dir, void *stream) {
  if (!jobs || njobs == 0 || (dir != 1 && dir != -1)) return HENTT_EINVAL;
  std::vector<uint64_t> key;
  key.push_back((uint64_t)(int64_t)dir);
  for (uint32_t j = 0; j < njobs; ++j) {
    key.push_back((uint64_t)(uintptr_t)jobs[j].data);
    key.push_back((uint64_t)(uintptr_t)jobs[j].t->s);
    key.push_back(((uint64_t)jobs[j].limbs << 32) | jobs[j].batch);
  }
  hentt_batch_plan *p = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) p = it->second;
  }
  if (!p) {
    int rc = plan_build(jobs, njobs, dir, &p);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (g_plans.size() >= 16) {  // evict one plan (waits for its last run)
      plan_free(g_plans.begin()->second);
      g_plans.erase(g_plans.begin());
    }
    g_plans[key] = p;
  }
  return hentt_batch_plan_run(p, stream);
}

int hentt_prof_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto &r : g_prof) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.clear();
  g_prof_agg.clear();
  g_prof_on = on != 0;
  return HENTT_OK;
}

int hentt_prof_count(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto &r : g_prof) {
    float ms = 0;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return hip_fail(e);
    bool found = false;
    for (auto &g : g_prof_agg)
      if (g.name == r.name) {
        g.ms += ms;
        g.n += 1;
        found = true;
      }
    if (!found) g_prof_agg.push_back({r.name, (double)ms, 1});
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.clear();
  return (int)g_prof_agg.size();
}

int hentt_prof_get(uint32_t i, char *name, uint32_t name_len, double *total_ms, uint32_t *launches) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (i >= g_prof_agg.size() || !name || name_len == 0) return HENTT_EINVAL;
  snprintf(name, name_len, "%s", g_prof_agg[i].name.c_str());
  if (total_ms) *total_ms = g_prof_agg[i].ms;
  if (launches) *launches = g_prof_agg[i].n;
  return HENTT_OK;
}

}  // extern "C"
