// Internal runtime of libhentt shared by its translation units: table
// storage, the workspace pool, launch timing, the launch plan per N and the
// dispatch entry points of each kernel family.  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hentt.h"
#include "ntt_kernels.hpp"

namespace hentt {
struct RsLimb;
struct KsLimb;
}  // namespace hentt

namespace hentt_rt {
using namespace hentt;

extern thread_local int g_last_hip;

inline int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return HENTT_EHIP;
}
#define HIPCHK(x)                              \
  do {                                         \
    hipError_t e_ = (x);                       \
    if (e_ != hipSuccess) return hip_fail(e_); \
  } while (0)

// ------------------------------------------------------------ table storage
// Device tables of one modulus chain at one N, shared by every handle (table
// or level view) and by the batch plans that point into them; freed when the
// last reference goes.
struct Storage {
  std::atomic<int> refs{1};
  uint32_t log_n = 0, limbs = 0;
  Tw *d_tw = nullptr;          // [limbs][2][N]
  LimbConst *d_lc = nullptr;   // [limbs]
  LimbConst *d_lcm = nullptr;  // [limbs] the same with N^-1 R mod q for N^-1 (after Montgomery products)
  MontLimb *d_mont = nullptr;  // [limbs] Montgomery constants
  std::vector<uint64_t> moduli;
  int device = 0;
  std::mutex rs_mu;                  // rescale and key-switch constants per level, made on first use
  std::map<uint32_t, RsLimb *> rs;   // per level (limb count)
  std::map<uint32_t, KsLimb *> ks;   // per level (limb count, the last one the special prime)
};
void retain(Storage *s);
void release(Storage *s);

// ------------------------------------------------------------ workspace pool
// Device buffers reused by capacity (the memory cache of section III-C-1); see
// hentt.hip.  pool_put returns a buffer right after the launches that use it
// are enqueued on `stream`: later users of the same entry enqueue on the same
// stream, so stream order keeps reuse after completion.
int pool_get(size_t bytes, hipStream_t stream, void **out);
void pool_put(void *p);

// ------------------------------------------------------------ launch timing
// While enabled (hentt_prof_enable), every launch is bracketed by HIP events
// recorded on its stream and filed under "name<log_n>".
// A NoTimerScope turns the timing off on its thread (entry points that must
// not create events).
extern std::atomic<bool> g_prof_on;
extern thread_local bool g_timer_off;
void prof_record(const char *name, int log_n, hipEvent_t a, hipEvent_t b);
struct NoTimerScope {
  bool old;
  NoTimerScope() : old(g_timer_off) { g_timer_off = true; }
  ~NoTimerScope() { g_timer_off = old; }
};
struct LaunchTimer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t st;
  const char *name;
  int ln;
  LaunchTimer(const char *nm, int log_n, hipStream_t s) : st(s), name(nm), ln(log_n) {
    if (!g_timer_off && g_prof_on.load(std::memory_order_relaxed) && hipEventCreate(&a) == hipSuccess &&
        hipEventCreate(&b) == hipSuccess)
      (void)hipEventRecord(a, st);
  }
  ~LaunchTimer() {
    if (a && b) {
      (void)hipEventRecord(b, st);
      prof_record(name, ln, a, b);
    }
  }
};

// ------------------------------------------------------------ roctx ranges
// With HENTT_ROCTX=1 in the environment (read once), the compute entry points
// are bracketed by roctx ranges named after them (rocprofv3 --marker-trace);
// the roctx library is opened on first use, and without it nothing happens.
struct ApiRange {
  bool on;
  explicit ApiRange(const char *name);
  ~ApiRange();
};

// ------------------------------------------------------------ launch plans
// Every operation has, per N, a list of compiled kernel instances (stage
// split, words per lane); instance 0 is the measured default and the
// autotuner may select another per (operation, N, shape class).  The shape
// class groups the (batch entry, limb) units of a call: < 64, < 1024, more.
constexpr int kTuneOps = 4;      // HENTT_OP_FWD, _INV, _POLYMUL, _TENSOR
constexpr int kTuneClasses = 3;
extern std::atomic<uint8_t> g_choice[kTuneOps][HENTT_LOG_N_MAX + 1][kTuneClasses];
uint32_t tune_class(uint64_t units);
uint32_t tune_choice(int op, uint32_t log_n, uint64_t units);
uint32_t transform_candidates(uint32_t log_n);
const char *transform_describe(uint32_t log_n, uint32_t choice);
uint32_t transform_cols(uint32_t log_n, uint32_t choice);

typedef void (*prod_fn)(const hentt_tables *, const ProdArgs &, uint32_t, bool, bool, uint64_t *, hipStream_t);
struct ProdCand {
  prod_fn fn;          // launch sequence (ws: the forward column pass's workspace, if pec > 0)
  uint32_t pec;        // column stages of a two-pass product (0: one kernel)
  const char *desc;
};
const ProdCand *prod_candidates(int mode, uint32_t log_n, uint32_t *count);
const ProdCand *tensor_candidates(uint32_t log_n, uint32_t *count);
// the instance a call runs: the tuned one for the fused coefficient-to-
// coefficient form, the default otherwise
const ProdCand &prod_select(int mode, uint32_t log_n, uint64_t units, bool fused);
uint32_t product_default_cols(uint32_t log_n);

inline ColArgs col_args(uint64_t *x, uint64_t sb) {
  ColArgs a{};
  a.src[0] = x;
  a.dst[0] = x;
  a.src_sb = a.dst_sb = sb;
  return a;
}

#define HENTT_SIZES(M) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15) M(16) M(17)

// ------------------------------------------------------------ dispatch
// tr_ntt.hip
int run_transform(const hentt_tables *t, uint64_t *x, uint32_t batch, hipStream_t st, bool inv);
void stage_split(uint32_t log_n, uint32_t *transform_cols, uint32_t *product_cols);
// tr_prod_mul.hip / tr_prod_tensor.hip: products, fused with the transforms
// when in_coeff / out_coeff; the workspace comes from the pool.
int run_prod(const hentt_tables *t, int mode, const ProdArgs &pa, uint32_t batch, bool in_coeff, bool out_coeff,
             hipStream_t st);
// tr_he.hip
int run_rescale(const hentt_tables *t, const uint64_t *c, uint64_t *out, uint32_t batch, bool ntt, hipStream_t st);
int run_relin(const hentt_tables *t, const uint64_t *c, const uint64_t *ksk, uint64_t *out, uint32_t batch,
              hipStream_t st);
int run_matmul(const hentt_tables *t, const uint64_t *A, const uint64_t *B, uint64_t *C, uint32_t m, uint32_t n,
               uint32_t k, hipStream_t st);
// tr_ladder.hip
int run_fwd_variant(const hentt_tables *t, uint64_t *x, uint32_t batch, int variant, hipStream_t st);

}  // namespace hentt_rt

struct hentt_tables {
  hentt_rt::Storage *s;
  uint32_t limbs;  // <= s->limbs
};
