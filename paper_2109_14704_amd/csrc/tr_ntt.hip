// Dispatch of the plain batched transforms (hentt_ntt_fwd / hentt_ntt_inv)
// and of the kernel-instance choices the autotuner selects between.
//
// Every N has a list of compiled instances ("candidates"): a whole transform
// per workgroup (one HBM round trip), or a column pass of EC stages followed
// by blocks of 2^(log_n - EC) words with 2^E words per lane.  Candidate 0 is
// the default; the autotuner may select another per (operation, N, shape
// class), where the shape class groups the number of (batch entry, limb)
// units of a call.
#include "runtime.hpp"

namespace hentt_rt {
namespace {

// Whole transform of one (batch entry, limb) per workgroup, 16 words per lane.
template <int LOGN>
void launch_whole(const hentt_tables *t, uint64_t *x, uint32_t batch, bool inv, hipStream_t st) {
  const uint32_t L = t->limbs, units = batch * L;
  if (!inv) {
    LaunchTimer lt_("k_fwd_whole", LOGN, st);
    hipLaunchKernelGGL((k_fwd_whole<LOGN, 4>), dim3(units), dim3(1 << (LOGN - 4)), 0, st, x, t->s->d_tw, t->s->d_lc,
                       batch, L);
  } else {
    LaunchTimer lt_("k_inv_whole", LOGN, st);
    hipLaunchKernelGGL((k_inv_whole<LOGN, 4>), dim3(units), dim3(1 << (LOGN - 4)), 0, st, x, t->s->d_tw, t->s->d_lc,
                       batch, L);
  }
}

// Column pass of EC stages and block pass on 2^(LOGN - EC) words, 2^E per lane.
template <int LOGN, int EC, int E>
void launch_two_pass(const hentt_tables *t, uint64_t *x, uint32_t batch, bool inv, hipStream_t st) {
  constexpr int B = LOGN - EC;
  const Tw *tw = t->s->d_tw;
  const LimbConst *lc = t->s->d_lc;
  const uint32_t L = t->limbs, units = batch * L;
  const dim3 gcols(units * ((1u << (LOGN - EC)) / (256 * ColCpl<EC>::value)));
  if (!inv) {
    {
      LaunchTimer lt_("k_cols_fwd", LOGN, st);
      hipLaunchKernelGGL((k_cols<LOGN, EC, false>), gcols, dim3(256), 0, st, col_args(x, (uint64_t)L << LOGN), tw, lc,
                         batch, L);
    }
    LaunchTimer lt_("k_fwd_blocks", LOGN, st);
    hipLaunchKernelGGL((k_fwd_blocks<LOGN, B, E>), dim3(units << (LOGN - B)), dim3(1 << (B - E)), 0, st, x, tw, lc,
                       batch, L);
  } else {
    {
      LaunchTimer lt_("k_inv_blocks", LOGN, st);
      hipLaunchKernelGGL((k_inv_blocks<LOGN, B, E>), dim3(units << (LOGN - B)), dim3(1 << (B - E)), 0, st, x, tw, lc,
                         batch, L);
    }
    LaunchTimer lt_("k_cols_inv", LOGN, st);
    hipLaunchKernelGGL((k_cols<LOGN, EC, true>), gcols, dim3(256), 0, st, col_args(x, (uint64_t)L << LOGN), tw, lc,
                       batch, L);
  }
}

typedef void (*tr_fn)(const hentt_tables *, uint64_t *, uint32_t, bool, hipStream_t);
struct TrCand {
  tr_fn fn;
  uint32_t ec;        // column stages (0: whole)
  const char *desc;
};

// Candidate lists per log_n (candidate 0 = default).  Defaults (measured): a
// whole transform up to 2^14; five column stages at 2^15 and 2^16, so that the
// HBM-bound column pass takes stages off the ALU-bound block pass (10-19%
// faster products than three or four stages); four at 2^17.
#define W(n) {launch_whole<n>, 0, "one kernel per (batch entry, limb), block words per lane 2^4"}
#define T(n, ec, e) {launch_two_pass<n, ec, e>, ec, "column stages " #ec ", block words per lane 2^" #e}
const TrCand c6[] = {W(6)}, c7[] = {W(7)}, c8[] = {W(8)}, c9[] = {W(9)}, c10[] = {W(10)}, c11[] = {W(11)},
             c12[] = {W(12)};
const TrCand c13[] = {W(13), T(13, 1, 4)};
const TrCand c14[] = {T(14, 2, 3), W(14), T(14, 2, 4)};
const TrCand c15[] = {T(15, 5, 4), T(15, 4, 4), T(15, 3, 4), T(15, 5, 3), T(15, 4, 3)};
const TrCand c16[] = {T(16, 5, 3), T(16, 5, 4), T(16, 4, 4), T(16, 4, 3)};
const TrCand c17[] = {T(17, 5, 3), T(17, 5, 4), T(17, 4, 4)};
#undef W
#undef T
struct TrList {
  const TrCand *c;
  uint32_t n;
};
#define L_(a) {a, (uint32_t)(sizeof(a) / sizeof(a[0]))}
const TrList k_tr[] = {L_(c6), L_(c7), L_(c8), L_(c9), L_(c10), L_(c11), L_(c12), L_(c13), L_(c14), L_(c15), L_(c16), L_(c17)};
#undef L_

}  // namespace

// ------------------------------------------------------------ tuned choices
std::atomic<uint8_t> g_choice[kTuneOps][HENTT_LOG_N_MAX + 1][kTuneClasses];

uint32_t tune_class(uint64_t units) { return units < 64 ? 0u : units < 1024 ? 1u : 2u; }

uint32_t tune_choice(int op, uint32_t log_n, uint64_t units) {
  return g_choice[op][log_n][tune_class(units)].load(std::memory_order_relaxed);
}

uint32_t transform_candidates(uint32_t log_n) { return k_tr[log_n - HENTT_LOG_N_MIN].n; }

const char *transform_describe(uint32_t log_n, uint32_t choice) { return k_tr[log_n - HENTT_LOG_N_MIN].c[choice].desc; }

uint32_t transform_cols(uint32_t log_n, uint32_t choice) { return k_tr[log_n - HENTT_LOG_N_MIN].c[choice].ec; }

int run_transform(const hentt_tables *t, uint64_t *x, uint32_t batch, hipStream_t st, bool inv) {
  const uint32_t ln = t->s->log_n;
  const TrList &l = k_tr[ln - HENTT_LOG_N_MIN];
  uint32_t c = tune_choice(inv ? HENTT_OP_INV : HENTT_OP_FWD, ln, (uint64_t)batch * t->limbs);
  if (c >= l.n) c = 0;
  l.c[c].fn(t, x, batch, inv, st);
  HIPCHK(hipGetLastError());
  return HENTT_OK;
}

void stage_split(uint32_t log_n, uint32_t *transform_cols, uint32_t *product_cols) {
  *transform_cols = k_tr[log_n - HENTT_LOG_N_MIN].c[0].ec;
  *product_cols = product_default_cols(log_n);
}

}  // namespace hentt_rt
