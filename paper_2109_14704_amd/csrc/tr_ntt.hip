// Dispatch of the plain batched transforms (hentt_ntt_fwd / hentt_ntt_inv):
// whole-transform kernels up to N = 2^14, column pass + block pass above.
#include "runtime.hpp"

namespace hentt_rt {
namespace {

template <int LOGN>
void launch_fwd(const hentt_tables *t, uint64_t *x, uint32_t batch, hipStream_t st) {
  const Tw *tw = t->s->d_tw;
  const LimbConst *lc = t->s->d_lc;
  const uint32_t L = t->limbs;
  const uint32_t units = batch * L;
  using P = Plan<LOGN>;
  if constexpr (P::WHOLE) {
    LaunchTimer lt_("k_fwd_whole", LOGN, st);
    hipLaunchKernelGGL((k_fwd_whole<LOGN, 4>), dim3(units), dim3(1 << (LOGN - 4)), 0, st, x, tw, lc, batch, L);
  } else {
    {
      LaunchTimer lt_("k_cols_fwd", LOGN, st);
      hipLaunchKernelGGL((k_cols<LOGN, P::EC, false>), dim3(units * ((1u << (LOGN - P::EC)) / (256 * ColCpl<P::EC>::value))),
                         dim3(256), 0, st, col_args(x, (uint64_t)L << LOGN), tw, lc, batch, L);
    }
    LaunchTimer lt_("k_fwd_blocks", LOGN, st);
    hipLaunchKernelGGL((k_fwd_blocks<LOGN, P::B, 4>), dim3(units << (LOGN - P::B)), dim3(1 << (P::B - 4)), 0, st, x,
                       tw, lc, batch, L);
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
    LaunchTimer lt_("k_inv_whole", LOGN, st);
    hipLaunchKernelGGL((k_inv_whole<LOGN, 4>), dim3(units), dim3(1 << (LOGN - 4)), 0, st, x, tw, lc, batch, L);
  } else {
    {
      LaunchTimer lt_("k_inv_blocks", LOGN, st);
      hipLaunchKernelGGL((k_inv_blocks<LOGN, P::B, 4>), dim3(units << (LOGN - P::B)), dim3(1 << (P::B - 4)), 0, st,
                         x, tw, lc, batch, L);
    }
    LaunchTimer lt_("k_cols_inv", LOGN, st);
    hipLaunchKernelGGL((k_cols<LOGN, P::EC, true>), dim3(units * ((1u << (LOGN - P::EC)) / (256 * ColCpl<P::EC>::value))),
                       dim3(256), 0, st, col_args(x, (uint64_t)L << LOGN), tw, lc, batch, L);
  }
}

typedef void (*launch_fn)(const hentt_tables *, uint64_t *, uint32_t, hipStream_t);
#define FWD_ENTRY(n) launch_fwd<n>,
#define INV_ENTRY(n) launch_inv<n>,
const launch_fn k_fwd_table[] = {HENTT_SIZES(FWD_ENTRY)};
const launch_fn k_inv_table[] = {HENTT_SIZES(INV_ENTRY)};

template <int LOGN> void split_of(uint32_t *ec, uint32_t *pec) {
  *ec = Plan<LOGN>::WHOLE ? 0u : (uint32_t)Plan<LOGN>::EC;
  *pec = Plan<LOGN>::PROD_WHOLE ? 0u : (uint32_t)Plan<LOGN>::PEC;
}
typedef void (*split_fn)(uint32_t *, uint32_t *);
#define SPLIT_ENTRY(n) split_of<n>,
const split_fn k_split_table[] = {HENTT_SIZES(SPLIT_ENTRY)};

}  // namespace

int run_transform(const hentt_tables *t, uint64_t *x, uint32_t batch, hipStream_t st, bool inv) {
  const int ln = (int)t->s->log_n;
  (inv ? k_inv_table : k_fwd_table)[ln - HENTT_LOG_N_MIN](t, x, batch, st);
  HIPCHK(hipGetLastError());
  return HENTT_OK;
}

void stage_split(uint32_t log_n, uint32_t *transform_cols, uint32_t *product_cols) {
  k_split_table[log_n - HENTT_LOG_N_MIN](transform_cols, product_cols);
}

}  // namespace hentt_rt
