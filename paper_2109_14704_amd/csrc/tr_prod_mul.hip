// Compiled instances of the dyadic product and the fused negacyclic polymul at
// every N (candidate 0 is the default and serves every domain combination),
// and the common entry of both product kinds.
#include "prod_launch.hpp"

namespace hentt_rt {
namespace {
#define D(n, pec, e) {launch_prod_cfg<n, PROD_MUL, pec, e, true>, pec, "column stages " #pec ", block words per lane 2^" #e}
#define C(n, pec, e) {launch_prod_cfg<n, PROD_MUL, pec, e, false>, pec, "column stages " #pec ", block words per lane 2^" #e}
const ProdCand m6[] = {D(6, 0, 4)}, m7[] = {D(7, 0, 4)}, m8[] = {D(8, 0, 4)}, m9[] = {D(9, 0, 4)},
               m10[] = {D(10, 0, 4)}, m11[] = {D(11, 0, 4)}, m12[] = {D(12, 0, 4)};
const ProdCand m13[] = {D(13, 0, 4), C(13, 1, 4)};
const ProdCand m14[] = {D(14, 2, 3), C(14, 2, 4), C(14, 3, 4)};
const ProdCand m15[] = {D(15, 5, 3), C(15, 5, 4), C(15, 4, 4), C(15, 4, 3)};
const ProdCand m16[] = {D(16, 5, 3), C(16, 5, 4), C(16, 4, 4)};
const ProdCand m17[] = {D(17, 5, 4), C(17, 4, 4)};
#undef D
#undef C
const ProdList k_mul[] = {HENTT_PROD_LIST(m6),  HENTT_PROD_LIST(m7),  HENTT_PROD_LIST(m8),  HENTT_PROD_LIST(m9),
                          HENTT_PROD_LIST(m10), HENTT_PROD_LIST(m11), HENTT_PROD_LIST(m12), HENTT_PROD_LIST(m13),
                          HENTT_PROD_LIST(m14), HENTT_PROD_LIST(m15), HENTT_PROD_LIST(m16), HENTT_PROD_LIST(m17)};
}  // namespace

const ProdCand *prod_candidates(int mode, uint32_t log_n, uint32_t *count) {
  if (mode == PROD_TENSOR) return tensor_candidates(log_n, count);
  const ProdList &l = k_mul[log_n - HENTT_LOG_N_MIN];
  *count = l.n;
  return l.c;
}

uint32_t product_default_cols(uint32_t log_n) { return k_mul[log_n - HENTT_LOG_N_MIN].c[0].pec; }

const ProdCand &prod_select(int mode, uint32_t log_n, uint64_t units, bool fused) {
  uint32_t n = 0;
  const ProdCand *c = prod_candidates(mode, log_n, &n);
  if (!fused) return c[0];  // the NTT-domain forms run the default instance
  uint32_t i = tune_choice(mode == PROD_MUL ? HENTT_OP_POLYMUL : HENTT_OP_TENSOR, log_n, units);
  return c[i < n ? i : 0];
}

int run_prod(const hentt_tables *t, int mode, const ProdArgs &pa, uint32_t batch, bool in_coeff, bool out_coeff,
             hipStream_t st) {
  const uint32_t ln = t->s->log_n;
  const int nin = mode == PROD_MUL ? 2 : 4;
  const uint64_t NL = (uint64_t)t->limbs << ln;
  const ProdCand &c = prod_select(mode, ln, (uint64_t)batch * t->limbs, in_coeff && out_coeff);
  void *ws = nullptr;
  if (in_coeff && c.pec > 0) {
    int rc = pool_get((size_t)nin * batch * NL * 8ull, st, &ws);
    if (rc) return rc;
  }
  c.fn(t, pa, batch, in_coeff, out_coeff, (uint64_t *)ws, st);
  hipError_t e = hipGetLastError();
  if (ws) pool_put(ws);
  if (e != hipSuccess) return hip_fail(e);
  return HENTT_OK;
}

}  // namespace hentt_rt
