// Dispatch of the dyadic product and the fused negacyclic polymul at every N,
// and the common entry of both product kinds (workspace from the pool).
#include "prod_launch.hpp"

namespace hentt_rt {
namespace {
#define MUL_ENTRY(n) launch_prod<n, PROD_MUL>,
const prod_fn k_mul_table[] = {HENTT_SIZES(MUL_ENTRY)};
}  // namespace

bool prod_needs_ws(uint32_t log_n) { return log_n > 12; }  // !Plan<log_n>::PROD_WHOLE

int run_prod(const hentt_tables *t, int mode, const ProdArgs &pa, uint32_t batch, bool in_coeff, bool out_coeff,
             hipStream_t st) {
  const uint32_t ln = t->s->log_n;
  const int nin = mode == PROD_MUL ? 2 : 4;
  const uint64_t NL = (uint64_t)t->limbs << ln;
  void *ws = nullptr;
  if (in_coeff && prod_needs_ws(ln)) {
    int rc = pool_get((size_t)nin * batch * NL * 8ull, st, &ws);
    if (rc) return rc;
  }
  if (mode == PROD_MUL) k_mul_table[ln - HENTT_LOG_N_MIN](t, pa, batch, in_coeff, out_coeff, (uint64_t *)ws, st);
  else launch_prod_tensor(ln, t, pa, batch, in_coeff, out_coeff, (uint64_t *)ws, st);
  hipError_t e = hipGetLastError();
  if (ws) pool_put(ws);
  if (e != hipSuccess) return hip_fail(e);
  return HENTT_OK;
}

}  // namespace hentt_rt
