// Dispatch of the ciphertext tensor product (section II-A, Mul) at every N.
#include "prod_launch.hpp"

namespace hentt_rt {
namespace {
#define TEN_ENTRY(n) launch_prod<n, PROD_TENSOR>,
const prod_fn k_ten_table[] = {HENTT_SIZES(TEN_ENTRY)};
}  // namespace

void launch_prod_tensor(uint32_t log_n, const hentt_tables *t, const ProdArgs &pa, uint32_t batch, bool in_coeff,
                        bool out_coeff, uint64_t *ws, hipStream_t st) {
  k_ten_table[log_n - HENTT_LOG_N_MIN](t, pa, batch, in_coeff, out_coeff, ws, st);
}

}  // namespace hentt_rt
