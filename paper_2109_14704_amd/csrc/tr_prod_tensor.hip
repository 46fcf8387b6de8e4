// Compiled instances of the ciphertext tensor product (section II-A, Mul) at
// every N; candidate 0 is the default and serves every domain combination.
#include "prod_launch.hpp"

namespace hentt_rt {
namespace {
#define D(n, pec, e) {launch_prod_cfg<n, PROD_TENSOR, pec, e, true>, pec, "column stages " #pec ", block words per lane 2^" #e}
#define C(n, pec, e) {launch_prod_cfg<n, PROD_TENSOR, pec, e, false>, pec, "column stages " #pec ", block words per lane 2^" #e}
const ProdCand t6[] = {D(6, 0, 3)}, t7[] = {D(7, 0, 3)}, t8[] = {D(8, 0, 3)}, t9[] = {D(9, 0, 3)},
               t10[] = {D(10, 0, 3)}, t11[] = {D(11, 0, 3)}, t12[] = {D(12, 0, 3)};
const ProdCand t13[] = {D(13, 1, 3), C(13, 2, 3)};
const ProdCand t14[] = {D(14, 3, 3), C(14, 2, 3)};
const ProdCand t15[] = {D(15, 5, 2), C(15, 5, 3), C(15, 4, 3)};
const ProdCand t16[] = {D(16, 5, 3), C(16, 4, 3), C(16, 5, 2)};
const ProdCand t17[] = {D(17, 5, 3), C(17, 5, 2)};
#undef D
#undef C
const ProdList k_ten[] = {HENTT_PROD_LIST(t6),  HENTT_PROD_LIST(t7),  HENTT_PROD_LIST(t8),  HENTT_PROD_LIST(t9),
                          HENTT_PROD_LIST(t10), HENTT_PROD_LIST(t11), HENTT_PROD_LIST(t12), HENTT_PROD_LIST(t13),
                          HENTT_PROD_LIST(t14), HENTT_PROD_LIST(t15), HENTT_PROD_LIST(t16), HENTT_PROD_LIST(t17)};
}  // namespace

const ProdCand *tensor_candidates(uint32_t log_n, uint32_t *count) {
  const ProdList &l = k_ten[log_n - HENTT_LOG_N_MIN];
  *count = l.n;
  return l.c;
}

}  // namespace hentt_rt
