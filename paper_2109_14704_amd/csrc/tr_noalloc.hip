// hentt_ct_tensor_noalloc: the ciphertext tensor product for callers that
// cannot allocate device memory (code under graph capture, tight serving
// loops).  Its only scratch -- the forward column pass's workspace of a
// two-pass product -- lives in a static device array, one copy per GPU,
// looked up once per device with hipGetSymbolAddress.
#include "runtime.hpp"

// Workspace of the two-pass tensor product: 4 batch limbs N words (the four
// input polynomials after the forward column pass).  64 MiB per GPU.
static __device__ __align__(256) uint64_t scratch[HENTT_NOALLOC_SCRATCH_WORDS];

namespace hentt_rt {
namespace {

constexpr uint64_t kScratchWords = HENTT_NOALLOC_SCRATCH_WORDS;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint64_t *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` per device

// The device address of this device's copy of `scratch` (the host-side name
// is only a stand-in and must never be passed to a kernel).
int scratch_ptr(uint64_t **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return HENTT_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return HENTT_EHIP;
    g_scratch_ptr[dev] = (uint64_t *)p;
  }
  *out = g_scratch_ptr[dev];
  return HENTT_OK;
}

}  // namespace
}  // namespace hentt_rt

using namespace hentt_rt;

extern "C" int hentt_ct_tensor_noalloc(const hentt_tables *t, const uint64_t *c, const uint64_t *d, uint64_t *out,
                                       uint32_t batch, uint32_t flags, void *stream) {
  if (!t || !c || !d || !out || batch == 0 || (flags & ~3u)) return HENTT_EINVAL;
  const uint32_t ln = t->s->log_n;
  const uint64_t NL = (uint64_t)t->limbs << ln;
  const uintptr_t o0 = (uintptr_t)out, o1 = o0 + (uintptr_t)(3 * NL * batch * 8);
  const uintptr_t c0 = (uintptr_t)c, c1 = c0 + (uintptr_t)(2 * NL * batch * 8);
  const uintptr_t d0 = (uintptr_t)d, d1 = d0 + (uintptr_t)(2 * NL * batch * 8);
  if ((o0 < c1 && c0 < o1) || (o0 < d1 && d0 < o1)) return HENTT_EINVAL;
  const bool in_coeff = !(flags & HENTT_IN_NTT), out_coeff = !(flags & HENTT_OUT_NTT);
  const ProdCand &cand = prod_select(PROD_TENSOR, ln, (uint64_t)batch * t->limbs, in_coeff && out_coeff);
  uint64_t *ws = nullptr;
  if (in_coeff && cand.pec > 0) {
    if (4 * NL * (uint64_t)batch > kScratchWords) return HENTT_ESCRATCH;
    int rc = scratch_ptr(&ws);
    if (rc) return rc;
  }
  ProdArgs pa{};
  pa.in[0] = c;
  pa.in[1] = c + NL;
  pa.in[2] = d;
  pa.in[3] = d + NL;
  for (int o = 0; o < 3; ++o) pa.out[o] = out + o * NL;
  pa.in_sb = 2 * NL;
  pa.out_sb = 3 * NL;
  hipStream_t st = (hipStream_t)stream;
  {
    NoTimerScope quiet;  // launch timing would create events
    cand.fn(t, pa, batch, in_coeff, out_coeff, ws, st);
  }
  HIPCHK(hipGetLastError());
  return HENTT_OK;
}
