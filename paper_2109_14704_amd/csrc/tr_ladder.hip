// The kernel-design ladder of the forward transform (section III-B and the
// NTT evaluation of section IV): reference designs timed against the
// library's kernels, all computing the same transform.
#include "runtime.hpp"

namespace hentt {
// ------------------------------------------------- design-ladder kernels --
// Reference points for the kernel-design ladder of section III-B, not used by
// the hot path.  k_naive_stage is the paper's naive radix-2 baseline: one
// butterfly per lane and one launch per stage, every stage a round trip of
// the whole batch through global memory (same butterfly arithmetic as the
// other kernels).  Stage s pairs j with j + N/2^(s+1) and uses
// psi_rev[2^s + j / (N/2^s)].  k_reduce8q is its separate last-round
// reduction from [0, 8q) to [0, q).
__global__ __launch_bounds__(256) void k_naive_stage(uint64_t *__restrict__ x, const Tw *__restrict__ tw,
                                                     const LimbConst *__restrict__ lc, uint32_t units,
                                                     uint32_t limbs, uint32_t logn, uint32_t s) {
  const uint64_t gid = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t lh = logn - 1;
  const uint64_t unit = gid >> lh;  // (batch entry, limb) polynomial
  if (unit >= units) return;
  const uint32_t i = (uint32_t)gid & ((1u << lh) - 1);
  const uint32_t limb = (uint32_t)(unit % limbs);
  const ModQ m = lc[limb].m;
  const uint32_t lt = lh - s;  // log2 of the gap
  const uint32_t grp = i >> lt;
  const uint32_t j = (grp << (lt + 1)) | (i & ((1u << lt) - 1));
  uint64_t *p = x + (unit << logn);
  const Tw w = tw[((size_t)limb << (logn + 1)) + (1u << s) + grp];
  uint64_t X = p[j], Y = p[j + (1u << lt)];
  ct_bfly(X, Y, w.w, w.ws, m);
  p[j] = X;
  p[j + (1u << lt)] = Y;
}

__global__ __launch_bounds__(256) void k_reduce8q(uint64_t *__restrict__ x, const LimbConst *__restrict__ lc,
                                                  uint64_t words, uint32_t limbs, uint32_t logn) {
  const uint64_t gid = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= words) return;
  x[gid] = reduce_8q(x[gid], lc[(uint32_t)((gid >> logn) % limbs)].m);
}

}  // namespace hentt

namespace hentt_rt {
namespace {

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

}  // namespace

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

}  // namespace hentt_rt
