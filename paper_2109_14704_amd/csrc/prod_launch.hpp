// Launch sequence of the products (dyadic product, ciphertext tensor), fused
// with the forward transforms of coefficient-domain inputs and the inverse
// transforms of coefficient-domain outputs.  Included by the two product
// translation units, one per product kind.
#pragma once
#include "runtime.hpp"

namespace hentt_rt {

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
  const char *kname = MODE == PROD_MUL ? "k_prod_mul" : "k_prod_tensor";
  using P = Plan<LOGN>;
  if (!in_coeff && !out_coeff) {
    const uint32_t tiles = LOGN > 11 ? (1u << (LOGN - 11)) : 1u;
    LaunchTimer lt_(MODE == PROD_MUL ? "k_elem_mul" : "k_elem_tensor", LOGN, st);
    hipLaunchKernelGGL((k_elem<MODE>), dim3(units * tiles), dim3(256), 0, st, pa, lc, batch, L, (uint32_t)LOGN, tiles);
    return;
  }
  constexpr int PE = ProdE<MODE>::E;
  if constexpr (P::PROD_WHOLE) {
    const dim3 g(units), blk(1 << (LOGN - PE));
    LaunchTimer lt_(kname, LOGN, st);
    if (in_coeff && out_coeff)
      hipLaunchKernelGGL((k_prod<LOGN, LOGN, PE, MODE, true, true>), g, blk, 0, st, pa, tw, lc, mont, batch, L);
    else if (in_coeff)
      hipLaunchKernelGGL((k_prod<LOGN, LOGN, PE, MODE, true, false>), g, blk, 0, st, pa, tw, lc, mont, batch, L);
    else
      hipLaunchKernelGGL((k_prod<LOGN, LOGN, PE, MODE, false, true>), g, blk, 0, st, pa, tw, lc, mont, batch, L);
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
      LaunchTimer lt_("k_cols_fwd", LOGN, st);
      hipLaunchKernelGGL((k_cols<LOGN, EC, false>), dim3(NIN * units * ((1u << (LOGN - EC)) / (256 * ColCpl<EC>::value))),
                         dim3(256), 0, st, ca, tw, lc, batch, L);
    }
    {
      const dim3 g(units << (LOGN - B)), blk(1 << (B - PE));
      LaunchTimer lt_(kname, LOGN, st);
      if (in_coeff && out_coeff)
        hipLaunchKernelGGL((k_prod<LOGN, B, PE, MODE, true, true>), g, blk, 0, st, pb, tw, lc, mont, batch, L);
      else if (in_coeff)
        hipLaunchKernelGGL((k_prod<LOGN, B, PE, MODE, true, false>), g, blk, 0, st, pb, tw, lc, mont, batch, L);
      else
        hipLaunchKernelGGL((k_prod<LOGN, B, PE, MODE, false, true>), g, blk, 0, st, pb, tw, lc, mont, batch, L);
    }
    if (out_coeff) {
      ColArgs ca{};
      for (int o = 0; o < NOUT; ++o) ca.src[o] = ca.dst[o] = pa.out[o];
      ca.src_sb = ca.dst_sb = pa.out_sb;
      LaunchTimer lt_("k_cols_inv", LOGN, st);
      hipLaunchKernelGGL((k_cols<LOGN, EC, true>), dim3(NOUT * units * ((1u << (LOGN - EC)) / (256 * ColCpl<EC>::value))),
                         dim3(256), 0, st, ca, tw, lc, batch, L);
    }
  }
}

typedef void (*prod_fn)(const hentt_tables *, const ProdArgs &, uint32_t, bool, bool, uint64_t *, hipStream_t);

}  // namespace hentt_rt
