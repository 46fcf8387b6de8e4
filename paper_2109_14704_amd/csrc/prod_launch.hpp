// Launch sequences of the products (dyadic product, ciphertext tensor), fused
// with the forward transforms of coefficient-domain inputs and the inverse
// transforms of coefficient-domain outputs, and their compiled instances
// ("candidates") for the autotuner.  Included by the two product translation
// units, one per product kind.
#pragma once
#include "runtime.hpp"

namespace hentt_rt {

// One product launch sequence at N = 2^LOGN: PEC = 0 runs the whole product
// in one kernel per (batch entry, limb); otherwise a forward column pass of
// PEC stages into the workspace, the fused block kernel on blocks of
// 2^(LOGN - PEC) words with 2^PE words per lane, and the inverse column pass
// in place on the outputs.  ALL_FLAGS: also the NTT-domain input / output
// forms (the default instance); tuned instances serve the fused
// coefficient-to-coefficient form only.
template <int LOGN, int MODE, int PEC, int PE, bool ALL_FLAGS>
void launch_prod_cfg(const hentt_tables *t, const ProdArgs &pa, uint32_t batch, bool in_coeff, bool out_coeff,
                     uint64_t *ws, hipStream_t st) {
  const Tw *tw = t->s->d_tw;
  // outputs going back to the coefficient domain take Montgomery products,
  // whose R^-1 the inverse transform's folded N^-1 R scaling cancels
  const LimbConst *lc = out_coeff ? t->s->d_lcm : t->s->d_lc;
  const MontLimb *mont = t->s->d_mont;
  const uint32_t L = t->limbs;
  const uint32_t units = batch * L;
  constexpr int NIN = ProdShape<MODE>::NIN, NOUT = ProdShape<MODE>::NOUT;
  constexpr int B = PEC ? LOGN - PEC : LOGN;
  const char *kname = MODE == PROD_MUL ? "k_prod_mul" : "k_prod_tensor";
  if constexpr (ALL_FLAGS) {
    if (!in_coeff && !out_coeff) {
      const uint32_t tiles = LOGN > 11 ? (1u << (LOGN - 11)) : 1u;
      LaunchTimer lt_(MODE == PROD_MUL ? "k_elem_mul" : "k_elem_tensor", LOGN, st);
      hipLaunchKernelGGL((k_elem<MODE>), dim3(units * tiles), dim3(256), 0, st, pa, lc, batch, L, (uint32_t)LOGN,
                         tiles);
      return;
    }
  }
  const uint64_t NL = (uint64_t)L << LOGN;
  ProdArgs pb = pa;
  if constexpr (PEC > 0) {
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
      hipLaunchKernelGGL((k_cols<LOGN, PEC, false>),
                         dim3(NIN * units * ((1u << (LOGN - PEC)) / (256 * ColCpl<PEC>::value))), dim3(256), 0, st,
                         ca, tw, lc, batch, L);
    }
  }
  {
    const dim3 g(units << (LOGN - B)), blk(1 << (B - PE));
    LaunchTimer lt_(kname, LOGN, st);
    if constexpr (ALL_FLAGS) {
      if (in_coeff && out_coeff)
        hipLaunchKernelGGL((k_prod<LOGN, B, PE, MODE, true, true>), g, blk, 0, st, pb, tw, lc, mont, batch, L);
      else if (in_coeff)
        hipLaunchKernelGGL((k_prod<LOGN, B, PE, MODE, true, false>), g, blk, 0, st, pb, tw, lc, mont, batch, L);
      else
        hipLaunchKernelGGL((k_prod<LOGN, B, PE, MODE, false, true>), g, blk, 0, st, pb, tw, lc, mont, batch, L);
    } else {
      hipLaunchKernelGGL((k_prod<LOGN, B, PE, MODE, true, true>), g, blk, 0, st, pb, tw, lc, mont, batch, L);
    }
  }
  if constexpr (PEC > 0) {
    if (out_coeff) {
      ColArgs ca{};
      for (int o = 0; o < NOUT; ++o) ca.src[o] = ca.dst[o] = pa.out[o];
      ca.src_sb = ca.dst_sb = pa.out_sb;
      LaunchTimer lt_("k_cols_inv", LOGN, st);
      hipLaunchKernelGGL((k_cols<LOGN, PEC, true>),
                         dim3(NOUT * units * ((1u << (LOGN - PEC)) / (256 * ColCpl<PEC>::value))), dim3(256), 0, st,
                         ca, tw, lc, batch, L);
    }
  }
}

struct ProdList {
  const ProdCand *c;
  uint32_t n;
};
#define HENTT_PROD_LIST(a) {a, (uint32_t)(sizeof(a) / sizeof(a[0]))}

}  // namespace hentt_rt
