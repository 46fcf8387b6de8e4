// Rescale RS (section II-A): drop the last prime qL of a level with rounding,
// c' = round(c / qL) mod q_i for the remaining limbs i.  With h = (qL - 1)/2
// and r = (c_L + h) mod qL (c_L the last limb's coefficient), the RNS form is
//   c'_i = (c_i - t_i) * qL^-1 mod q_i,   t_i = (r - h) mod q_i,
// and, the transforms being linear, the same holds in the NTT domain with
// t_i replaced by NTT_i(t_i): the last limb is inverse-transformed once, and
// for every remaining limb its t_i is forward-transformed modulo q_i with the
// reduction fused into the first load (prologue) and the subtraction and
// scaling fused into the last store (epilogue).
#pragma once
#include "ntt_kernels.hpp"

namespace hentt {

struct RsLimb {   // per remaining limb i of a level
  uint64_t mu;    // floor(2^64 / q_i)
  uint64_t nh;    // q_i - (h mod q_i)
  uint64_t w, ws; // qL^-1 mod q_i and its Shoup quotient
};

// t_i from the last limb's canonical coefficient x (mod qL), in [0, 3 q_i):
// s = (x + h) mod qL; s - floor-estimate(s / q_i) q_i is in [0, 2 q_i) (the
// estimate floor(s mu / 2^64) is short by at most one); adding nh subtracts h.
__device__ __forceinline__ uint64_t rs_prologue(uint64_t x, uint64_t qL, uint64_t h, const RsLimb &r, uint64_t q) {
  uint64_t s = x + h;
  s = s >= qL ? s - qL : s;
  return s - mulhi64(s, r.mu) * q + r.nh;
}

// (c - t) qL^-1 mod q for canonical c, t: canonical.
__device__ __forceinline__ uint64_t rs_epilogue(uint64_t c, uint64_t t, const RsLimb &r, const ModQ &m) {
  return reduce_4q(shoup(r.w, r.ws, c + m.q - t, m.nq), m);
}

struct RsArgs {
  const uint64_t *c;    // [batch][L + 1][N] input (NTT or coefficient domain)
  const uint64_t *tl;   // [batch][N] last limb in the coefficient domain (NTT path)
  uint64_t *out;        // [batch][L][N]
  const RsLimb *rs;     // [L]
  uint64_t qL, h;
  uint32_t batch, L;
};

// Unit u of a launch: output limb i of batch entry b, limb-major so that
// neighbouring workgroups share limb i's twiddles.
__device__ __forceinline__ void rs_unit(uint32_t u, uint32_t batch, uint32_t &b, uint32_t &i) {
  i = u / batch;
  b = u % batch;
}

// Whole transform per workgroup (N <= 2^14): prologue, forward rounds,
// canonical reduction, epilogue.
template <int LOGN, int E>
__global__ __launch_bounds__(1 << (LOGN - E)) void k_rs_whole(RsArgs a, const Tw *__restrict__ tw,
                                                               const LimbConst *__restrict__ lc) {
  __shared__ uint64_t lds[LdsSize<LOGN>::value];
  uint32_t b, i;
  rs_unit(blockIdx.x, a.batch, b, i);
  const ModQ m = lc[i].m;
  const RsLimb r = a.rs[i];
  const Tw *t = tw + (size_t)i * 2 * (1u << LOGN);
  const uint32_t tid = threadIdx.x;
  using F = FwdFirst<LOGN, E>;
  uint64_t v[1 << E];
  load_global<LOGN, E, F::LO, F::R>(v, a.tl + ((uint64_t)b << LOGN), RoundMap<LOGN, E, F::LO, F::R>::lane_part(tid));
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) v[s] = rs_prologue(v[s], a.qL, a.h, r, m.q);
  fwd_block_rounds<LOGN, E, F::LO, F::R>(v, LOGN, lds, tid, 0, t, m);
  reduce_fwd<E>(v, m, lc[i].mu, lc[i].k);
  uint64_t cv[1 << E];
  load_global_m0<LOGN, E>(cv, a.c + (((uint64_t)b * (a.L + 1) + i) << LOGN), lds, tid);
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) v[s] = rs_epilogue(cv[s], v[s], r, m);
  store_global_m0<LOGN, E>(v, a.out + (((uint64_t)b * a.L + i) << LOGN), lds, tid);
}

// Column pass (first EC forward stages) of t_i from the last limb, into out.
// Batch-entry-major order: the L units of one batch entry read the same
// last-limb columns one after another, so all but the first read hit the
// XCD's L2 (tile t of every unit lands on the same XCD when the tile count is
// a multiple of 8); limb-major order re-read the whole batch's last limbs
// from HBM or the MALL once per limb.
template <int LOGN, int EC>
__global__ __launch_bounds__(256) void k_rs_cols(RsArgs a, const Tw *__restrict__ tw,
                                                 const LimbConst *__restrict__ lc) {
  constexpr uint32_t tiles = (1u << (LOGN - EC)) / 256;
  constexpr int LO = LOGN - EC;
  const uint32_t u = blockIdx.x / tiles;
  const uint32_t b = u / a.L, i = u % a.L;
  const uint32_t col = (blockIdx.x % tiles) * 256 + threadIdx.x;
  const ModQ m = lc[i].m;
  const RsLimb r = a.rs[i];
  uint64_t v[1 << EC];
  load_global<LOGN, EC, LO, EC, true>(v, a.tl + ((uint64_t)b << LOGN), col);
#pragma unroll
  for (int s = 0; s < (1 << EC); ++s) v[s] = rs_prologue(v[s], a.qL, a.h, r, m.q);
  fwd_round<LOGN, EC, LO, EC, 0>(v, LOGN, 0, col, tw + (size_t)i * 2 * (1u << LOGN), m);
  store_global<LOGN, EC, LO, EC, true>(v, a.out + (((uint64_t)b * a.L + i) << LOGN), col);
}

// Block pass (remaining stages) in place on out, then the epilogue.
template <int LOGN, int B, int E>
__global__ __launch_bounds__(1 << (B - E)) void k_rs_blocks(RsArgs a, const Tw *__restrict__ tw,
                                                             const LimbConst *__restrict__ lc) {
  __shared__ uint64_t lds[LdsSize<B>::value];
  constexpr uint32_t tiles = 1u << (LOGN - B);
  uint32_t b, i;
  rs_unit(blockIdx.x / tiles, a.batch, b, i);
  const uint32_t blockStart = (blockIdx.x % tiles) << B;
  const ModQ m = lc[i].m;
  const RsLimb r = a.rs[i];
  uint64_t *p = a.out + (((uint64_t)b * a.L + i) << LOGN) + blockStart;
  const uint32_t tid = threadIdx.x;
  using F = FwdFirst<B, E>;
  uint64_t v[1 << E];
  load_global<B, E, F::LO, F::R>(v, p, RoundMap<B, E, F::LO, F::R>::lane_part(tid));
  fwd_block_rounds<B, E, F::LO, F::R>(v, LOGN, lds, tid, blockStart, tw + (size_t)i * 2 * (1u << LOGN), m);
  reduce_fwd<E>(v, m, lc[i].mu, lc[i].k);
  uint64_t cv[1 << E];
  load_global_m0<B, E>(cv, a.c + (((uint64_t)b * (a.L + 1) + i) << LOGN) + blockStart, lds, tid);
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) v[s] = rs_epilogue(cv[s], v[s], r, m);
  store_global_m0<B, E>(v, p, lds, tid);
}

// Coefficient-domain rescale: element-wise, tiles of 2048 words.
__global__ __launch_bounds__(256) void k_rs_coeff(RsArgs a, const LimbConst *__restrict__ lc, uint32_t log_n,
                                                  uint32_t tiles) {
  uint32_t b, i;
  rs_unit(blockIdx.x / tiles, a.batch, b, i);
  const uint32_t n = 1u << log_n, base = (blockIdx.x % tiles) * 2048u;
  const ModQ m = lc[i].m;
  const RsLimb r = a.rs[i];
  const uint64_t *ci = a.c + (((uint64_t)b * (a.L + 1) + i) << log_n);
  const uint64_t *cl = a.c + (((uint64_t)b * (a.L + 1) + a.L) << log_n);
  uint64_t *o = a.out + (((uint64_t)b * a.L + i) << log_n);
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const uint32_t k = base + threadIdx.x + 256u * s;
    if (k < n) o[k] = rs_epilogue(ci[k], reduce_4q(rs_prologue(cl[k], a.qL, a.h, r, m.q), m), r, m);
  }
}

}  // namespace hentt
