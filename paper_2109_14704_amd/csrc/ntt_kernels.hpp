// Staged negacyclic NTT kernels for gfx950 (CDNA4), section III-B of the paper
// re-planned for a 64-wide wavefront, a 160 KB LDS and 512 VGPRs per lane.
//
// Data: x[poly][N] uint64, poly = batch * limbs + limb (limb fastest among
// polynomials, coefficient fastest overall).  Twiddles per limb: forward table
// psi^brv(k) and inverse table psi^-brv(k), k < N, each stored as (W, W')
// 16-byte pairs with W' = floor(W 2^64 / q) (the root powers and root power
// quotients of Algorithm 1).
//
// A transform is a sequence of "rounds".  A round applies R consecutive
// butterfly stages to groups of 2^R elements held in one lane's registers;
// the butterfly pairs of those stages differ in the index bits
// [LO, LO + R).  Rounds exchange data through LDS (inside a workgroup) or
// through HBM (between the column pass and the block pass of large N), as in
// the staged global -> local -> register design of section III-B, with the
// radix-2^R register blocking of its high-radix subsection.
#pragma once
#include <type_traits>

#include "modarith.hpp"

namespace hentt {

// LDS padding: one spare element after every 16, so that the lane-strided
// accesses of every round hit distinct banks.
__device__ __forceinline__ constexpr uint32_t lds_pad(uint32_t i) { return i + (i >> 4); }
template <int B> struct LdsSize { static constexpr int value = (1 << B) + (1 << B) / 16; };

// Which block index bits a lane owns in a round over bits [LO, LO+R) of a
// block of 2^B elements, with 2^E elements per lane (E >= R), 2^(B-E) lanes.
// Lane bits fill the lowest free positions (coalescing), the remaining
// E - R "group" bits the rest.
template <int B, int E, int LO, int R>
struct RoundMap {
  static_assert(E >= R && LO + R <= B && E <= B, "bad round");
  static constexpr int TB = B - E;
  static constexpr bool LANE_LOW = (TB <= LO);  // all lane bits below LO: twiddles uniform per block
  __device__ static __forceinline__ uint32_t lane_part(uint32_t tid) {
    if constexpr (LANE_LOW) return tid;
    else return (tid & ((1u << LO) - 1)) | ((tid >> LO) << (LO + R));
  }
  static constexpr uint32_t g_part(int g) {
    uint32_t r = 0;
    int bit = 0;
    if constexpr (LANE_LOW) {
      for (int pos = TB; pos < LO; ++pos, ++bit) if ((g >> bit) & 1) r |= 1u << pos;
      for (int pos = LO + R; pos < B; ++pos, ++bit) if ((g >> bit) & 1) r |= 1u << pos;
    } else {
      for (int pos = TB + R; pos < B; ++pos, ++bit) if ((g >> bit) & 1) r |= 1u << pos;
    }
    return r;
  }
  static constexpr uint32_t slot_part(int s) { return g_part(s >> R) | (uint32_t)((s & ((1 << R) - 1)) << LO); }
};

// Twiddle tables are never written while a kernel runs, so they are read
// through the constant address space: a wave-uniform index becomes a scalar
// load even when the table pointer was itself read from memory.
__device__ __forceinline__ Tw ld_tw(const Tw* t, uint32_t i) {
  const __attribute__((address_space(4))) uint64_t* p = (const __attribute__((address_space(4))) uint64_t*)(t + i);
  return Tw{p[0], p[1]};
}

// Limb constants through the constant address space as well: with a
// wave-uniform pointer (also one read from memory) they become scalar loads
// into SGPRs instead of 24 VGPRs of per-lane copies.
__device__ __forceinline__ LimbConst ld_lc(const LimbConst *p) {
  const __attribute__((address_space(4))) uint64_t *w = (const __attribute__((address_space(4))) uint64_t *)p;
  LimbConst c;
  c.m = ModQ{w[0], w[1], w[2], w[3], w[4], w[5]};
  c.ninv = w[6];
  c.ninv_s = w[7];
  c.ninvw = w[8];
  c.ninvw_s = w[9];
  c.mu = w[10];
  c.k = (uint32_t)w[11];
  c.pad = 0;
  return c;
}

// ---------------------------------------------------------------- rounds --
// Forward stages with global index s = LOGN - LO - R + u, u < R.  Stage s
// pairs j with j + N/2^(s+1) and uses psi_rev[2^s + (j >> (LOGN - s))].
// P0 >= 0: the library's butterfly (ct_bfly16, values below 16q), P0 being
// the parity of the round's first stage within its pass (a stage corrects X
// when its index within the pass is even).  P0 < 0: the classic butterfly
// (every stage corrects, values below 8q), for the reference designs.
template <int B, int E, int LO, int R, int P0 = -1>
__device__ __forceinline__ void fwd_round(uint64_t (&x)[1 << E], uint32_t logn, uint32_t blockStart,
                                          uint32_t lanePart, const Tw* __restrict__ tw, const ModQ &m) {
  using M = RoundMap<B, E, LO, R>;
#pragma unroll
  for (int g = 0; g < (1 << (E - R)); ++g) {
    const uint32_t J0 = M::LANE_LOW ? (blockStart | M::g_part(g)) : (blockStart | lanePart | M::g_part(g));
#pragma unroll
    for (int u = 0; u < R; ++u) {
      // stage s = logn - LO - R + u: 2^s = 2^(logn - B) * 2^(B - LO - R + u)
      const uint32_t base = ((1u << (logn - B)) << (B - LO - R + u)) + (J0 >> (LO + R - u));
      const int h = 1 << (R - 1 - u);
#pragma unroll
      for (int k = 0; k < (1 << R); ++k) {
        if (k & h) continue;
        const Tw w = ld_tw(tw, base + (k >> (R - u)));
        if constexpr (P0 < 0) ct_bfly(x[(g << R) + k], x[(g << R) + k + h], w.w, w.ws, m);
        else if (((P0 + u) & 1) == 0) ct_bfly16<true>(x[(g << R) + k], x[(g << R) + k + h], w.w, w.ws, m);
        else ct_bfly16<false>(x[(g << R) + k], x[(g << R) + k + h], w.w, w.ws, m);
      }
    }
  }
}

// Inverse stages v = LO + u.  Stage v pairs j with j + 2^v and uses
// psi_rev^-1[N/2^(v+1) + (j >> (v+1))].  The last stage (v = LOGN-1) also
// multiplies both outputs by N^-1.
template <int B, int E, int LO, int R>
__device__ __forceinline__ void inv_round(uint64_t (&x)[1 << E], uint32_t logn, uint32_t blockStart,
                                          uint32_t lanePart, const Tw* __restrict__ itw, const LimbConst& c) {
  using M = RoundMap<B, E, LO, R>;
#pragma unroll
  for (int g = 0; g < (1 << (E - R)); ++g) {
    const uint32_t J0 = M::LANE_LOW ? (blockStart | M::g_part(g)) : (blockStart | lanePart | M::g_part(g));
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int v = LO + u;
      const int d = 1 << u;
      // only the block's top stage can be the transform's last one
      if (LO + u == B - 1 && (uint32_t)v == logn - 1) {
        // last stage: one group, twiddle psi^-brv(1) folded with N^-1
#pragma unroll
        for (int k = 0; k < (1 << R); ++k) {
          if (k & d) continue;
          uint64_t& X = x[(g << R) + k];
          uint64_t& Y = x[(g << R) + k + d];
          const uint64_t s = X + Y, df = (X + c.m.q4) - Y;
          X = shoup(c.ninv, c.ninv_s, s, c.m.nq);
          Y = shoup(c.ninvw, c.ninvw_s, df, c.m.nq);
        }
      } else {
        const uint32_t base = ((1u << logn) >> (v + 1)) + (J0 >> (v + 1));
#pragma unroll
        for (int k = 0; k < (1 << R); ++k) {
          if (k & d) continue;
          const Tw w = ld_tw(itw, base + (k >> (u + 1)));
          gs_bfly(x[(g << R) + k], x[(g << R) + k + d], w.w, w.ws, c.m);
        }
      }
    }
  }
}

// ------------------------------------------------------------ data moves --
// Polynomial words are addressed as a base pointer plus a 32-bit byte offset
// (every index below lies inside one polynomial or block, < 2^17 words), in
// the global address space.  The compiler then issues global loads with one
// base for the wave and one 32-bit offset per lane, instead of a flat load
// with a 64-bit address per element, which matters where the base pointer
// was itself read from memory (the persistent batch kernel).
//
// NT: non-temporal (streaming) accesses, chosen per kernel by measurement:
// the column passes stream both ways (each word is read and written once, and
// the next pass over it comes after the whole batch has gone through the
// caches: 10-18% faster), the fused product kernels stream their loads (2-4%
// faster).  The block and whole-transform kernels, and the persistent batch
// kernel (which reads pass-1 results back from L2), were slower with
// streaming accesses (the forward block pass at N = 2^15 took twice as long)
// and use ordinary ones.
#define HENTT_GLOBAL __attribute__((address_space(1)))
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
template <bool NT> __device__ __forceinline__ uint64_t gload(const uint64_t* base, uint32_t i) {
  const HENTT_GLOBAL uint64_t* p = (const HENTT_GLOBAL uint64_t*)((const HENTT_GLOBAL char*)base + (i << 3));
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT> __device__ __forceinline__ void gstore(uint64_t* base, uint32_t i, uint64_t v) {
  HENTT_GLOBAL uint64_t* p = (HENTT_GLOBAL uint64_t*)((HENTT_GLOBAL char*)base + (i << 3));
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

template <int B, int E, int LO, int R, bool NT = false>
__device__ __forceinline__ void load_global(uint64_t (&x)[1 << E], const uint64_t* __restrict__ src, uint32_t lp) {
  using M = RoundMap<B, E, LO, R>;
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) x[s] = gload<NT>(src, lp + M::slot_part(s));
}
template <int B, int E, int LO, int R, bool NT = false>
__device__ __forceinline__ void store_global(const uint64_t (&x)[1 << E], uint64_t* __restrict__ dst, uint32_t lp) {
  using M = RoundMap<B, E, LO, R>;
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) gstore<NT>(dst, lp + M::slot_part(s), x[s]);
}
template <int B, int E, int LO, int R>
__device__ __forceinline__ void load_lds(uint64_t (&x)[1 << E], const uint64_t* lds, uint32_t lp) {
  using M = RoundMap<B, E, LO, R>;
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) x[s] = lds[lds_pad(lp + M::slot_part(s))];
}
template <int B, int E, int LO, int R>
__device__ __forceinline__ void store_lds(const uint64_t (&x)[1 << E], uint64_t* lds, uint32_t lp) {
  using M = RoundMap<B, E, LO, R>;
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) lds[lds_pad(lp + M::slot_part(s))] = x[s];
}

// Global stores and loads of the (0, E) map, in which every lane holds 2^E
// consecutive words, routed through LDS: the global side uses the map whose
// lanes own the lowest block bits, so that each memory instruction covers
// consecutive words across the lanes instead of one word every 2^E.  Both
// begin with a barrier (the workgroup's earlier LDS reads are done); the load
// also ends with one, so that the caller may write LDS next.
#ifndef HENTT_TS
#define HENTT_TS 1
#endif
#ifndef HENTT_TL
#define HENTT_TL 1
#endif
template <int B, int E, bool NT = false>
__device__ __forceinline__ void store_global_m0(uint64_t (&x)[1 << E], uint64_t* __restrict__ dst, uint64_t* lds,
                                                uint32_t tid) {
#if HENTT_TS
  using MT = RoundMap<B, E, B - E, E>;
  __syncthreads();
  store_lds<B, E, 0, E>(x, lds, RoundMap<B, E, 0, E>::lane_part(tid));
  __syncthreads();
  load_lds<B, E, B - E, E>(x, lds, MT::lane_part(tid));
  store_global<B, E, B - E, E, NT>(x, dst, MT::lane_part(tid));
#else
  store_global<B, E, 0, E, NT>(x, dst, RoundMap<B, E, 0, E>::lane_part(tid));
#endif
}
template <int B, int E, bool NT = false>
__device__ __forceinline__ void load_global_m0(uint64_t (&x)[1 << E], const uint64_t* __restrict__ src, uint64_t* lds,
                                               uint32_t tid) {
#if HENTT_TL
  using MT = RoundMap<B, E, B - E, E>;
  load_global<B, E, B - E, E, NT>(x, src, MT::lane_part(tid));
  __syncthreads();
  store_lds<B, E, B - E, E>(x, lds, MT::lane_part(tid));
  __syncthreads();
  load_lds<B, E, 0, E>(x, lds, RoundMap<B, E, 0, E>::lane_part(tid));
  __syncthreads();
#else
  load_global<B, E, 0, E, NT>(x, src, RoundMap<B, E, 0, E>::lane_part(tid));
#endif
}

// The same load for a workgroup whose LDS holds nothing yet (the first
// access of a kernel or of a persistent tile): direct global-to-LDS loads
// (global_load_lds_dwordx4), which move each lane's 16 bytes into the wave's
// 1 KB LDS window without passing through registers, then one 16-byte LDS
// read per word pair.  One instruction fills a contiguous window, so the LDS
// layout is set by which global pair each lane fetches: pair P = 8t + k of
// the block sits at LDS pair 8t + (k ^ (t mod 8)) (the map is its own
// inverse), which puts the eight pairs one 8-lane group reads in eight
// different 16-byte bank groups.  Ends with a barrier, like load_global_m0.
#ifndef HENTT_DMA_LOAD
#define HENTT_DMA_LOAD 1
#endif
__device__ __forceinline__ uint32_t dma_swz(uint32_t pair) { return pair ^ ((pair >> 3) & 7u); }
template <int B, int E>
__device__ __forceinline__ void load_global_m0_fresh(uint64_t (&x)[1 << E], const uint64_t* __restrict__ src,
                                                     uint64_t* lds, uint32_t tid) {
  constexpr uint32_t LANES = 1u << (B - E);
  if constexpr (HENTT_DMA_LOAD && LANES % 64 == 0 && E >= 1) {
    constexpr uint32_t WAVE_WORDS = 64u << E;   // the words one wave moves
    const uint32_t wave = tid >> 6, lane = tid & 63;
    typedef __attribute__((address_space(3))) void lds_void;
#pragma unroll
    for (uint32_t i = 0; i < WAVE_WORDS / 128; ++i) {
      const uint32_t win = wave * WAVE_WORDS + 128 * i;   // first word of this instruction's window
      const uint32_t pair = win / 2 + lane;                  // LDS pair this lane fills
      __builtin_amdgcn_global_load_lds(src + 2 * dma_swz(pair), (lds_void*)(lds + win), 16, 0, 0);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < (1u << (E - 1)); ++j) {
      const u64x2 w = *(const u64x2*)(lds + 2 * dma_swz((tid << (E - 1)) + j));
      x[2 * j] = w.x;
      x[2 * j + 1] = w.y;
    }
    __syncthreads();
  } else {
    load_global_m0<B, E>(x, src, lds, tid);
  }
}

// Canonical reductions of forward outputs ([0, 16q)) and inverse outputs
// ([0, 4q)).  Forward: moduli above 2^33 (bit length k >= 34; mu is the
// limb's Barrett constant) take the quotient estimate and one conditional
// subtraction, smaller ones the chain of four conditional subtractions (k
// is uniform per workgroup, so the branch is a scalar one).
template <int E>
__device__ __forceinline__ void reduce_fwd(uint64_t (&x)[1 << E], const ModQ &m, uint64_t mu, uint32_t k) {
  if (k >= 34) {
    const uint32_t c = est_c(mu, k), sh = k - 33;
#pragma unroll
    for (int s = 0; s < (1 << E); ++s) x[s] = csubn(reduce_est(x[s], m.nq, c, sh), m.nq);
  } else {
#pragma unroll
    for (int s = 0; s < (1 << E); ++s) x[s] = reduce_16q(x[s], m);
  }
}
template <int E> __device__ __forceinline__ void reduce_inv(uint64_t (&x)[1 << E], const ModQ &m) {
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) x[s] = reduce_4q(x[s], m);
}

// --------------------------------------------------- block transforms ----
// Forward rounds over the block bits [0, LO+R) (the first round covers
// [LO, LO+R)), starting from registers already loaded with the first round's
// map.  Ends with the lane holding the last round (LO = 0) map in registers,
// i.e. 2^E consecutive elements, values in [0, 16q).  P: parity of the
// round's first stage within the block pass.
template <int B, int E, int LO, int R, int P = 0>
__device__ __forceinline__ void fwd_block_rounds(uint64_t (&x)[1 << E], uint32_t logn, uint64_t* lds, uint32_t tid,
                                                 uint32_t blockStart, const Tw* __restrict__ tw, const ModQ &m) {
  using M = RoundMap<B, E, LO, R>;
  const uint32_t lp = M::lane_part(tid);
  fwd_round<B, E, LO, R, P>(x, logn, blockStart, lp, tw, m);
  if constexpr (LO > 0) {
    constexpr int R2 = E;
    constexpr int LO2 = LO - R2;
    static_assert(LO2 >= 0, "rounds must tile the block");
    store_lds<B, E, LO, R>(x, lds, lp);
    __syncthreads();
    using M2 = RoundMap<B, E, LO2, R2>;
    load_lds<B, E, LO2, R2>(x, lds, M2::lane_part(tid));
    fwd_block_rounds<B, E, LO2, R2, (P + R) & 1>(x, logn, lds, tid, blockStart, tw, m);
  }
}

// Inverse rounds over block bits [LO, B), starting from registers loaded with
// the (LO, R) map.  Ends with the lane holding the last round's map
// (covering [B - Rlast, B)); values in [0, 2q).
template <int B, int E, int LO, int R>
__device__ __forceinline__ void inv_block_rounds(uint64_t (&x)[1 << E], uint32_t logn, uint64_t* lds, uint32_t tid,
                                                 uint32_t blockStart, const Tw* __restrict__ itw,
                                                 const LimbConst& c) {
  using M = RoundMap<B, E, LO, R>;
  const uint32_t lp = M::lane_part(tid);
  inv_round<B, E, LO, R>(x, logn, blockStart, lp, itw, c);
  if constexpr (LO + R < B) {
    constexpr int LO2 = LO + R;
    constexpr int R2 = (B - LO2) < E ? (B - LO2) : E;
    store_lds<B, E, LO, R>(x, lds, lp);
    __syncthreads();
    using M2 = RoundMap<B, E, LO2, R2>;
    load_lds<B, E, LO2, R2>(x, lds, M2::lane_part(tid));
    inv_block_rounds<B, E, LO2, R2>(x, logn, lds, tid, blockStart, itw, c);
  }
}

// Round geometry helpers.
template <int B, int E> struct FwdFirst {   // forward: first round is the short one
  static constexpr int R = (B % E) ? (B % E) : E;
  static constexpr int LO = B - R;
};
template <int B, int E> struct InvLast {    // inverse: last round is the short one
  static constexpr int R = (B % E) ? (B % E) : E;
  static constexpr int LO = B - R;
};

// Map blockIdx -> (polynomial, tile): limb-major, batch next, tile fastest, so
// that concurrently running workgroups share one limb's twiddle table in L2.
struct Unit {
  uint32_t poly, limb, tile;
};
__device__ __forceinline__ Unit unit_of(uint32_t bid, uint32_t tiles, uint32_t batch, uint32_t limbs) {
  Unit u;
  u.tile = bid % tiles;
  uint32_t r = bid / tiles;
  u.limb = r / batch;
  uint32_t b = r % batch;
  u.poly = b * limbs + u.limb;
  return u;
}

// ------------------------------------------------------------- kernels ----
// Whole transform of one polynomial per workgroup (N = 2^LOGN fits in LDS).
template <int LOGN, int E>
__global__ __launch_bounds__(1 << (LOGN - E)) void k_fwd_whole(uint64_t* __restrict__ x, const Tw* __restrict__ tw,
                                                                const LimbConst* __restrict__ lc, uint32_t batch,
                                                                uint32_t limbs) {
  __shared__ __attribute__((aligned(16))) uint64_t lds[LdsSize<LOGN>::value];
  const Unit un = unit_of(blockIdx.x, 1, batch, limbs);
  const ModQ m = lc[un.limb].m;
  const Tw* t = tw + (size_t)un.limb * 2 * (1u << LOGN);
  uint64_t* p = x + (size_t)un.poly * (1u << LOGN);
  const uint32_t tid = threadIdx.x;
  using F = FwdFirst<LOGN, E>;
  uint64_t v[1 << E];
  load_global<LOGN, E, F::LO, F::R>(v, p, RoundMap<LOGN, E, F::LO, F::R>::lane_part(tid));
  fwd_block_rounds<LOGN, E, F::LO, F::R>(v, LOGN, lds, tid, 0, t, m);
  reduce_fwd<E>(v, m, lc[un.limb].mu, lc[un.limb].k);
  store_global_m0<LOGN, E>(v, p, lds, tid);
}

template <int LOGN, int E>
__global__ __launch_bounds__(1 << (LOGN - E)) void k_inv_whole(uint64_t* __restrict__ x, const Tw* __restrict__ tw,
                                                                const LimbConst* __restrict__ lc, uint32_t batch,
                                                                uint32_t limbs) {
  __shared__ __attribute__((aligned(16))) uint64_t lds[LdsSize<LOGN>::value];
  const Unit un = unit_of(blockIdx.x, 1, batch, limbs);
  const LimbConst c = lc[un.limb];
  const Tw* it = tw + ((size_t)un.limb * 2 + 1) * (1u << LOGN);
  uint64_t* p = x + (size_t)un.poly * (1u << LOGN);
  const uint32_t tid = threadIdx.x;
  using L = InvLast<LOGN, E>;
  uint64_t v[1 << E];
  load_global_m0_fresh<LOGN, E>(v, p, lds, tid);
  inv_block_rounds<LOGN, E, 0, (LOGN < E ? LOGN : E)>(v, LOGN, lds, tid, 0, it, c);
  reduce_inv<E>(v, c.m);
  store_global<LOGN, E, L::LO, L::R>(v, p, RoundMap<LOGN, E, L::LO, L::R>::lane_part(tid));
}

// Column pass: the first E forward stages (or the last E inverse stages) on
// 2^E elements at stride N / 2^E; workgroup of 256 lanes = 256 columns.
// Twiddles are the same for every lane (scalar loads).  Up to four
// polynomial sets ("components") per launch, each read from src[c] and
// written to dst[c] (equal for in place).
struct ColArgs {
  const uint64_t *src[4];
  uint64_t *dst[4];
  uint64_t src_sb, dst_sb;  // words between consecutive batch entries
};

// One column of the column pass: 2^E elements at stride N / 2^E starting at
// word `col`, read from src and written to dst (equal for in place).  `t` is
// the limb's forward table, or its inverse table when INV.
template <int LOGN, int E, bool INV>
__device__ __forceinline__ void col_pass(const uint64_t *src, uint64_t *dst, uint32_t col, const Tw *t,
                                         const LimbConst &c) {
  constexpr int LO = LOGN - E;
  uint64_t v[1 << E];
  load_global<LOGN, E, LO, E, true>(v, src, col);
  if constexpr (!INV) {
    fwd_round<LOGN, E, LO, E, 0>(v, LOGN, 0, col, t, c.m);
  } else {
    inv_round<LOGN, E, LO, E>(v, LOGN, 0, col, t, c);
    reduce_inv<E>(v, c.m);
  }
  store_global<LOGN, E, LO, E, true>(v, dst, col);
}

// Columns per lane: two neighbouring columns (16-byte accesses) for passes of
// up to 16 words per lane; at 32 words per lane the doubled registers cost
// more than the wider accesses gain (measured: column passes of 2^17
// transforms 12% faster, of the 2^15 and 2^16 products 6-10% slower).
template <int E> struct ColCpl { static constexpr int value = E <= 4 ? 2 : 1; };
// Two neighbouring columns per lane: 16-byte accesses.
template <int LOGN, int E, bool INV>
__device__ __forceinline__ void col_pass2(const uint64_t *src, uint64_t *dst, uint32_t col, const Tw *t,
                                          const LimbConst &c) {
  constexpr int LO = LOGN - E;
  uint64_t v0[1 << E], v1[1 << E];
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) {
    const HENTT_GLOBAL u64x2 *p = (const HENTT_GLOBAL u64x2 *)((const HENTT_GLOBAL char *)src + ((col + (s << LO)) << 3));
    const u64x2 w = __builtin_nontemporal_load(p);
    v0[s] = w.x;
    v1[s] = w.y;
  }
  if constexpr (!INV) {
    fwd_round<LOGN, E, LO, E, 0>(v0, LOGN, 0, col, t, c.m);
    fwd_round<LOGN, E, LO, E, 0>(v1, LOGN, 0, col, t, c.m);
  } else {
    inv_round<LOGN, E, LO, E>(v0, LOGN, 0, col, t, c);
    inv_round<LOGN, E, LO, E>(v1, LOGN, 0, col, t, c);
    reduce_inv<E>(v0, c.m);
    reduce_inv<E>(v1, c.m);
  }
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) {
    HENTT_GLOBAL u64x2 *p = (HENTT_GLOBAL u64x2 *)((HENTT_GLOBAL char *)dst + ((col + (s << LO)) << 3));
    u64x2 w;
    w.x = v0[s];
    w.y = v1[s];
    __builtin_nontemporal_store(w, p);
  }
}

// Workgroup `blk` of a column pass over batch x limbs units of every
// component of `a` (the body of k_cols and of its grouped form).
template <int LOGN, int E, bool INV>
__device__ __forceinline__ void cols_block(const ColArgs &a, const Tw *__restrict__ tw,
                                           const LimbConst *__restrict__ lc, uint32_t batch, uint32_t limbs,
                                           uint32_t blk) {
  constexpr uint32_t CPL = ColCpl<E>::value;
  constexpr uint32_t tiles = (1u << (LOGN - E)) / (256 * CPL);
  const uint32_t units = batch * limbs;
  const uint32_t tile = blk % tiles;
  const uint32_t r = blk / tiles;
  const uint32_t comp = r / units, u = r % units;
  const uint32_t limb = u / batch, b = u % batch;
  const LimbConst c = lc[limb];
  const uint64_t off = (uint64_t)limb << LOGN;
  const uint64_t *src = a.src[comp] + (uint64_t)b * a.src_sb + off;
  uint64_t *dst = a.dst[comp] + (uint64_t)b * a.dst_sb + off;
  const Tw *t = tw + ((size_t)limb * 2 + (INV ? 1 : 0)) * (1u << LOGN);
  if constexpr (CPL == 2) col_pass2<LOGN, E, INV>(src, dst, tile * 512 + 2 * threadIdx.x, t, c);
  else col_pass<LOGN, E, INV>(src, dst, tile * 256 + threadIdx.x, t, c);
}

// Workgroups per component of a column pass over `units` (batch x limbs) units.
template <int LOGN, int E> constexpr uint32_t cols_blocks_per_unit() {
  return (1u << (LOGN - E)) / (256 * ColCpl<E>::value);
}

template <int LOGN, int E, bool INV>
__global__ __launch_bounds__(256) void k_cols(ColArgs a, const Tw *__restrict__ tw, const LimbConst *__restrict__ lc,
                                              uint32_t batch, uint32_t limbs) {
  cols_block<LOGN, E, INV>(a, tw, lc, batch, limbs, blockIdx.x);
}

// Block pass of the forward transform: stages LOGN-B .. LOGN-1 on contiguous
// blocks of 2^B elements; canonical output.
template <int LOGN, int B, int E>
__global__ __launch_bounds__(1 << (B - E)) void k_fwd_blocks(uint64_t *__restrict__ x, const Tw *__restrict__ tw,
                                                              const LimbConst *__restrict__ lc, uint32_t batch,
                                                              uint32_t limbs) {
  __shared__ __attribute__((aligned(16))) uint64_t lds[LdsSize<B>::value];
  constexpr uint32_t tiles = 1u << (LOGN - B);
  const Unit un = unit_of(blockIdx.x, tiles, batch, limbs);
  const ModQ m = lc[un.limb].m;
  const Tw *t = tw + (size_t)un.limb * 2 * (1u << LOGN);
  const uint32_t blockStart = un.tile << B;
  uint64_t *p = x + (size_t)un.poly * (1u << LOGN) + blockStart;
  const uint32_t tid = threadIdx.x;
  using F = FwdFirst<B, E>;
  uint64_t v[1 << E];
  load_global<B, E, F::LO, F::R>(v, p, RoundMap<B, E, F::LO, F::R>::lane_part(tid));
  fwd_block_rounds<B, E, F::LO, F::R>(v, LOGN, lds, tid, blockStart, t, m);
  reduce_fwd<E>(v, m, lc[un.limb].mu, lc[un.limb].k);
  store_global_m0<B, E>(v, p, lds, tid);
}

// Block pass of the inverse transform: stages 0 .. B-1; lazy [0, 2q) output.
template <int LOGN, int B, int E>
__global__ __launch_bounds__(1 << (B - E)) void k_inv_blocks(uint64_t *__restrict__ x, const Tw *__restrict__ tw,
                                                              const LimbConst *__restrict__ lc, uint32_t batch,
                                                              uint32_t limbs) {
  __shared__ __attribute__((aligned(16))) uint64_t lds[LdsSize<B>::value];
  constexpr uint32_t tiles = 1u << (LOGN - B);
  const Unit un = unit_of(blockIdx.x, tiles, batch, limbs);
  const LimbConst c = lc[un.limb];
  const Tw *it = tw + ((size_t)un.limb * 2 + 1) * (1u << LOGN);
  const uint32_t blockStart = un.tile << B;
  uint64_t *p = x + (size_t)un.poly * (1u << LOGN) + blockStart;
  const uint32_t tid = threadIdx.x;
  using L = InvLast<B, E>;
  uint64_t v[1 << E];
  load_global_m0_fresh<B, E>(v, p, lds, tid);
  inv_block_rounds<B, E, 0, E>(v, LOGN, lds, tid, blockStart, it, c);
  store_global<B, E, L::LO, L::R>(v, p, RoundMap<B, E, L::LO, L::R>::lane_part(tid));
}

// ------------------------------------------------------ fused products ----
// Compile-time loop: f(std::integral_constant<int, I>) for I in [I0, I1), so
// that array indices stay constants (no stack arrays) even for loop bodies too
// large for the unroller.
template <int I0, int I1, typename F> __device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I0 < I1) {
    f(std::integral_constant<int, I0>{});
    static_for<I0 + 1, I1>(f);
  }
}

// Returns p unchanged but hides that from the optimiser (adds an opaque,
// wave-uniform zero), so loads through it are not merged with earlier ones.
template <typename T> __device__ __forceinline__ const T *opaque(const T *p) {
  uint32_t z = 0;
  asm volatile("" : "+s"(z));
  return p + z;
}

// Products of section II: PROD_MUL is the dyadic product of two polynomials
// (a (.) b); PROD_TENSOR the ciphertext Mul tensor (c0 d0, c0 d1 + c1 d0,
// c1 d1) with the middle term reduced once (mad_mod, section III-A-1).
enum { PROD_MUL = 0, PROD_TENSOR = 1 };
template <int MODE> struct ProdShape {
  static constexpr int NIN = MODE == PROD_MUL ? 2 : 4;
  static constexpr int NOUT = MODE == PROD_MUL ? 1 : 3;
};
struct ProdArgs {
  const uint64_t *in[4];
  uint64_t *out[3];
  uint64_t in_sb, out_sb;  // words between consecutive batch entries
};

// arr[i] for a wave-uniform i < N, as a chain of selects: indexing the
// kernel-argument array with a loop counter directly made the compiler copy
// it to scratch and load the pointer from there into VGPRs.
// Each element passes through an (empty) scalar-register asm first, so the
// select chain is not folded back into an indexed load.
template <typename T, int N> __device__ __forceinline__ T pick_ptr(T const (&arr)[N], int i) {
  T r = arr[0];
  asm volatile("" : "+s"(r));
#pragma unroll
  for (int k = 1; k < N; ++k) {
    T c = arr[k];
    asm volatile("" : "+s"(c));
    r = (i == k) ? c : r;
  }
  return r;
}

template <int MODE, int E>
__device__ __forceinline__ void products(uint64_t (&X)[ProdShape<MODE>::NIN][1 << E],
                                         uint64_t (&Y)[ProdShape<MODE>::NOUT][1 << E], const LimbConst &c) {
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) {
    if constexpr (MODE == PROD_MUL) {
      Y[0][s] = mulmod(X[0][s], X[1][s], c.m.q, c.mu, c.k);
    } else {
      Y[0][s] = mulmod(X[0][s], X[2][s], c.m.q, c.mu, c.k);
      Y[1][s] = madmod(X[0][s], X[3][s], X[1][s], X[2][s], c.m.q, c.mu, c.k);
      Y[2][s] = mulmod(X[1][s], X[3][s], c.m.q, c.mu, c.k);
    }
  }
}

// The products ahead of an inverse transform, in Montgomery form: every
// output is off by R^-1 (R = 2^64), a constant factor the inverse transform
// removes with its N^-1 scaling, taken from the folded constants N^-1 R.
// Inputs: MUL factors below 4q (a b < 16 q^2 < q R as q < 2^60); TENSOR
// factors below 2q (c0 d1 + c1 d0 < 8 q^2 < q R).  Outputs in [0, 2q), a valid
// inverse-transform input.
template <int MODE, int E>
__device__ __forceinline__ void products_mont(uint64_t (&X)[ProdShape<MODE>::NIN][1 << E],
                                              uint64_t (&Y)[ProdShape<MODE>::NOUT][1 << E], uint64_t q,
                                              uint64_t qinv) {
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) {
    if constexpr (MODE == PROD_MUL) {
      Y[0][s] = mont_mul(X[0][s], X[1][s], q, qinv);
    } else {
      Y[0][s] = mont_mul(X[0][s], X[2][s], q, qinv);
      Y[1][s] = mont_mad(X[0][s], X[3][s], X[1][s], X[2][s], q, qinv);
      Y[2][s] = mont_mul(X[1][s], X[3][s], q, qinv);
    }
  }
}

// Forward outputs ([0, 16q)) brought to the factor range of products_mont.
// Factors below 16q already keep a product below q R for q < 2^56
// (256 q^2 < q 2^64), and the tensor's sum of two products for q < 2^55:
// such limbs skip the reduction (k, the bit length, is uniform per
// workgroup, so the test is a scalar branch).
template <int MODE, int E>
__device__ __forceinline__ void reduce_for_mont(uint64_t (&x)[1 << E], const ModQ &m, uint64_t mu, uint32_t k) {
  if (k <= (MODE == PROD_TENSOR ? 55u : 56u)) return;
  if (k >= 34) {  // quotient estimate: [0, 2q) for either product
    const uint32_t c = est_c(mu, k), sh = k - 33;
#pragma unroll
    for (int s = 0; s < (1 << E); ++s) x[s] = reduce_est(x[s], m.nq, c, sh);
    return;
  }
#pragma unroll
  for (int s = 0; s < (1 << E); ++s) {
    x[s] = csubn(csubn(x[s], m.nq4 + m.nq4), m.nq4);
    if constexpr (MODE == PROD_TENSOR) x[s] = csubn(x[s], m.nq2);
  }
}

// One workgroup per block of 2^B coefficients of one (batch entry, limb):
// forward block rounds of every input (DO_FWD; otherwise the inputs are
// already NTT-domain values), the products in registers, then the inverse
// block rounds of every output (DO_INV).  The forward transform ends and the
// inverse transform begins with each lane holding 2^E consecutive NTT-domain
// values, so the product needs no data exchange and the NTT-domain values
// never leave the chip.  With B == LOGN the whole product is one kernel;
// with B < LOGN the forward column pass runs before it and the inverse
// column pass after it.  With DO_INV the products are Montgomery products
// and lc must hold the folded constants (N^-1 R in place of N^-1), also for
// the inverse column pass that completes the transform.  Without DO_INV the
// products are exact (Barrett) and lc the plain constants.
// Workgroup `blk` of the fused product over batch x limbs units (the body of
// k_prod and of its grouped form).
template <int LOGN, int B, int E, int MODE, bool DO_FWD, bool DO_INV>
__device__ __forceinline__ void prod_block(const ProdArgs &a, const Tw *__restrict__ tw,
                                           const LimbConst *__restrict__ lc, const MontLimb *__restrict__ mont,
                                           uint32_t batch, uint32_t limbs, uint32_t blk) {
  constexpr int NIN = ProdShape<MODE>::NIN, NOUT = ProdShape<MODE>::NOUT;
  __shared__ __attribute__((aligned(16))) uint64_t lds[(DO_FWD || DO_INV) ? LdsSize<B>::value : 2];
  constexpr uint32_t tiles = 1u << (LOGN - B);
  const uint32_t tile = blk % tiles;
  const uint32_t r = blk / tiles;
  const uint32_t limb = r / batch, b = r % batch;
  const LimbConst c = lc[limb];
  const Tw *t = tw + (size_t)limb * 2 * (1u << LOGN);
  const Tw *it = t + (1u << LOGN);
  const uint32_t blockStart = tile << B;
  const uint64_t in_off = (uint64_t)b * a.in_sb + ((uint64_t)limb << LOGN) + blockStart;
  const uint64_t out_off = (uint64_t)b * a.out_sb + ((uint64_t)limb << LOGN) + blockStart;
  const uint32_t tid = threadIdx.x;
  using F = FwdFirst<B, E>;
  using L = InvLast<B, E>;
  // The transform code appears once for all inputs and once for all outputs
  // (rolled loops): unrolled per polynomial it would outgrow the instruction
  // cache.  Results move between the loop's working registers and the
  // per-polynomial arrays through compile-time-indexed copies.
  uint64_t X[NIN][1 << E];
#pragma unroll 1
  for (int p = 0; p < NIN; ++p) {
    uint64_t v[1 << E];
    if constexpr (DO_FWD) {
      if (p > 0) __syncthreads();  // the previous input's last LDS reads are done
      // an opaque copy of the table pointer per input: the twiddles are re-read
      // from cache instead of being hoisted out of the loop into VGPRs
      const Tw *tp = opaque(t);
      load_global<B, E, F::LO, F::R, true>(v, pick_ptr(a.in, p) + in_off, RoundMap<B, E, F::LO, F::R>::lane_part(tid));
      fwd_block_rounds<B, E, F::LO, F::R>(v, LOGN, lds, tid, blockStart, tp, c.m);
      if constexpr (DO_INV) reduce_for_mont<MODE, E>(v, c.m, c.mu, c.k);
      else reduce_fwd<E>(v, c.m, c.mu, c.k);
    } else {
      load_global_m0<B, E, true>(v, pick_ptr(a.in, p) + in_off, lds, tid);
    }
    static_for<0, NIN>([&](auto P) {
      if (p == decltype(P)::value) {
        // distinct marker per branch: keeps the branches from being merged
        // into one dynamically indexed (stack) store
        if constexpr (MODE == PROD_TENSOR) asm volatile("; sel %0" ::"n"(decltype(P)::value));
#pragma unroll
        for (int s2 = 0; s2 < (1 << E); ++s2) X[decltype(P)::value][s2] = v[s2];
      }
    });
  }
  uint64_t Y[NOUT][1 << E];
  if constexpr (DO_INV) products_mont<MODE, E>(X, Y, c.m.q, mont[limb].qinv);
  else products<MODE, E>(X, Y, c);
#pragma unroll 1
  for (int o = 0; o < NOUT; ++o) {
    uint64_t v[1 << E];
    static_for<0, NOUT>([&](auto O) {
      if (o == decltype(O)::value) {
        if constexpr (MODE == PROD_TENSOR) asm volatile("; sel %0" ::"n"(decltype(O)::value));
#pragma unroll
        for (int s2 = 0; s2 < (1 << E); ++s2) v[s2] = Y[decltype(O)::value][s2];
      }
    });
    if constexpr (DO_INV) {
      __syncthreads();  // earlier LDS reads of this workgroup are done
      inv_block_rounds<B, E, 0, E>(v, LOGN, lds, tid, blockStart, opaque(it), c);
      if constexpr (B == LOGN) reduce_inv<E>(v, c.m);
      store_global<B, E, L::LO, L::R>(v, pick_ptr(a.out, o) + out_off, RoundMap<B, E, L::LO, L::R>::lane_part(tid));
    } else {
      store_global_m0<B, E>(v, pick_ptr(a.out, o) + out_off, lds, tid);
    }
  }
}

template <int LOGN, int B, int E, int MODE, bool DO_FWD, bool DO_INV>
__global__ __launch_bounds__(1 << (B - E)) void k_prod(ProdArgs a, const Tw *__restrict__ tw,
                                                        const LimbConst *__restrict__ lc,
                                                        const MontLimb *__restrict__ mont, uint32_t batch,
                                                        uint32_t limbs) {
  prod_block<LOGN, B, E, MODE, DO_FWD, DO_INV>(a, tw, lc, mont, batch, limbs, blockIdx.x);
}

// Encrypted element-wise polynomial matrix product (section IV-E), NTT
// domain: C (m x n) += A (m x k) * B (k x n) with ciphertext elements, every
// element product the Mul tensor with one reduction per output (the middle
// term's two products summed first, mad_mod).  For k >= 3 the reductions are
// Montgomery's (R = 2^64): the accumulators start from C R^-1 (a Montgomery
// reduction of C itself, taken in the first step after the loads of A and B
// are issued, so that all three overlap), take the products' sums lazily
// below 2q over k, and one Shoup product by R mod q per word removes the
// common R^-1.  That conversion costs about as much as two and a half
// multiply-adds save, so smaller k accumulate with Barrett (mac1mod,
// mac2mod) directly on C (the host picks the instance; FULL when N >= 2048).
// One workgroup per (limb, i, j, tile of 2048 coefficients), j and
// the tile fastest so that consecutive workgroups share A's tiles in L2; 8
// coefficients per lane, the three accumulators in registers over k.
// One tile of k_ct_matmul.  FULL: every word of the tile lies below N (all
// tiles when N >= 2048), so the loads carry no per-word guard and are issued
// together; otherwise words at or beyond N are skipped.  MONT: Montgomery
// accumulation, else Barrett.
template <bool FULL, bool MONT>
__device__ __forceinline__ void ct_matmul_tile(const uint64_t *A, const uint64_t *B, uint64_t *c,
                                               const LimbConst &lc, const MontLimb &mc, uint64_t P, uint64_t off,
                                               uint32_t ia, uint32_t jb, uint32_t n, uint32_t k, uint32_t valid) {
  const ModQ &mq = lc.m;
  const uint64_t q = mq.q, qinv = mc.qinv;
  uint64_t c0[8], c1[8], c2[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const uint32_t e = threadIdx.x + 256u * s;
    const bool in = FULL || e < valid;
    c0[s] = in ? c[e] : 0;
    c1[s] = in ? c[P + e] : 0;
    c2[s] = in ? c[2 * P + e] : 0;
  }
  for (uint32_t l = 0; l < k; ++l) {
    const uint64_t *a = A + ((uint64_t)ia * k + l) * 2 * P + off;
    const uint64_t *b = B + ((uint64_t)l * n + jb) * 2 * P + off;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const uint32_t e = threadIdx.x + 256u * s;
      if (FULL || e < valid) {
        const uint64_t a0 = a[e], a1 = a[P + e], b0 = b[e], b1 = b[P + e];
        if constexpr (MONT) {
          if (l == 0) {
            c0[s] = redc(0, c0[s], q, qinv);
            c1[s] = redc(0, c1[s], q, qinv);
            c2[s] = redc(0, c2[s], q, qinv);
          }
          c0[s] = csubn(c0[s] + mont_mul(a0, b0, q, qinv), mq.nq2);
          c1[s] = csubn(c1[s] + mont_mad(a0, b1, a1, b0, q, qinv), mq.nq2);
          c2[s] = csubn(c2[s] + mont_mul(a1, b1, q, qinv), mq.nq2);
        } else {
          c0[s] = mac1mod(a0, b0, c0[s], q, lc.mu, lc.k);
          c1[s] = mac2mod(a0, b1, a1, b0, c1[s], q, lc.mu, lc.k);
          c2[s] = mac1mod(a1, b1, c2[s], q, lc.mu, lc.k);
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const uint32_t e = threadIdx.x + 256u * s;
    if (FULL || e < valid) {
      if constexpr (MONT) {
        c0[s] = reduce_4q(shoup(mc.r, mc.rs, c0[s], mq.nq), mq);
        c1[s] = reduce_4q(shoup(mc.r, mc.rs, c1[s], mq.nq), mq);
        c2[s] = reduce_4q(shoup(mc.r, mc.rs, c2[s], mq.nq), mq);
      }
      c[e] = c0[s];
      c[P + e] = c1[s];
      c[2 * P + e] = c2[s];
    }
  }
}

template <bool FULL, bool MONT>
__global__ __launch_bounds__(256) void k_ct_matmul(const uint64_t *__restrict__ A, const uint64_t *__restrict__ B,
                                                   uint64_t *__restrict__ C, const LimbConst *__restrict__ lc,
                                                   const MontLimb *__restrict__ mont, uint32_t m, uint32_t n,
                                                   uint32_t k, uint32_t limbs, uint32_t log_n, uint32_t tiles) {
  uint32_t r = blockIdx.x;
  const uint32_t tile = r % tiles;
  r /= tiles;
  const uint32_t j = r % n;
  r /= n;
  const uint32_t i = r % m, limb = r / m;
  const LimbConst cst = lc[limb];
  const MontLimb mc = mont[limb];
  const uint64_t P = (uint64_t)limbs << log_n;
  const uint64_t off = ((uint64_t)limb << log_n) + tile * 2048u;
  uint64_t *c = C + ((uint64_t)i * n + j) * 3 * P + off;
  ct_matmul_tile<FULL, MONT>(A, B, c, cst, mc, P, off, i, j, n, k, FULL ? 2048u : (1u << log_n));
}

// Element-wise products of NTT-domain inputs (no transform): tiles of 2048
// words of one (batch entry, limb), coalesced, limb constants uniform per
// workgroup.
template <int MODE>
__device__ __forceinline__ void elem_block(const ProdArgs &a, const LimbConst *__restrict__ lc, uint32_t batch,
                                           uint32_t limbs, uint32_t log_n, uint32_t tiles, uint32_t blk) {
  constexpr int NIN = ProdShape<MODE>::NIN, NOUT = ProdShape<MODE>::NOUT;
  const uint32_t tile = blk % tiles;
  const uint32_t r = blk / tiles;
  const uint32_t limb = r / batch, b = r % batch;
  const LimbConst c = lc[limb];
  const uint32_t n = 1u << log_n;
  const uint64_t in_off = (uint64_t)b * a.in_sb + ((uint64_t)limb << log_n) + tile * 2048u;
  const uint64_t out_off = (uint64_t)b * a.out_sb + ((uint64_t)limb << log_n) + tile * 2048u;
  uint64_t X[NIN][8], Y[NOUT][8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const uint32_t i = threadIdx.x + 256u * s;
#pragma unroll
    for (int p = 0; p < NIN; ++p) X[p][s] = (tile * 2048u + i < n) ? a.in[p][in_off + i] : 0;
  }
  products<MODE, 3>(X, Y, c);
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const uint32_t i = threadIdx.x + 256u * s;
    if (tile * 2048u + i < n) {
#pragma unroll
      for (int o = 0; o < NOUT; ++o) a.out[o][out_off + i] = Y[o][s];
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_elem(ProdArgs a, const LimbConst *__restrict__ lc, uint32_t batch,
                                              uint32_t limbs, uint32_t log_n, uint32_t tiles) {
  elem_block<MODE>(a, lc, batch, limbs, log_n, tiles, blockIdx.x);
}

}  // namespace hentt
