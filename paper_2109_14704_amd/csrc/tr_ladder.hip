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


// ----------------------------------------------------- wave-shuffle stages --
// The staged radix-2 transform with the smallest gaps exchanged between the
// lanes of a wavefront instead of through LDS (the SIMD shuffling of section
// III-B).  A lane holds S pairs ("register slots"): a wave holds a chunk of
// 2^C = 128 S consecutive words, and the stages with gaps 2^(C-1) .. 1 run in
// the wave; the larger gaps of a 2048-word block go through LDS, one radix-2
// stage per exchange.  The paper's SIMD(TER_SIMD_GAP_SZ, SIMD_WIDTH) variants
// map to SIMD(64 S, 64) here: SIMD(64,64), SIMD(128,64), SIMD(256,64) for
// S = 1, 2, 4, the 64-wide analogues of its SIMD(8,8), SIMD(16,8), SIMD(32,8).
//
// Wave layout: register index k (RB = log2(2S) bits), lane l (6 bits).  On
// entry register bit rb holds chunk bit 6 + rb and lane bit j chunk bit j.
// The first RB stages (pair bits C-1 .. 6) pair registers of one lane.  Each
// of the remaining six (pair bit j = 5 .. 0) first swaps lane bit j with
// register bit 0 between partner lanes l and l ^ 2^j: the lane whose bit j is
// 0 sends its registers with bit 0 set and receives the partner's registers
// with bit 0 clear into them, and the other way round (one 64-bit word per
// register pair crosses lanes).  After that swap register bit 0 holds chunk
// bit j, lane bit j holds chunk bit j + 1, and lane bits above j (swapped
// earlier) hold chunk bits one higher.
template <int S> struct SimdPlan {
  static constexpr int RB = S == 1 ? 1 : S == 2 ? 2 : 3;  // register bits: 2S words per lane
  static constexpr int C = 6 + RB;                         // chunk bits
  static constexpr int B = 11;                             // block of 2048 words
  static constexpr int LANES = (1 << B) >> RB;
};

// Lane exchange of a 32-bit value with the lane l ^ 2^J: DPP for J = 0, 1
// (quad permutations) and J = 3 (row rotation by 8), ds_swizzle for J = 2, 4
// (xor masks within 32 lanes), ds_bpermute across the two halves (J = 5).
template <int J> __device__ __forceinline__ uint32_t lane_xor32(uint32_t v, uint32_t lane) {
  if constexpr (J == 0) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);
  else if constexpr (J == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);
  else if constexpr (J == 2) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x101F);
  else if constexpr (J == 3) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, true);
  else if constexpr (J == 4) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);
  else return (uint32_t)__builtin_amdgcn_ds_bpermute((int)((lane ^ 32u) << 2), (int)v);
}
template <int J> __device__ __forceinline__ uint64_t lane_xor64(uint64_t v, uint32_t lane) {
  return ((uint64_t)lane_xor32<J>(hi32(v), lane) << 32) | lane_xor32<J>(lo32(v), lane);
}

// Radix-2 LDS rounds over block bits LO, LO-1, .., STOP (one stage each);
// the last round's words end in LDS (stored and past a barrier).
template <int B, int E, int LO, int STOP>
__device__ __forceinline__ void lds_r2_rounds(uint64_t (&x)[1 << E], uint32_t logn, uint64_t *lds, uint32_t tid,
                                              uint32_t blockStart, const Tw *__restrict__ tw, const ModQ &m) {
  using M = RoundMap<B, E, LO, 1>;
  const uint32_t lp = M::lane_part(tid);
  fwd_round<B, E, LO, 1>(x, logn, blockStart, lp, tw, m);
  if constexpr (LO == B - 1) __syncthreads();  // (the first round's words came from HBM)
  store_lds<B, E, LO, 1>(x, lds, lp);
  __syncthreads();
  if constexpr (LO > STOP) {
    load_lds<B, E, LO - 1, 1>(x, lds, RoundMap<B, E, LO - 1, 1>::lane_part(tid));
    __syncthreads();
    lds_r2_rounds<B, E, LO - 1, STOP>(x, logn, lds, tid, blockStart, tw, m);
  }
}

// Wave stage I (0-based) of the chunk: pair bit P = C - 1 - I.
template <int S, int I>
__device__ __forceinline__ void simd_stage(uint64_t (&v)[2 * S], uint32_t lane, uint32_t chunkStart, uint32_t logn,
                                           const Tw *__restrict__ tw, const ModQ &m) {
  using SP = SimdPlan<S>;
  constexpr int P = SP::C - 1 - I;
  constexpr bool IN_REG = I < SP::RB;
  constexpr int RBIT = IN_REG ? (SP::RB - 1 - I) : 0;  // register bit of the pair
  if constexpr (!IN_REG) {
    const bool hi = (lane >> P) & 1u;
#pragma unroll
    for (int k = 0; k < 2 * S; k += 2) {
      const uint64_t recv = lane_xor64<P>(hi ? v[k] : v[k + 1], lane);
      if (hi) v[k] = recv;
      else v[k + 1] = recv;
    }
  }
  // chunk index of the lower word of each pair, lane part
  const uint32_t lpart = IN_REG ? lane : ((lane & ((1u << P) - 1)) | ((lane >> P) << (P + 1)));
  const uint32_t base = 1u << (logn - 1 - P);
#pragma unroll
  for (int k = 0; k < 2 * S; ++k) {
    if (k & (1 << RBIT)) continue;
    const uint32_t rpart = IN_REG ? ((uint32_t)k << 6) : ((uint32_t)(k >> 1) << 7);
    const uint32_t g = chunkStart + lpart + rpart;
    const Tw w = ld_tw(tw, base + (g >> (P + 1)));
    ct_bfly(v[k], v[k | (1 << RBIT)], w.w, w.ws, m);
  }
  if constexpr (I + 1 < SP::C) simd_stage<S, I + 1>(v, lane, chunkStart, logn, tw, m);
}

// Forward stages LOGN-11 .. LOGN-1 on 2048-word blocks: LDS radix-2 rounds
// for the gaps of 1024 down to 2^C, the wave stages for the rest, the
// reduction to [0, q), and a coalesced store through LDS.
template <int LOGN, int S>
__global__ __launch_bounds__(SimdPlan<S>::LANES) void k_fwd_simd(uint64_t *__restrict__ x, const Tw *__restrict__ tw,
                                                                 const LimbConst *__restrict__ lc, uint32_t batch,
                                                                 uint32_t limbs) {
  using SP = SimdPlan<S>;
  constexpr int B = SP::B, E = SP::RB, C = SP::C;
  __shared__ uint64_t lds[LdsSize<B>::value];
  constexpr uint32_t tiles = 1u << (LOGN - B);
  const Unit un = unit_of(blockIdx.x, tiles, batch, limbs);
  const ModQ m = lc[un.limb].m;
  const Tw *t = tw + (size_t)un.limb * 2 * (1u << LOGN);
  const uint32_t blockStart = un.tile << B;
  uint64_t *p = x + (size_t)un.poly * (1u << LOGN) + blockStart;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  uint64_t v[2 * S];
  load_global<B, E, B - 1, 1>(v, p, RoundMap<B, E, B - 1, 1>::lane_part(tid));
  lds_r2_rounds<B, E, B - 1, C>(v, LOGN, lds, tid, blockStart, t, m);
  const uint32_t chunk = wave << C;
#pragma unroll
  for (int k = 0; k < 2 * S; ++k) v[k] = lds[lds_pad(chunk + (lane | ((uint32_t)k << 6)))];
  simd_stage<S, 0>(v, lane, blockStart + chunk, LOGN, t, m);
  // final layout: register bit 0 = chunk bit 0, lane bits = chunk bits 1..6,
  // register bits >= 1 = chunk bits 7..
  __syncthreads();  // every wave has read its chunk from LDS
#pragma unroll
  for (int k = 0; k < 2 * S; ++k)
    lds[lds_pad(chunk + ((uint32_t)(k & 1) | (lane << 1) | ((uint32_t)(k >> 1) << 7)))] = reduce_8q(v[k], m);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 2 * S; ++k) {
    const uint32_t i = tid + (uint32_t)k * SP::LANES;
    p[i] = lds[lds_pad(i)];
  }
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

template <int S> void launch_simd15(const hentt_tables *t, uint64_t *x, uint64_t units, uint32_t batch,
                                   hipStream_t st) {
  launch_naive_stages(t, x, units, 0, 4, st);
  LaunchTimer lt_(S == 1 ? "k_fwd_simd1" : S == 2 ? "k_fwd_simd2" : "k_fwd_simd4", 15, st);
  hipLaunchKernelGGL((k_fwd_simd<15, S>), dim3((uint32_t)(units << 4)), dim3(SimdPlan<S>::LANES), 0, st, x,
                     t->s->d_tw, t->s->d_lc, batch, t->limbs);
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
    case HENTT_VARIANT_SIMD1:
    case HENTT_VARIANT_SIMD2:
    case HENTT_VARIANT_SIMD4:
      if (ln != 15 || ((units << 14) + 255) / 256 > 0x7fffffffu) return HENTT_EINVAL;
      if (variant == HENTT_VARIANT_SIMD1) launch_simd15<1>(t, x, units, batch, st);
      else if (variant == HENTT_VARIANT_SIMD2) launch_simd15<2>(t, x, units, batch, st);
      else launch_simd15<4>(t, x, units, batch, st);
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
