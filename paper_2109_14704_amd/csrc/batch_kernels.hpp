// Uneven batches in one persistent launch (the batch x RNS-limb parallelism of
// section III-B: every (polynomial, limb) of every job is an independent
// transform).  Workgroups of 256 lanes pull tiles from a queue (one atomic
// counter).  A transform of N = 2^12 is one tile; a larger transform is a
// pass-1 set of tiles and a pass-2 set: forward = column pass, then 2^12
// blocks; inverse = 2^12 blocks, then column pass.  Pass-2 tiles wait on a
// per-(polynomial, limb) counter of finished pass-1 tiles.  Tiles are handed
// out in dependency order (every pass-1 tile before any pass-2 tile), so a
// waiting tile only waits on tiles already held by running workgroups; the
// wait is also bounded (spin limit), after which the tile sets an error flag
// and is skipped, so every workgroup always exits.
#pragma once
#include "ntt_kernels.hpp"

namespace hentt {

struct BatchUnit {        // one (polynomial, limb) of a job
  uint64_t *data;         // N words, in place
  const Tw *tw;           // this limb's table for the launch direction
  const LimbConst *lc;    // this limb's constants
  uint32_t logn;          // 12 .. 17
  uint32_t pass1;         // pass-1 tiles of this unit (0: one whole-transform tile)
};
struct BatchTile {
  uint32_t unit;
  uint32_t kind_idx;      // kind << 16 | tile index; kind 0 whole, 1 pass 1, 2 pass 2
};
enum { BT_WHOLE = 0, BT_PASS1 = 1, BT_PASS2 = 2 };
enum { BATCH_B = 12, BATCH_E = 4, BATCH_LANES = 256 };

// Loads and stores here are ordinary (not streaming): pass 2 reads pass 1's
// results back from L2, and streaming even the first read or the last write
// of a word made the uneven workload 18% slower.

// Forward block pass (stages logn-12 .. logn-1) on the 2^12 words at p.
__device__ __forceinline__ void batch_fwd_block(uint64_t *p, uint32_t blockStart, uint32_t logn, const Tw *t,
                                                const LimbConst &c, uint64_t *lds, uint32_t tid) {
  using F = FwdFirst<BATCH_B, BATCH_E>;
  uint64_t v[1 << BATCH_E];
  load_global<BATCH_B, BATCH_E, F::LO, F::R>(v, p, RoundMap<BATCH_B, BATCH_E, F::LO, F::R>::lane_part(tid));
  fwd_block_rounds<BATCH_B, BATCH_E, F::LO, F::R>(v, logn, lds, tid, blockStart, t, c.m);
  reduce_fwd<BATCH_E>(v, c.m, c.mu, c.k);
  store_global_m0<BATCH_B, BATCH_E>(v, p, lds, tid);
}

// Inverse block pass (stages 0 .. 11); canonical when it is the whole transform.
__device__ __forceinline__ void batch_inv_block(uint64_t *p, uint32_t blockStart, uint32_t logn, const Tw *it,
                                                const LimbConst &c, uint64_t *lds, uint32_t tid) {
  using L = InvLast<BATCH_B, BATCH_E>;
  uint64_t v[1 << BATCH_E];
  load_global_m0_fresh<BATCH_B, BATCH_E>(v, p, lds, tid);  // the previous tile ended with a barrier
  inv_block_rounds<BATCH_B, BATCH_E, 0, BATCH_E>(v, logn, lds, tid, blockStart, it, c);
  if (logn == BATCH_B) reduce_inv<BATCH_E>(v, c.m);
  store_global<BATCH_B, BATCH_E, L::LO, L::R>(v, p, RoundMap<BATCH_B, BATCH_E, L::LO, L::R>::lane_part(tid));
}

// Column accesses whose per-element offset goes into the (wave-uniform, scalar)
// base address: every element shares the lane's one offset register instead
// of holding an address register of its own across the butterfly round.
// The base itself is made opaque first, so that the store side recomputes
// the element bases instead of keeping the load side's live in SGPRs.
template <int LOGN, int EC>
__device__ __forceinline__ const uint64_t *col_elem(const uint64_t *p, int s) {
  const uint64_t *e = p + ((uint64_t)s << (LOGN - EC));
  asm volatile("" : "+s"(e));
  return e;
}
__device__ __forceinline__ const uint64_t *opaque_s(const uint64_t *p) {
  asm volatile("" : "+s"(p));
  return p;
}

// Column pass of 2^EC stages (N = 2^(12+EC)) on a tile of 4096 coefficients:
// 256 lanes x CPL columns each (CPL = 16 / 2^EC, at least 1).
template <int EC, bool INV>
__device__ __forceinline__ void batch_cols(uint64_t *p, uint32_t tile, uint32_t tid, const Tw *t,
                                           const LimbConst &c) {
  constexpr int LOGN = BATCH_B + EC, LO = BATCH_B;
  constexpr uint32_t CPL = EC >= 4 ? 1u : (16u >> EC);
#pragma unroll
  for (uint32_t j = 0; j < CPL; ++j) {
    const uint32_t col = (tile * CPL + j) * BATCH_LANES + tid;
    uint64_t v[1 << EC];
    const uint64_t *pl = opaque_s(p);
#pragma unroll
    for (int s = 0; s < (1 << EC); ++s) v[s] = gload<false>(col_elem<LOGN, EC>(pl, s), col);
    if constexpr (!INV) {
      fwd_round<LOGN, EC, LO, EC, 0>(v, LOGN, 0, col, t, c.m);
    } else {
      inv_round<LOGN, EC, LO, EC>(v, LOGN, 0, col, t, c);
      reduce_inv<EC>(v, c.m);
    }
    const uint64_t *ps = opaque_s(p);
#pragma unroll
    for (int s = 0; s < (1 << EC); ++s) gstore<false>(const_cast<uint64_t *>(col_elem<LOGN, EC>(ps, s)), col, v[s]);
  }
}

template <bool INV>
__device__ __forceinline__ void batch_cols_any(uint32_t logn, uint64_t *p, uint32_t tile, uint32_t tid,
                                               const Tw *t, const LimbConst &c) {
  switch (logn) {
    case 13: batch_cols<1, INV>(p, tile, tid, t, c); break;
    case 14: batch_cols<2, INV>(p, tile, tid, t, c); break;
    case 15: batch_cols<3, INV>(p, tile, tid, t, c); break;
    case 16: batch_cols<4, INV>(p, tile, tid, t, c); break;
    default: batch_cols<5, INV>(p, tile, tid, t, c); break;
  }
}

// Column tiles per (polynomial, limb): 4096 coefficients each, 16 for N = 2^17.
__host__ __device__ inline uint32_t batch_col_tiles(uint32_t logn) { return logn >= 16 ? 16u : (1u << (logn - BATCH_B)); }

// One queue per XCD (the chip's 8 compute dies, each with its own L2).  A
// workgroup serves the queue of the XCD it runs on (hardware register
// XCC_ID), so both passes of a (polynomial, limb) run on one XCD: pass-2
// tiles read pass-1 results from that XCD's L2, which needs only completed
// stores on the writer side and an L1 invalidate on the reader side (no L2
// write-back).  ctl layout: [0, NQ) queue heads, [NQ] error flag,
// [NQ + 1, NQ + 1 + units) finished pass-1 tiles per unit.
enum { BATCH_NQ = 8 };

__device__ __forceinline__ uint32_t xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15u; }

// Invalidates this CU's vector L1 (the workgroup-scope invalidate of the
// CDNA3/4 memory model), so the loads that follow read pass-1 results from
// the XCD's L2.  An agent-scope acquire fence would also invalidate the L2's
// non-coherent lines; it is not needed (both passes of a unit run on one
// XCD) and it made pass-2 tiles about 1.6x slower.
__device__ __forceinline__ void invalidate_l1() { asm volatile("buffer_inv sc0" ::: "memory"); }

template <bool INV>
__global__ __launch_bounds__(BATCH_LANES, 4) void k_batch(const BatchUnit *__restrict__ units,
                                                       const BatchTile *__restrict__ tiles,
                                                       const uint32_t *__restrict__ qoff,
                                                       const uint32_t *__restrict__ qmap, uint32_t *ctl,
                                                       uint32_t spin_limit) {
  __shared__ __attribute__((aligned(16))) uint64_t lds[LdsSize<BATCH_B>::value];
  __shared__ uint32_t s_tile, s_ok;
  const uint32_t q = qmap[xcc_id()];
  if (q >= BATCH_NQ) return;  // an XCD the plan did not see: its queue is served elsewhere
  const uint32_t q0 = qoff[q], qn = qoff[q + 1] - q0;
  uint32_t *cnt = ctl + BATCH_NQ + 1;
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(&ctl[q], 1u);
    __syncthreads();
    const uint32_t ti = s_tile;
    // The lane index is re-read every tile (opaque to the optimiser), so the
    // per-lane addressing of every tile path is not hoisted out of this loop
    // and held live across all of them.
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    if (ti >= qn) return;                           // uniform: every workgroup leaves here
    const BatchTile tile = tiles[q0 + ti];
    const BatchUnit u = units[tile.unit];
    const uint32_t kind = tile.kind_idx >> 16, idx = tile.kind_idx & 0xffffu;
    const LimbConst c = ld_lc(u.lc);
    if (kind == BT_PASS2) {
      if (tid == 0) {
        uint32_t spins = 0, ok = 1;
        while (__hip_atomic_load(&cnt[tile.unit], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < u.pass1) {
          __builtin_amdgcn_s_sleep(2);
          if (++spins > spin_limit) {
            ok = 0;
            atomicOr(&ctl[BATCH_NQ], 1u);
            break;
          }
        }
        s_ok = ok;
      }
      __syncthreads();
      invalidate_l1();  // drop stale L1 lines before reading pass-1 results
      if (!s_ok) {
        __syncthreads();
        continue;
      }
    }
    if constexpr (!INV) {
      if (kind == BT_WHOLE) batch_fwd_block(u.data, 0, BATCH_B, u.tw, c, lds, tid);
      else if (kind == BT_PASS1) batch_cols_any<false>(u.logn, u.data, idx, tid, u.tw, c);
      else batch_fwd_block(u.data + ((uint64_t)idx << BATCH_B), idx << BATCH_B, u.logn, u.tw, c, lds, tid);
    } else {
      if (kind == BT_WHOLE) batch_inv_block(u.data, 0, BATCH_B, u.tw, c, lds, tid);
      else if (kind == BT_PASS1) batch_inv_block(u.data + ((uint64_t)idx << BATCH_B), idx << BATCH_B, u.logn, u.tw, c, lds, tid);
      else batch_cols_any<true>(u.logn, u.data, idx, tid, u.tw, c);
    }
    if (kind == BT_PASS1) {
      __builtin_amdgcn_s_waitcnt(0);  // this lane's stores have reached the XCD's L2
      __syncthreads();
      if (tid == 0) __hip_atomic_fetch_add(&cnt[tile.unit], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();  // LDS and s_tile are reused by the next tile
  }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, uint32_t n, uint32_t value) {
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = value;
}

// Records the XCC_ID of every workgroup (placement probe).
__global__ void k_xcc_probe(uint32_t *out) {
  if (threadIdx.x == 0) out[blockIdx.x] = xcc_id();
}

}  // namespace hentt
