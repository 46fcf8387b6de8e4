// Microbenchmarks behind the benchmark's roofline (built on its own into
// libhentt_mb.so; measurement code, not part of the library):
//   * HBM stream bandwidth: a copy (each byte read once, written once) and a
//     read-only sweep, 16-byte accesses, grid-stride;
//   * VALU issue rate of the 32-bit integer multiplies the modular
//     arithmetic is built from (v_mad_u64_u32, v_mul_hi_u32, v_mul_lo_u32),
//     of the other instructions its butterflies issue (the 64-bit add
//     v_lshl_add_u64, the 64-bit compare, the three-input add, register
//     moves), of a plain v_add_u32 for comparison, and of the library's own
//     lazy forward butterfly (multiplies, additions, compares and selects as
//     the kernels issue them).
// Every issue kernel keeps 8 independent dependency chains per lane and
// writes every chain's final value, so no operation can be removed or
// hoisted; the single-instruction kernels spell the instruction in inline
// assembly so that the compiler can neither combine nor reassociate it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modarith.hpp"

namespace hentt_mb {

typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

// Copy of n 16-byte vectors: each workgroup moves chunks of 4 x 256
// vectors (four independent loads in flight per lane), grid-stride over the
// chunks, a guarded tail.  NT: streaming (non-temporal) loads and stores.
template <bool NT>
__global__ __launch_bounds__(256) void mb_copy_k(const u64x2 *__restrict__ src, u64x2 *__restrict__ dst, uint64_t n) {
  const uint64_t chunks = n / 1024;
  for (uint64_t c = blockIdx.x; c < chunks; c += gridDim.x) {
    const uint64_t base = c * 1024 + threadIdx.x;
    u64x2 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = NT ? __builtin_nontemporal_load(src + base + 256 * k) : src[base + 256 * k];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (NT) __builtin_nontemporal_store(v[k], dst + base + 256 * k);
      else dst[base + 256 * k] = v[k];
    }
  }
  for (uint64_t i = chunks * 1024 + (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
    dst[i] = src[i];
}

__global__ __launch_bounds__(256) void mb_read_k(const u64x2 *__restrict__ src, uint64_t n, uint64_t *out) {
  uint64_t acc = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    const u64x2 v = __builtin_nontemporal_load(src + i);
    acc ^= v.x + v.y;
  }
  out[(uint64_t)blockIdx.x * 256 + threadIdx.x] = acc;
}

enum { MB_MAD64 = 0, MB_MULHI = 1, MB_MULLO = 2, MB_ADD = 3, MB_BFLY = 4, MB_ADD64 = 5, MB_CMP64 = 6, MB_ADD3 = 7,
       MB_MOV = 8 };

// The butterfly's constants arrive as kernel arguments, as the library's
// kernels load theirs from memory, so that the compiler cannot specialise
// the arithmetic to known values.
template <int KIND>
__global__ __launch_bounds__(256) void mb_issue_k(uint64_t *out, uint32_t iters, uint32_t a, uint64_t w, uint64_t ws,
                                                  hentt::ModQ m) {
  const uint64_t gid = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if constexpr (KIND == MB_BFLY) {
    const uint64_t q = m.q;
    uint64_t x[8], y[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      x[j] = (gid * 8 + j) % q;
      y[j] = (gid * 8 + j + 1) % q;
    }
#pragma unroll 2
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
      for (int j = 0; j < 8; ++j) hentt::ct_bfly(x[j], y[j], w, ws, m);
    }
    uint64_t r = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) r ^= x[j] + y[j];
    out[gid] = r;
  } else if constexpr (KIND == MB_MAD64) {
    uint64_t acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = gid * 8 + j;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = (uint64_t)(uint32_t)acc[j] * a + acc[j];   // v_mad_u64_u32
    }
    uint64_t r = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) r ^= acc[j];
    out[gid] = r;
  } else if constexpr (KIND == MB_ADD64 || KIND == MB_CMP64) {
    uint64_t z[8];
    const uint64_t a64 = ((uint64_t)a << 32) | (a ^ 0x5555u);
#pragma unroll
    for (int j = 0; j < 8; ++j) z[j] = gid * 8 + j;
    uint32_t hits = 0;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if constexpr (KIND == MB_ADD64) {
          asm volatile("v_lshl_add_u64 %0, %0, 0, %1" : "+v"(z[j]) : "v"(a64));
        } else {
          // the compare's result lands in VCC and is not read: the chain
          // is the compare itself, one per element and iteration
          asm volatile("v_cmp_lt_u64 vcc, %0, %1" ::"v"(z[j]), "v"(a64) : "vcc");
        }
      }
      hits += 1;
    }
    uint64_t r = hits;
#pragma unroll
    for (int j = 0; j < 8; ++j) r ^= z[j];
    out[gid] = r;
  } else {
    uint32_t x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = (uint32_t)(gid * 8 + j) | 1u;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if constexpr (KIND == MB_MULHI) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(x[j]) : "v"(a));
        else if constexpr (KIND == MB_MULLO) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x[j]) : "v"(a));
        else if constexpr (KIND == MB_ADD3) asm volatile("v_add3_u32 %0, %0, %1, %1" : "+v"(x[j]) : "v"(a));
        else if constexpr (KIND == MB_MOV) asm volatile("v_mov_b32 %0, %1" : "=v"(x[j]) : "v"(x[(j + 1) & 7]));
        else asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[j]) : "v"(a));
      }
    }
    uint64_t r = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) r ^= x[j];
    out[gid] = r;
  }
}

}  // namespace hentt_mb

using namespace hentt_mb;

extern "C" {

// Copies `bytes` (a multiple of 16) from src to dst on `stream`; streaming
// (non-temporal) accesses when nt.
int mb_copy(void *dst, const void *src, uint64_t bytes, uint32_t grid, int nt, void *stream) {
  if (!dst || !src || bytes % 16 || grid == 0) return -1;
  if (nt)
    hipLaunchKernelGGL(mb_copy_k<true>, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const u64x2 *)src,
                       (u64x2 *)dst, bytes / 16);
  else
    hipLaunchKernelGGL(mb_copy_k<false>, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const u64x2 *)src,
                       (u64x2 *)dst, bytes / 16);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// Reads `bytes` (a multiple of 16) of src; out receives grid * 256 words.
int mb_read(const void *src, uint64_t bytes, uint64_t *out, uint32_t grid, void *stream) {
  if (!out || !src || bytes % 16 || grid == 0) return -1;
  hipLaunchKernelGGL(mb_read_k, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const u64x2 *)src, bytes / 16, out);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// Issue-rate kernel `kind` (0 v_mad_u64_u32, 1 v_mul_hi_u32, 2 v_mul_lo_u32,
// 3 v_add_u32, 4 forward butterfly, 5 v_lshl_add_u64, 6 v_cmp_lt_u64,
// 7 v_add3_u32, 8 v_mov_b32): grid workgroups of 256 lanes, each lane
// running 8 chains of `iters` operations; out receives grid * 256 words.
// For kind 4, w, ws, q are a twiddle, its Shoup quotient and the modulus.
int mb_issue(int kind, uint64_t *out, uint32_t iters, uint32_t grid, uint32_t a, uint64_t w, uint64_t ws, uint64_t q,
             void *stream) {
  if (!out || grid == 0) return -1;
  hipStream_t st = (hipStream_t)stream;
  const hentt::ModQ m{q, 0 - q, 2 * q, 0 - 2 * q, 4 * q, 0 - 4 * q};
  switch (kind) {
    case MB_MAD64: hipLaunchKernelGGL(mb_issue_k<MB_MAD64>, dim3(grid), dim3(256), 0, st, out, iters, a, w, ws, m); break;
    case MB_MULHI: hipLaunchKernelGGL(mb_issue_k<MB_MULHI>, dim3(grid), dim3(256), 0, st, out, iters, a, w, ws, m); break;
    case MB_MULLO: hipLaunchKernelGGL(mb_issue_k<MB_MULLO>, dim3(grid), dim3(256), 0, st, out, iters, a, w, ws, m); break;
    case MB_ADD: hipLaunchKernelGGL(mb_issue_k<MB_ADD>, dim3(grid), dim3(256), 0, st, out, iters, a, w, ws, m); break;
    case MB_BFLY: hipLaunchKernelGGL(mb_issue_k<MB_BFLY>, dim3(grid), dim3(256), 0, st, out, iters, a, w, ws, m); break;
    case MB_ADD64: hipLaunchKernelGGL(mb_issue_k<MB_ADD64>, dim3(grid), dim3(256), 0, st, out, iters, a, w, ws, m); break;
    case MB_CMP64: hipLaunchKernelGGL(mb_issue_k<MB_CMP64>, dim3(grid), dim3(256), 0, st, out, iters, a, w, ws, m); break;
    case MB_ADD3: hipLaunchKernelGGL(mb_issue_k<MB_ADD3>, dim3(grid), dim3(256), 0, st, out, iters, a, w, ws, m); break;
    case MB_MOV: hipLaunchKernelGGL(mb_issue_k<MB_MOV>, dim3(grid), dim3(256), 0, st, out, iters, a, w, ws, m); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // extern "C"
