// Grouped ciphertext tensor products (section II-A, Mul; the batching of
// section III-B across jobs of different sizes): one launch per kernel of the
// product runs every job of one ring dimension N -- each job with its own
// operands, limb count (level) and tables -- so that many small products
// (a serving step of single-ciphertext requests at mixed levels) fill the GPU
// with three launches instead of three per job.
//
// The job table travels in the kernel's argument segment.  Job j owns the
// workgroups [ustart_j, ustart_j + units_j) x (workgroups per unit) of a
// launch, units_j = batch_j x limbs_j; a workgroup finds its job with a
// binary search over the (uniform) unit starts and runs the same body as
// the single-job kernel.
#pragma once
#include "ntt_kernels.hpp"

namespace hentt {

// One job of a grouped launch.  `a` holds the kernel's own argument form:
// ColArgs for a column pass (the components' source and destination bases),
// ProdArgs for the fused block kernel and the element-wise product.
struct GroupJob {
  union {
    ColArgs ca;
    ProdArgs pa;
  };
  const Tw *tw;           // [limbs][2][N]
  const LimbConst *lc;    // [limbs] plain or folded constants (host's choice)
  const MontLimb *mont;   // [limbs]
  uint32_t batch, limbs;
  uint32_t ustart;        // sum of batch x limbs over the earlier jobs of the launch
  uint32_t pad_;
};

constexpr int kGroupJobs = 24;  // jobs per launch: the table stays below 3 KB of kernel arguments

struct GroupTable {
  uint32_t n;  // jobs in use
  uint32_t pad_[3];
  GroupJob j[kGroupJobs];
};

// Index of the job owning global unit u: the last j with ustart_j <= u.
__device__ __forceinline__ uint32_t group_job(const GroupTable &g, uint32_t u) {
  uint32_t lo = 0, hi = g.n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (g.j[mid].ustart <= u) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Column pass over `COMPS` components of every job (forward into the
// workspace, or the inverse in place on the outputs).
template <int LOGN, int E, bool INV, int COMPS>
__global__ __launch_bounds__(256) void k_cols_g(GroupTable g) {
  constexpr uint32_t per = COMPS * cols_blocks_per_unit<LOGN, E>();
  const GroupJob &J = g.j[group_job(g, blockIdx.x / per)];
  cols_block<LOGN, E, INV>(J.ca, J.tw, J.lc, J.batch, J.limbs, blockIdx.x - J.ustart * per);
}

template <int LOGN, int B, int E, int MODE, bool DO_FWD, bool DO_INV>
__global__ __launch_bounds__(1 << (B - E)) void k_prod_g(GroupTable g) {
  constexpr uint32_t per = 1u << (LOGN - B);
  const GroupJob &J = g.j[group_job(g, blockIdx.x / per)];
  prod_block<LOGN, B, E, MODE, DO_FWD, DO_INV>(J.pa, J.tw, J.lc, J.mont, J.batch, J.limbs,
                                              blockIdx.x - J.ustart * per);
}

template <int MODE>
__global__ __launch_bounds__(256) void k_elem_g(GroupTable g, uint32_t log_n, uint32_t tiles) {
  const GroupJob &J = g.j[group_job(g, blockIdx.x / tiles)];
  elem_block<MODE>(J.pa, J.lc, J.batch, J.limbs, log_n, tiles, blockIdx.x - J.ustart * tiles);
}

}  // namespace hentt
