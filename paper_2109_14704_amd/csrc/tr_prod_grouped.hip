// hentt_ct_tensor_grouped: many ciphertext tensor products (section II-A,
// Mul) of different levels and ring dimensions in a few launches.  Jobs are
// taken per ring dimension N, largest first, in chunks of up to kGroupJobs;
// each chunk is the product's launch sequence (forward column pass, fused
// block kernel, inverse column pass) with every kernel covering all jobs of
// the chunk.  The stage split is the one of the single-job product's default
// instance at that N (tuned choices are not consulted).
#include <algorithm>
#include <vector>

#include "grouped_kernels.hpp"
#include "runtime.hpp"

namespace hentt_rt {
namespace {

// Column stages and log2 words per lane of the grouped product at N = 2^log_n
// (the single-job tensor's default instance; 0 column stages = one kernel per
// block of N).
constexpr int grouped_pec(int log_n) { return log_n >= 14 ? (log_n == 14 ? 3 : 5) : log_n == 13 ? 1 : 0; }
constexpr int grouped_pe(int log_n) { return log_n == 15 ? 2 : 3; }

struct HostJob {
  const uint64_t *c, *d;
  uint64_t *out;
  const hentt_tables *t;
  uint32_t batch;
};

// Workspace words of one job: its four inputs after the forward column pass.
uint64_t ws_words(const HostJob &h) { return 4ull * h.batch * ((uint64_t)h.t->limbs << h.t->s->log_n); }

// One launch sequence over jobs[0, n), n <= kGroupJobs, all at N = 2^LOGN.
// ws: workspace of sum(ws_words) words when the forward column pass runs.
template <int LOGN>
int launch_group(const HostJob *jobs, uint32_t n, bool in_coeff, bool out_coeff, uint64_t *ws, hipStream_t st) {
  constexpr int PEC = grouped_pec(LOGN), PE = grouped_pe(LOGN);
  constexpr int B = PEC ? LOGN - PEC : LOGN;
  GroupTable g{};
  g.n = n;
  uint64_t units = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const Storage *s = jobs[i].t->s;
    GroupJob &J = g.j[i];
    J.tw = s->d_tw;
    // outputs going back to the coefficient domain take Montgomery products
    J.lc = out_coeff ? s->d_lcm : s->d_lc;
    J.mont = s->d_mont;
    J.batch = jobs[i].batch;
    J.limbs = jobs[i].t->limbs;
    J.ustart = (uint32_t)units;
    units += (uint64_t)J.batch * J.limbs;
  }
  // units < 2^24 per chunk and at most 64 workgroups per unit in any kernel
  // here: every grid stays below 2^30
  const uint32_t u = (uint32_t)units;
  auto nl = [&](uint32_t i) { return (uint64_t)g.j[i].limbs << LOGN; };

  if (!in_coeff && !out_coeff) {
    const uint32_t tiles = LOGN > 11 ? (1u << (LOGN - 11)) : 1u;
    for (uint32_t i = 0; i < n; ++i) {
      ProdArgs &a = g.j[i].pa;
      a = ProdArgs{};
      a.in[0] = jobs[i].c;
      a.in[1] = jobs[i].c + nl(i);
      a.in[2] = jobs[i].d;
      a.in[3] = jobs[i].d + nl(i);
      for (int o = 0; o < 3; ++o) a.out[o] = jobs[i].out + o * nl(i);
      a.in_sb = 2 * nl(i);
      a.out_sb = 3 * nl(i);
    }
    LaunchTimer lt_("k_elem_tensor_g", LOGN, st);
    hipLaunchKernelGGL((k_elem_g<PROD_TENSOR>), dim3(u * tiles), dim3(256), 0, st, g, (uint32_t)LOGN, tiles);
    return HENTT_OK;
  }
  const bool fwd_cols = PEC > 0 && in_coeff;
  if constexpr (PEC > 0) {
    if (fwd_cols) {
      uint64_t off = 0;
      for (uint32_t i = 0; i < n; ++i) {
        ColArgs &a = g.j[i].ca;
        a = ColArgs{};
        a.src[0] = jobs[i].c;
        a.src[1] = jobs[i].c + nl(i);
        a.src[2] = jobs[i].d;
        a.src[3] = jobs[i].d + nl(i);
        for (int p = 0; p < 4; ++p) a.dst[p] = ws + off + p * jobs[i].batch * nl(i);
        a.src_sb = 2 * nl(i);
        a.dst_sb = nl(i);
        off += 4 * jobs[i].batch * nl(i);
      }
      LaunchTimer lt_("k_cols_fwd_g", LOGN, st);
      hipLaunchKernelGGL((k_cols_g<LOGN, PEC, false, 4>), dim3(4 * u * cols_blocks_per_unit<LOGN, PEC>()), dim3(256),
                         0, st, g);
    }
  }
  {
    uint64_t off = 0;
    for (uint32_t i = 0; i < n; ++i) {
      ProdArgs &a = g.j[i].pa;
      a = ProdArgs{};
      if (fwd_cols) {
        for (int p = 0; p < 4; ++p) a.in[p] = ws + off + p * jobs[i].batch * nl(i);
        a.in_sb = nl(i);
        off += 4 * jobs[i].batch * nl(i);
      } else {
        a.in[0] = jobs[i].c;
        a.in[1] = jobs[i].c + nl(i);
        a.in[2] = jobs[i].d;
        a.in[3] = jobs[i].d + nl(i);
        a.in_sb = 2 * nl(i);
      }
      for (int o = 0; o < 3; ++o) a.out[o] = jobs[i].out + o * nl(i);
      a.out_sb = 3 * nl(i);
    }
    const dim3 grid(u << (LOGN - B)), blk(1 << (B - PE));
    LaunchTimer lt_("k_prod_tensor_g", LOGN, st);
    if (in_coeff && out_coeff)
      hipLaunchKernelGGL((k_prod_g<LOGN, B, PE, PROD_TENSOR, true, true>), grid, blk, 0, st, g);
    else if (in_coeff)
      hipLaunchKernelGGL((k_prod_g<LOGN, B, PE, PROD_TENSOR, true, false>), grid, blk, 0, st, g);
    else
      hipLaunchKernelGGL((k_prod_g<LOGN, B, PE, PROD_TENSOR, false, true>), grid, blk, 0, st, g);
  }
  if constexpr (PEC > 0) {
    if (out_coeff) {
      for (uint32_t i = 0; i < n; ++i) {
        ColArgs &a = g.j[i].ca;
        a = ColArgs{};
        for (int o = 0; o < 3; ++o) a.src[o] = a.dst[o] = jobs[i].out + o * nl(i);
        a.src_sb = a.dst_sb = 3 * nl(i);
      }
      LaunchTimer lt_("k_cols_inv_g", LOGN, st);
      hipLaunchKernelGGL((k_cols_g<LOGN, PEC, true, 3>), dim3(3 * u * cols_blocks_per_unit<LOGN, PEC>()), dim3(256),
                         0, st, g);
    }
  }
  return HENTT_OK;
}

typedef int (*GroupFn)(const HostJob *, uint32_t, bool, bool, uint64_t *, hipStream_t);
#define HENTT_GROUP_FN(n) launch_group<n>,
const GroupFn k_group_fn[] = {HENTT_SIZES(HENTT_GROUP_FN)};
#undef HENTT_GROUP_FN

struct Span {
  uintptr_t a, b;
};
Span span_of(const void *p, uint64_t words) { return Span{(uintptr_t)p, (uintptr_t)p + (uintptr_t)(words * 8)}; }

// HENTT_OK if no output range overlaps another output or any input range.
int check_overlaps(const std::vector<HostJob> &jobs) {
  std::vector<Span> outs;
  outs.reserve(jobs.size());
  for (const HostJob &h : jobs) outs.push_back(span_of(h.out, 3 * h.batch * ((uint64_t)h.t->limbs << h.t->s->log_n)));
  std::sort(outs.begin(), outs.end(), [](const Span &x, const Span &y) { return x.a < y.a; });
  for (size_t i = 1; i < outs.size(); ++i)
    if (outs[i].a < outs[i - 1].b) return HENTT_EINVAL;
  // disjoint and sorted by start, the outputs are sorted by end too
  auto hits = [&](Span x) {
    auto it = std::upper_bound(outs.begin(), outs.end(), x.a, [](uintptr_t v, const Span &y) { return v < y.b; });
    return it != outs.end() && it->a < x.b;
  };
  for (const HostJob &h : jobs) {
    const uint64_t words = 2 * h.batch * ((uint64_t)h.t->limbs << h.t->s->log_n);
    if (hits(span_of(h.c, words)) || hits(span_of(h.d, words))) return HENTT_EINVAL;
  }
  return HENTT_OK;
}

}  // namespace
}  // namespace hentt_rt

using namespace hentt_rt;

extern "C" int hentt_ct_tensor_grouped(const hentt_ct_job *jobs, uint32_t njobs, uint32_t flags, void *stream) {
  ApiRange range_("hentt_ct_tensor_grouped");
  if (njobs == 0) return HENTT_OK;
  if (!jobs || (flags & ~3u)) return HENTT_EINVAL;
  std::vector<HostJob> hj(njobs);
  for (uint32_t i = 0; i < njobs; ++i) {
    const hentt_ct_job &j = jobs[i];
    if (!j.c || !j.d || !j.out || !j.t || j.batch == 0 || j.reserved != 0) return HENTT_EINVAL;
    if ((uint64_t)j.batch * j.t->limbs >= (1ull << 24)) return HENTT_EINVAL;
    hj[i] = HostJob{j.c, j.d, j.out, j.t, j.batch};
  }
  if (int rc = check_overlaps(hj)) return rc;
  // largest N first; the caller's order within one N
  std::stable_sort(hj.begin(), hj.end(),
                   [](const HostJob &x, const HostJob &y) { return x.t->s->log_n > y.t->s->log_n; });
  const bool in_coeff = !(flags & HENTT_IN_NTT), out_coeff = !(flags & HENTT_OUT_NTT);
  // chunks: runs of one N, at most kGroupJobs jobs and 2^24 units each
  struct Chunk {
    uint32_t first, n;
    uint64_t ws;
  };
  std::vector<Chunk> chunks;
  uint64_t ws_max = 0;
  for (uint32_t i = 0; i < njobs;) {
    const uint32_t ln = hj[i].t->s->log_n;
    Chunk ch{i, 0, 0};
    uint64_t units = 0;
    while (i < njobs && hj[i].t->s->log_n == ln && ch.n < (uint32_t)kGroupJobs &&
           units + (uint64_t)hj[i].batch * hj[i].t->limbs < (1ull << 24)) {
      units += (uint64_t)hj[i].batch * hj[i].t->limbs;
      if (in_coeff && grouped_pec((int)ln) > 0) ch.ws += ws_words(hj[i]);
      ++ch.n;
      ++i;
    }
    ws_max = std::max(ws_max, ch.ws);
    chunks.push_back(ch);
  }
  hipStream_t st = (hipStream_t)stream;
  void *ws = nullptr;
  if (ws_max) {
    // one buffer for the call: the chunks run one after another on `st`
    int rc = pool_get((size_t)ws_max * 8ull, st, &ws);
    if (rc) return rc;
  }
  int rc = HENTT_OK;
  for (const Chunk &ch : chunks) {
    const uint32_t ln = hj[ch.first].t->s->log_n;
    rc = k_group_fn[ln - HENTT_LOG_N_MIN](&hj[ch.first], ch.n, in_coeff, out_coeff, (uint64_t *)ws, st);
    if (rc) break;
  }
  hipError_t e = hipGetLastError();
  if (ws) pool_put(ws);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e);
  return HENTT_OK;
}
