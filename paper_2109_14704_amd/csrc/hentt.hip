// libhentt: C ABI, twiddle tables, workspace pool, launch timing, argument
// checks and the plans of uneven batches.  The kernel families are dispatched
// from their own translation units (tr_*.hip).
#include <hip/hip_runtime.h>
#include <dlfcn.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <new>

#include "batch_kernels.hpp"
#include "host_tables.hpp"
#include "runtime.hpp"

using namespace hentt;
using namespace hentt_rt;

namespace hentt_rt {

thread_local int g_last_hip = 0;

// ------------------------------------------------------------ table storage
void retain(Storage *s) { s->refs.fetch_add(1); }

void release(Storage *s) {
  if (s->refs.fetch_sub(1) == 1) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(s->device);
    if (s->d_tw) (void)hipFree(s->d_tw);
    if (s->d_lc) (void)hipFree(s->d_lc);
    if (s->d_lcm) (void)hipFree(s->d_lcm);
    if (s->d_mont) (void)hipFree(s->d_mont);
    for (auto &kv : s->rs) (void)hipFree(kv.second);
    for (auto &kv : s->ks) (void)hipFree(kv.second);
    (void)hipSetDevice(cur);
    delete s;
  }
}

// ------------------------------------------------------------ workspace pool
// Device buffers reused by capacity: a request takes the smallest free buffer
// of its device and stream that is large enough, else allocates (the memory
// cache of section III-C-1).  hentt_pool_trim frees the idle ones.
namespace {
struct PoolEntry {
  void *ptr;
  size_t bytes;
  int device;
  hipStream_t stream;
  bool busy;
};
std::mutex g_pool_mu;
std::vector<PoolEntry> g_pool;
}  // namespace

// Frees the idle buffers after waiting for the streams that last used them
// (caller holds g_pool_mu).
static void pool_trim_locked() {
  int cur = 0;
  (void)hipGetDevice(&cur);
  std::vector<PoolEntry> keep;
  for (auto &e : g_pool) {
    if (e.busy) {
      keep.push_back(e);
      continue;
    }
    // queued work may still use the buffer: wait for its stream first
    (void)hipSetDevice(e.device);
    (void)hipStreamSynchronize(e.stream);
    (void)hipFree(e.ptr);
  }
  (void)hipSetDevice(cur);
  g_pool.swap(keep);
}

// Soft cap on the pool's bytes from HENTT_POOL_MAX_BYTES (0 or unset: none).
static uint64_t pool_cap() {
  static const uint64_t cap = [] {
    const char *v = getenv("HENTT_POOL_MAX_BYTES");
    return v ? strtoull(v, nullptr, 10) : 0ull;
  }();
  return cap;
}

namespace {
typedef int (*roctx_push_fn)(const char *);
typedef int (*roctx_pop_fn)();
struct Roctx {
  roctx_push_fn push = nullptr;
  roctx_pop_fn pop = nullptr;
};
const Roctx &roctx() {
  static const Roctx r = [] {
    Roctx x;
    const char *v = getenv("HENTT_ROCTX");
    if (!v || strcmp(v, "1") != 0) return x;
    void *h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (!h) return x;
    x.push = (roctx_push_fn)dlsym(h, "roctxRangePushA");
    x.pop = (roctx_pop_fn)dlsym(h, "roctxRangePop");
    if (!x.push || !x.pop) x = Roctx{};
    return x;
  }();
  return r;
}
}  // namespace

ApiRange::ApiRange(const char *name) : on(roctx().push != nullptr) {
  if (on) roctx().push(name);
}
ApiRange::~ApiRange() {
  if (on) roctx().pop();
}

int pool_get(size_t bytes, hipStream_t stream, void **out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_pool_mu);
  int best = -1;
  for (size_t i = 0; i < g_pool.size(); ++i) {
    PoolEntry &e = g_pool[i];
    if (e.busy || e.device != dev || e.bytes < bytes) continue;
    if (e.stream != stream) continue;  // reuse only in the stream order that last used it
    if (best < 0 || e.bytes < g_pool[best].bytes) best = (int)i;
  }
  if (best >= 0) {
    g_pool[best].busy = true;
    *out = g_pool[best].ptr;
    return HENTT_OK;
  }
  if (const uint64_t cap = pool_cap()) {
    uint64_t held = 0;
    for (auto &pe : g_pool) held += pe.bytes;
    if (held + bytes > cap) pool_trim_locked();  // idle buffers go before the pool grows past the cap
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    return HENTT_ENOMEM;
  }
  g_pool.push_back({p, bytes, dev, stream, true});
  *out = p;
  return HENTT_OK;
}

void pool_put(void *p) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  for (auto &e : g_pool)
    if (e.ptr == p) e.busy = false;
}

// ------------------------------------------------------------ launch timing
std::atomic<bool> g_prof_on{false};
thread_local bool g_timer_off = false;
namespace {
struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};
struct ProfAgg {
  std::string name;
  double ms;
  uint32_t n;
};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof;
std::vector<ProfAgg> g_prof_agg;
}  // namespace

void prof_record(const char *name, int log_n, hipEvent_t a, hipEvent_t b) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.push_back({std::string(name) + "<" + std::to_string(log_n) + ">", a, b});
}

}  // namespace hentt_rt

// ------------------------------------------------------------ input check
namespace {

// Debug check of the input contract (canonical residues, [0, q_l)): one
// workgroup per tile of 2048 words of one (batch entry, limb), the modulus
// uniform per workgroup.  res[0] counts the words x >= q; res[1] is the
// smallest flat index of such a word (starts at ~0).
__global__ __launch_bounds__(256) void k_check_canonical(const uint64_t *__restrict__ x,
                                                         const LimbConst *__restrict__ lc, uint32_t limbs,
                                                         uint32_t log_n, uint32_t tiles,
                                                         unsigned long long *res) {
  const uint32_t poly = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  const uint64_t q = lc[poly % limbs].m.q;
  const uint32_t n = 1u << log_n;
  const uint64_t base = ((uint64_t)poly << log_n) + (uint64_t)tile * 2048u;
  unsigned long long bad = 0, first = ~0ull;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const uint32_t i = tile * 2048u + threadIdx.x + 256u * s;
    if (i < n && x[base + threadIdx.x + 256u * s] >= q) {
      ++bad;
      if (first == ~0ull) first = base + threadIdx.x + 256u * s;
    }
  }
  if (bad) {
    atomicAdd(&res[0], bad);
    atomicMin(&res[1], first);
  }
}

__global__ void k_check_init(unsigned long long *res) {
  if (threadIdx.x == 0) {
    res[0] = 0;
    res[1] = ~0ull;
  }
}

}  // namespace

// ------------------------------------------------------------ uneven batches
struct hentt_batch_plan {
  int dir = 1;
  int device = 0;
  uint32_t nunits = 0, ntiles = 0, grid = 0, nq = 0;
  uint32_t look_pct = 200;               // pass-2 lookahead, percent of the workgroups serving a queue
  uint32_t group_max = 8;                // units of one twiddle table ordered block-major together
  std::vector<BatchUnit> units;          // host copy (queues are rebuilt when the grid changes)
  BatchUnit *d_units = nullptr;
  BatchTile *d_tiles = nullptr;
  uint32_t *d_qoff = nullptr;            // BATCH_NQ + 1 tile offsets
  uint32_t *d_qmap = nullptr;            // 16 entries: XCC_ID -> queue (or ~0)
  uint32_t *d_ctl = nullptr;             // BATCH_NQ + 1 + nunits words
  std::vector<uint32_t> qlen;
  std::vector<hentt_job> small;          // jobs with N < 2^12: ordinary launches
  std::vector<hentt_tables> small_views;
  std::vector<Storage *> storages;       // tables the plan points into, one reference each
  std::atomic<int> graphs{0};            // live graphs captured from this plan
  hipEvent_t done = nullptr;             // recorded after every run and every graph replay
};

struct hentt_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hentt_batch_plan *plan = nullptr;
};

namespace {

const uint32_t kSpinLimit = 1u << 22;   // bounded wait of a pass-2 tile (s_sleep 2 per try)

// Every workgroup of the persistent kernel resident at once: the kernel's
// occupancy per compute unit (LDS and VGPRs allow four 256-lane workgroups on
// gfx950) times the compute units.
int default_grid() {
  int dev = 0, cus = 256, per_f = 0, per_i = 0;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_f, k_batch<false>, BATCH_LANES, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_i, k_batch<true>, BATCH_LANES, 0) != hipSuccess)
    per_f = per_i = 2;
  const int per = per_f < per_i ? per_f : per_i;
  return cus * (per < 1 ? 1 : per);
}

void plan_free(hentt_batch_plan *p) {
  if (p->done) (void)hipEventSynchronize(p->done), (void)hipEventDestroy(p->done);
  for (void *d : {(void *)p->d_units, (void *)p->d_tiles, (void *)p->d_qoff, (void *)p->d_qmap, (void *)p->d_ctl})
    if (d) (void)hipFree(d);
  for (Storage *s : p->storages) release(s);
  delete p;
}

uint32_t pass1_tiles(uint32_t ln, int dir) {
  if (ln == BATCH_B) return 0;
  return dir > 0 ? batch_col_tiles(ln) : (1u << (ln - BATCH_B));
}
uint32_t pass2_tiles(uint32_t ln, int dir) {
  if (ln == BATCH_B) return 0;
  return dir > 0 ? (1u << (ln - BATCH_B)) : batch_col_tiles(ln);
}

// Places the plan's workgroups (probe kernel), maps XCDs to queues, spreads
// the units over the queues (largest first, least-loaded queue) and orders
// each queue.  A queue is two streams merged: pass-1 (and whole) tiles, and
// pass-2 tiles, each grouped by twiddle table.  A group's pass-2 tiles are placed at
// least LOOK tiles after the group's last pass-1 tile, where LOOK is a
// multiple of the number of workgroups serving the queue (twice by default):
// by the time a workgroup takes the pass-2 tile, the workgroups that took
// those pass-1 tiles have most likely finished them, so the dependency wait
// is rarely taken.  A shorter lookahead keeps a unit's pass-1 results more
// likely in the XCD's L2 when pass 2 reads them, at the price of more waits.
int plan_queues(hentt_batch_plan *p) {
  const uint32_t grid = std::max(1u, p->grid);
  uint32_t *d_probe = nullptr;
  HIPCHK(hipMalloc(&d_probe, grid * sizeof(uint32_t)));
  hipLaunchKernelGGL(k_xcc_probe, dim3(grid), dim3(64), 0, 0, d_probe);
  std::vector<uint32_t> where(grid);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpy(where.data(), d_probe, grid * sizeof(uint32_t), hipMemcpyDeviceToHost);
  (void)hipFree(d_probe);
  if (e != hipSuccess) return hip_fail(e);
  uint32_t qmap[16];
  for (auto &m : qmap) m = ~0u;
  uint32_t nq = 0;
  for (uint32_t x : where)
    if (qmap[x & 15] == ~0u && nq < BATCH_NQ) qmap[x & 15] = nq++;
  p->nq = nq;
  std::vector<uint32_t> served(BATCH_NQ, 0);  // workgroups serving each queue
  for (uint32_t x : where)
    if (qmap[x & 15] < BATCH_NQ) ++served[qmap[x & 15]];
  // Units that share a twiddle table (same limb, size and direction) go to
  // one queue back to back, so that the table is read into that XCD's L2 once
  // rather than from memory per unit: the block pass of an N = 2^17
  // transform reads about as many twiddle bytes as data bytes.  Groups are cut
  // into pieces of at most half a fair share (cost ~ N log N per unit) and the
  // pieces placed largest first on the least-loaded queue; each queue then
  // runs its pieces largest N first.
  auto cost = [&](uint32_t i) { return (double)(1u << p->units[i].logn) * p->units[i].logn; };
  std::map<const Tw *, std::vector<uint32_t>> by_table;
  double total = 0;
  for (uint32_t i = 0; i < p->units.size(); ++i) {
    by_table[p->units[i].tw].push_back(i);
    total += cost(i);
  }
  const double cap = std::max(total / nq / 2, 1.0);
  std::vector<std::vector<uint32_t>> pieces;
  for (auto &g : by_table) {
    std::vector<uint32_t> cur;
    double c = 0;
    for (uint32_t i : g.second) {
      if (!cur.empty() && c + cost(i) > cap) {
        pieces.push_back(cur);
        cur.clear();
        c = 0;
      }
      cur.push_back(i);
      c += cost(i);
    }
    if (!cur.empty()) pieces.push_back(cur);
  }
  auto piece_cost = [&](const std::vector<uint32_t> &pc) { return cost(pc[0]) * pc.size(); };
  std::stable_sort(pieces.begin(), pieces.end(),
                   [&](const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) { return piece_cost(a) > piece_cost(b); });
  std::vector<std::vector<const std::vector<uint32_t> *>> qpieces(nq);
  std::vector<double> load(nq, 0.0);
  for (const auto &pc : pieces) {
    uint32_t best = 0;
    for (uint32_t k = 1; k < nq; ++k)
      if (load[k] < load[best]) best = k;
    qpieces[best].push_back(&pc);
    load[best] += piece_cost(pc);
  }
  std::vector<std::vector<uint32_t>> qunits(nq);
  for (uint32_t k = 0; k < nq; ++k) {
    std::stable_sort(qpieces[k].begin(), qpieces[k].end(), [&](const std::vector<uint32_t> *a, const std::vector<uint32_t> *b) {
      return p->units[(*a)[0]].logn > p->units[(*b)[0]].logn;
    });
    for (const auto *pc : qpieces[k]) qunits[k].insert(qunits[k].end(), pc->begin(), pc->end());
  }
  std::vector<BatchTile> tiles;
  std::vector<uint32_t> qoff(BATCH_NQ + 1, 0);
  std::vector<size_t> ready(p->units.size(), 0);  // queue position after a unit's last pass-1 tile
  for (uint32_t k = 0; k < BATCH_NQ; ++k) {
    qoff[k] = (uint32_t)tiles.size();
    if (k >= nq) continue;
    const size_t look = (size_t)served[k] * p->look_pct / 100;
    const std::vector<uint32_t> &us = qunits[k];
    // groups: runs of at most group_max consecutive units sharing a twiddle
    // table (short runs keep column tiles, which are HBM-bound, interleaved
    // with block tiles, which are ALU-bound)
    std::vector<std::vector<uint32_t>> groups;
    for (uint32_t i : us) {
      if (groups.empty() || p->units[groups.back()[0]].tw != p->units[i].tw || groups.back().size() >= p->group_max)
        groups.emplace_back();
      groups.back().push_back(i);
    }
    // Block passes read about as many twiddle bytes per block as data bytes,
    // and block b of every unit of a group reads the same twiddles: their
    // tiles go block-major across the group's units, so that consecutive
    // tiles (run at about the same time) share the twiddles in L2.  Column
    // passes read a few scalar twiddles per column: unit-major.
    const bool p1_blocks = p->dir < 0;  // inverse: pass 1 = blocks, pass 2 = columns
    std::vector<BatchTile> first;       // whole and pass-1 tiles
    std::vector<uint32_t> first_group;
    std::vector<size_t> gleft(groups.size(), 0), gready(groups.size(), 0);
    for (uint32_t gi = 0; gi < groups.size(); ++gi) {
      const std::vector<uint32_t> &g = groups[gi];
      const BatchUnit &u0 = p->units[g[0]];
      if (u0.logn == BATCH_B) {
        for (uint32_t i : g) first.push_back({i, (uint32_t)BT_WHOLE << 16}), first_group.push_back(gi);
        continue;
      }
      const uint32_t n1 = u0.pass1;
      gleft[gi] = (size_t)n1 * g.size();
      if (p1_blocks) {
        for (uint32_t t = 0; t < n1; ++t)
          for (uint32_t i : g) first.push_back({i, ((uint32_t)BT_PASS1 << 16) | t}), first_group.push_back(gi);
      } else {
        for (uint32_t i : g)
          for (uint32_t t = 0; t < n1; ++t) first.push_back({i, ((uint32_t)BT_PASS1 << 16) | t}), first_group.push_back(gi);
      }
    }
    size_t next = 0;
    auto emit_first = [&]() {
      const BatchTile bt = first[next];
      const uint32_t gi = first_group[next++];
      tiles.push_back(bt);
      if ((bt.kind_idx >> 16) == BT_PASS1 && --gleft[gi] == 0) gready[gi] = tiles.size();
    };
    for (uint32_t gi = 0; gi < groups.size(); ++gi) {
      const std::vector<uint32_t> &g = groups[gi];
      const uint32_t n2 = pass2_tiles(p->units[g[0]].logn, p->dir);
      if (n2 == 0) continue;
      // every pass-1 tile of the group is queued, and LOOK more tiles after it
      while (next < first.size() && (gready[gi] == 0 || tiles.size() < gready[gi] + look)) emit_first();
      if (!p1_blocks) {
        for (uint32_t t = 0; t < n2; ++t)
          for (uint32_t i : g) tiles.push_back({i, ((uint32_t)BT_PASS2 << 16) | t});
      } else {
        for (uint32_t i : g)
          for (uint32_t t = 0; t < n2; ++t) tiles.push_back({i, ((uint32_t)BT_PASS2 << 16) | t});
      }
    }
    while (next < first.size()) emit_first();
  }
  qoff[BATCH_NQ] = (uint32_t)tiles.size();
  p->ntiles = (uint32_t)tiles.size();
  p->qlen.assign(BATCH_NQ, 0);
  for (uint32_t k = 0; k < BATCH_NQ; ++k) p->qlen[k] = qoff[k + 1] - qoff[k];
  // the tile count does not depend on the grid: the buffer is made once and
  // keeps its address when the grid changes
  if (!p->d_tiles) e = hipMalloc(&p->d_tiles, std::max<size_t>(1, tiles.size()) * sizeof(BatchTile));
  if (e == hipSuccess && !tiles.empty())
    e = hipMemcpy(p->d_tiles, tiles.data(), tiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_qoff, qoff.data(), qoff.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_qmap, qmap, sizeof(qmap), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e);
  return HENTT_OK;
}

int plan_build(const hentt_job *jobs, uint32_t njobs, int dir, hentt_batch_plan **out) {
  if (!jobs || njobs == 0 || !out || (dir != 1 && dir != -1)) return HENTT_EINVAL;
  for (uint32_t j = 0; j < njobs; ++j) {
    const hentt_job &jb = jobs[j];
    if (!jb.data || !jb.t || jb.batch == 0 || jb.limbs == 0 || jb.limbs > jb.t->limbs) return HENTT_EINVAL;
  }
  hentt_batch_plan *p = new (std::nothrow) hentt_batch_plan();
  if (!p) return HENTT_ENOMEM;
  p->dir = dir;
  (void)hipGetDevice(&p->device);
  for (uint32_t j = 0; j < njobs; ++j)  // one reference per table storage the plan points into
    if (std::find(p->storages.begin(), p->storages.end(), jobs[j].t->s) == p->storages.end()) {
      retain(jobs[j].t->s);
      p->storages.push_back(jobs[j].t->s);
    }
  for (uint32_t j = 0; j < njobs; ++j) {
    const hentt_job &jb = jobs[j];
    const uint32_t ln = jb.t->s->log_n;
    const uint64_t N = 1ull << ln;
    if (ln < BATCH_B) {
      p->small.push_back(jb);
      continue;
    }
    for (uint32_t b = 0; b < jb.batch; ++b)
      for (uint32_t l = 0; l < jb.limbs; ++l) {
        BatchUnit u;
        u.data = jb.data + ((uint64_t)b * jb.limbs + l) * N;
        u.tw = jb.t->s->d_tw + ((size_t)l * 2 + (dir < 0 ? 1 : 0)) * N;
        u.lc = jb.t->s->d_lc + l;
        u.logn = ln;
        u.pass1 = pass1_tiles(ln, dir);
        p->units.push_back(u);
      }
  }
  for (auto &sj : p->small) p->small_views.push_back(hentt_tables{sj.t->s, sj.limbs});
  p->nunits = (uint32_t)p->units.size();
  p->grid = (uint32_t)default_grid();
  hipError_t e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
  if (p->nunits && e == hipSuccess) {
    e = hipMalloc(&p->d_units, p->units.size() * sizeof(BatchUnit));
    if (e == hipSuccess) e = hipMalloc(&p->d_qoff, (BATCH_NQ + 1) * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&p->d_qmap, 16 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&p->d_ctl, (BATCH_NQ + 1 + p->units.size()) * sizeof(uint32_t));
    if (e == hipSuccess)
      e = hipMemcpy(p->d_units, p->units.data(), p->units.size() * sizeof(BatchUnit), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    plan_free(p);
    g_last_hip = (int)e;
    return e == hipErrorOutOfMemory ? HENTT_ENOMEM : HENTT_EHIP;
  }
  if (p->nunits) {
    int rc = plan_queues(p);
    if (rc) {
      plan_free(p);
      return rc;
    }
  }
  *out = p;
  return HENTT_OK;
}

int plan_launch(hentt_batch_plan *p, hipStream_t st) {
  const int LOGN = 0;  // timer label
  if (p->nunits) {
    const uint32_t n = BATCH_NQ + 1 + p->nunits;
    hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024), dim3(256), 0, st, p->d_ctl, n, 0u);
    HIPCHK(hipGetLastError());
    const uint32_t grid = p->grid;  // every workgroup of the probed placement (idle ones exit at once)
    if (p->dir > 0) {
      LaunchTimer lt_("k_batch_fwd", LOGN, st);
      hipLaunchKernelGGL(k_batch<false>, dim3(grid), dim3(BATCH_LANES), 0, st, p->d_units, p->d_tiles, p->d_qoff,
                         p->d_qmap, p->d_ctl, kSpinLimit);
    } else {
      LaunchTimer lt_("k_batch_inv", LOGN, st);
      hipLaunchKernelGGL(k_batch<true>, dim3(grid), dim3(BATCH_LANES), 0, st, p->d_units, p->d_tiles, p->d_qoff,
                         p->d_qmap, p->d_ctl, kSpinLimit);
    }
    HIPCHK(hipGetLastError());
  }
  for (size_t i = 0; i < p->small.size(); ++i) {
    int rc = run_transform(&p->small_views[i], p->small[i].data, p->small[i].batch, st, p->dir < 0);
    if (rc) return rc;
  }
  return HENTT_OK;
}

int plan_status(hentt_batch_plan *p) {
  if (!p->nunits) return HENTT_OK;
  HIPCHK(hipEventSynchronize(p->done));
  uint32_t h[BATCH_NQ + 1];
  HIPCHK(hipMemcpy(h, p->d_ctl, sizeof(h), hipMemcpyDeviceToHost));
  if (h[BATCH_NQ]) return HENTT_ETIMEOUT;
  for (uint32_t k = 0; k < BATCH_NQ; ++k)
    if (h[k] < p->qlen[k]) return HENTT_ETIMEOUT;  // a queue no workgroup served
  return HENTT_OK;
}

// Plans made by hentt_ntt_batch, keyed by the job list (bounded cache).  A
// plan holds a reference on every table storage it points into, so its
// device pointers stay valid; destroying a table evicts the plans that use
// its storage.  Entries are shared pointers: a plan evicted while another
// thread runs it is freed when that run has been enqueued.
std::mutex g_plan_mu;
std::map<std::vector<uint64_t>, std::shared_ptr<hentt_batch_plan>> g_plans;
const size_t kPlanCacheMax = 16;

std::vector<uint64_t> plan_key(const hentt_job *jobs, uint32_t njobs, int dir) {
  std::vector<uint64_t> key;
  key.push_back((uint64_t)(int64_t)dir);
  for (uint32_t j = 0; j < njobs; ++j) {
    key.push_back((uint64_t)(uintptr_t)jobs[j].data);
    key.push_back((uint64_t)(uintptr_t)jobs[j].t->s);
    key.push_back(((uint64_t)jobs[j].t->s->log_n << 48) ^ ((uint64_t)jobs[j].limbs << 32) ^ jobs[j].batch);
  }
  return key;
}

std::shared_ptr<hentt_batch_plan> cached_plan(const std::vector<uint64_t> &key) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto it = g_plans.find(key);
  return it == g_plans.end() ? nullptr : it->second;
}

void evict_plans_of(Storage *s) {
  std::vector<std::shared_ptr<hentt_batch_plan>> gone;  // freed outside the lock
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto it = g_plans.begin(); it != g_plans.end();) {
      const auto &st = it->second->storages;
      if (std::find(st.begin(), st.end(), s) != st.end()) {
        gone.push_back(it->second);
        it = g_plans.erase(it);
      } else {
        ++it;
      }
    }
  }
}

}  // namespace

// ================================================================== C ABI
extern "C" {

const char *hentt_status_str(int s) {
  switch (s) {
    case HENTT_OK: return "ok";
    case HENTT_EINVAL: return "invalid argument";
    case HENTT_EMODULUS: return "bad modulus (must be prime, 1 mod 2N, 2^7 < q < 2^60)";
    case HENTT_ENOMEM: return "out of memory";
    case HENTT_EHIP: return "HIP runtime error";
    case HENTT_ETIMEOUT: return "a batch tile waited past its spin limit (results incomplete)";
    case HENTT_EBUSY: return "the plan has live graphs (destroy them first)";
    case HENTT_ENONCANON: return "input words outside [0, q)";
    case HENTT_ESCRATCH: return "the call needs more workspace than the static scratch array holds";
    default: return "unknown status";
  }
}

int hentt_last_hip_error(void) { return g_last_hip; }

int hentt_stage_split(uint32_t log_n, uint32_t *transform_cols, uint32_t *product_cols) {
  if (!transform_cols || !product_cols || log_n < HENTT_LOG_N_MIN || log_n > HENTT_LOG_N_MAX) return HENTT_EINVAL;
  stage_split(log_n, transform_cols, product_cols);
  return HENTT_OK;
}

int hentt_psi(uint64_t q, uint32_t log_n, uint64_t *psi) {
  if (!psi || log_n < 1 || log_n > 30) return HENTT_EINVAL;
  if (q < 3 || (q - 1) % (2ull << log_n) != 0 || !host::is_prime(q)) return HENTT_EMODULUS;
  const uint64_t p = host::psi(q, (int)log_n);
  if (!p) return HENTT_EMODULUS;
  *psi = p;
  return HENTT_OK;
}

int hentt_tables_create(uint32_t log_n, uint32_t limbs, const uint64_t *moduli_host, void *stream,
                        hentt_tables **out) {
  if (!out || !moduli_host || limbs == 0 || limbs > HENTT_LIMBS_MAX) return HENTT_EINVAL;
  if (log_n < HENTT_LOG_N_MIN || log_n > HENTT_LOG_N_MAX) return HENTT_EINVAL;
  *out = nullptr;
  for (uint32_t l = 0; l < limbs; ++l)
    if (!host::modulus_ok(moduli_host[l], (int)log_n)) return HENTT_EMODULUS;
  const uint32_t N = 1u << log_n;
  std::vector<Tw> tw((size_t)limbs * 2 * N);
  std::vector<LimbConst> lc(limbs), lcm(limbs);
  std::vector<MontLimb> mont(limbs);
  std::vector<uint64_t> pw(N), ipw(N);
  for (uint32_t l = 0; l < limbs; ++l) {
    Tw *f = &tw[(size_t)l * 2 * N];
    if (!host::make_limb(moduli_host[l], (int)log_n, f, f + N, lc[l], lcm[l], mont[l], pw.data(), ipw.data()))
      return HENTT_EMODULUS;
  }
  Storage *s = new (std::nothrow) Storage();
  if (!s) return HENTT_ENOMEM;
  s->log_n = log_n;
  s->limbs = limbs;
  s->moduli.assign(moduli_host, moduli_host + limbs);
  (void)hipGetDevice(&s->device);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMalloc(&s->d_tw, tw.size() * sizeof(Tw));
  if (e == hipSuccess) e = hipMalloc(&s->d_lc, lc.size() * sizeof(LimbConst));
  if (e == hipSuccess) e = hipMemcpyAsync(s->d_tw, tw.data(), tw.size() * sizeof(Tw), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMalloc(&s->d_lcm, lcm.size() * sizeof(LimbConst));
  if (e == hipSuccess) e = hipMalloc(&s->d_mont, mont.size() * sizeof(MontLimb));
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_lc, lc.data(), lc.size() * sizeof(LimbConst), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_lcm, lcm.data(), lcm.size() * sizeof(LimbConst), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_mont, mont.data(), mont.size() * sizeof(MontLimb), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    release(s);
    g_last_hip = (int)e;
    return e == hipErrorOutOfMemory ? HENTT_ENOMEM : HENTT_EHIP;
  }
  hentt_tables *h = new (std::nothrow) hentt_tables{s, limbs};
  if (!h) {
    release(s);
    return HENTT_ENOMEM;
  }
  *out = h;
  return HENTT_OK;
}

int hentt_tables_destroy(hentt_tables *t) {
  if (!t) return HENTT_EINVAL;
  evict_plans_of(t->s);
  release(t->s);
  delete t;
  return HENTT_OK;
}

int hentt_tables_view(const hentt_tables *t, uint32_t limbs, hentt_tables **view) {
  if (!t || !view || limbs == 0 || limbs > t->limbs) return HENTT_EINVAL;
  hentt_tables *h = new (std::nothrow) hentt_tables{t->s, limbs};
  if (!h) return HENTT_ENOMEM;
  retain(t->s);
  *view = h;
  return HENTT_OK;
}

int hentt_tables_info(const hentt_tables *t, uint32_t *log_n, uint32_t *limbs) {
  if (!t) return HENTT_EINVAL;
  if (log_n) *log_n = t->s->log_n;
  if (limbs) *limbs = t->limbs;
  return HENTT_OK;
}

int hentt_tables_device_ptrs(const hentt_tables *t, const uint64_t **fwd, const uint64_t **inv,
                             const uint64_t **moduli) {
  if (!t) return HENTT_EINVAL;
  const size_t N = 1u << t->s->log_n;
  // per limb: fwd pairs then inv pairs; callers index limb l at l * 2N pairs
  if (fwd) *fwd = (const uint64_t *)t->s->d_tw;
  if (inv) *inv = (const uint64_t *)(t->s->d_tw + N);
  if (moduli) *moduli = (const uint64_t *)t->s->d_lc;
  return HENTT_OK;
}

int hentt_check_canonical(const hentt_tables *t, const uint64_t *x, uint32_t batch, uint64_t *bad_words,
                          uint64_t *first_bad, void *stream) {
  ApiRange range_("hentt_check_canonical");
  if (!t || !x || batch == 0) return HENTT_EINVAL;
  const uint32_t ln = t->s->log_n;
  const uint32_t tiles = ln > 11 ? (1u << (ln - 11)) : 1u;
  const uint64_t grid = (uint64_t)batch * t->limbs * tiles;
  if (grid > 0x7fffffffu) return HENTT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  void *res = nullptr;
  int rc = pool_get(2 * sizeof(unsigned long long), st, &res);
  if (rc) return rc;
  unsigned long long h[2] = {0, ~0ull};
  hipLaunchKernelGGL(k_check_init, dim3(1), dim3(64), 0, st, (unsigned long long *)res);
  hipLaunchKernelGGL(k_check_canonical, dim3((uint32_t)grid), dim3(256), 0, st, x, t->s->d_lc, t->limbs, ln, tiles,
                     (unsigned long long *)res);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  pool_put(res);
  if (e != hipSuccess) return hip_fail(e);
  if (bad_words) *bad_words = h[0];
  if (first_bad) *first_bad = h[1];
  return h[0] ? HENTT_ENONCANON : HENTT_OK;
}

int hentt_ntt_fwd(const hentt_tables *t, uint64_t *x, uint32_t batch, void *stream) {
  ApiRange range_("hentt_ntt_fwd");
  if (!t || !x || batch == 0) return HENTT_EINVAL;
  return run_transform(t, x, batch, (hipStream_t)stream, false);
}

int hentt_ntt_inv(const hentt_tables *t, uint64_t *x, uint32_t batch, void *stream) {
  ApiRange range_("hentt_ntt_inv");
  if (!t || !x || batch == 0) return HENTT_EINVAL;
  return run_transform(t, x, batch, (hipStream_t)stream, true);
}

int hentt_ntt_fwd_variant(const hentt_tables *t, uint64_t *x, uint32_t batch, int variant, void *stream) {
  ApiRange range_("hentt_ntt_fwd_variant");
  if (!t || !x || batch == 0) return HENTT_EINVAL;
  return run_fwd_variant(t, x, batch, variant, (hipStream_t)stream);
}

}  // extern "C"

namespace {
// [p, p + bytes) as an address range.
struct Span {
  uintptr_t a, b;
};
Span span(const void *p, uint64_t words) { return Span{(uintptr_t)p, (uintptr_t)p + (uintptr_t)(words * 8)}; }
bool overlap(Span x, Span y) { return x.a < y.b && y.a < x.b; }
}  // namespace

extern "C" {

int hentt_rescale(const hentt_tables *t, const uint64_t *c, uint64_t *out, uint32_t batch, uint32_t flags,
                  void *stream) {
  ApiRange range_("hentt_rescale");
  if (!t || !c || !out || batch == 0 || t->limbs < 2) return HENTT_EINVAL;
  const bool ntt = flags == (HENTT_IN_NTT | HENTT_OUT_NTT);
  if (!ntt && flags != 0) return HENTT_EINVAL;
  const uint64_t N = 1ull << t->s->log_n;
  if (overlap(span(c, batch * (uint64_t)t->limbs * N), span(out, batch * (uint64_t)(t->limbs - 1) * N)))
    return HENTT_EINVAL;
  return run_rescale(t, c, out, batch, ntt, (hipStream_t)stream);
}

int hentt_ct_matmul(const hentt_tables *t, const uint64_t *A, const uint64_t *B, uint64_t *C, uint32_t m, uint32_t n,
                    uint32_t k, void *stream) {
  ApiRange range_("hentt_ct_matmul");
  if (!t || !A || !B || !C || m == 0 || n == 0 || k == 0) return HENTT_EINVAL;
  const uint64_t P = (uint64_t)t->limbs << t->s->log_n;
  const Span c = span(C, (uint64_t)m * n * 3 * P);
  if (overlap(c, span(A, (uint64_t)m * k * 2 * P)) || overlap(c, span(B, (uint64_t)k * n * 2 * P)))
    return HENTT_EINVAL;
  return run_matmul(t, A, B, C, m, n, k, (hipStream_t)stream);
}

int hentt_relin(const hentt_tables *t, const uint64_t *c, const uint64_t *ksk, uint64_t *out, uint32_t batch,
                void *stream) {
  ApiRange range_("hentt_relin");
  if (!t || !c || !ksk || !out || batch == 0 || t->limbs < 2) return HENTT_EINVAL;
  const uint64_t N = 1ull << t->s->log_n, l = t->limbs - 1;
  const Span o = span(out, batch * 2 * l * N);
  if (overlap(o, span(c, batch * 3 * l * N)) || overlap(o, span(ksk, l * 2 * (l + 1) * N))) return HENTT_EINVAL;
  return run_relin(t, c, ksk, out, batch, (hipStream_t)stream);
}

int hentt_dyadic_mul(const hentt_tables *t, const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t batch,
                     void *stream) {
  ApiRange range_("hentt_dyadic_mul");
  if (!t || !a || !b || !out || batch == 0) return HENTT_EINVAL;
  const uint64_t words = (uint64_t)batch * t->limbs << t->s->log_n;
  const Span o = span(out, words);
  // element-wise: out may be a or b exactly, but no partial overlap
  if ((out != a && overlap(o, span(a, words))) || (out != b && overlap(o, span(b, words)))) return HENTT_EINVAL;
  ProdArgs pa{};
  pa.in[0] = a;
  pa.in[1] = b;
  pa.out[0] = out;
  pa.in_sb = pa.out_sb = (uint64_t)t->limbs << t->s->log_n;
  return run_prod(t, PROD_MUL, pa, batch, false, false, (hipStream_t)stream);
}

int hentt_polymul(const hentt_tables *t, const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t batch,
                  void *stream) {
  ApiRange range_("hentt_polymul");
  if (!t || !a || !b || !out || batch == 0) return HENTT_EINVAL;
  const uint64_t words = (uint64_t)batch * t->limbs << t->s->log_n;
  const Span o = span(out, words);
  if (overlap(o, span(a, words)) || overlap(o, span(b, words))) return HENTT_EINVAL;
  ProdArgs pa{};
  pa.in[0] = a;
  pa.in[1] = b;
  pa.out[0] = out;
  pa.in_sb = pa.out_sb = (uint64_t)t->limbs << t->s->log_n;
  return run_prod(t, PROD_MUL, pa, batch, true, true, (hipStream_t)stream);
}

int hentt_ct_tensor(const hentt_tables *t, const uint64_t *c, const uint64_t *d, uint64_t *out, uint32_t batch,
                    uint32_t flags, void *stream) {
  ApiRange range_("hentt_ct_tensor");
  if (!t || !c || !d || !out || batch == 0 || (flags & ~3u)) return HENTT_EINVAL;
  const uint64_t NL = (uint64_t)t->limbs << t->s->log_n;
  const Span o = span(out, 3 * NL * batch);
  if (overlap(o, span(c, 2 * NL * batch)) || overlap(o, span(d, 2 * NL * batch))) return HENTT_EINVAL;
  ProdArgs pa{};
  pa.in[0] = c;
  pa.in[1] = c + NL;
  pa.in[2] = d;
  pa.in[3] = d + NL;
  for (int o = 0; o < 3; ++o) pa.out[o] = out + o * NL;
  pa.in_sb = 2 * NL;
  pa.out_sb = 3 * NL;
  return run_prod(t, PROD_TENSOR, pa, batch, !(flags & HENTT_IN_NTT), !(flags & HENTT_OUT_NTT), (hipStream_t)stream);
}

int hentt_batch_plan_create(const hentt_job *jobs, uint32_t njobs, int dir, hentt_batch_plan **out) {
  return plan_build(jobs, njobs, dir, out);
}

int hentt_batch_plan_set_grid(hentt_batch_plan *p, uint32_t workgroups) {
  if (!p) return HENTT_EINVAL;
  if (p->graphs.load() > 0) return HENTT_EBUSY;  // captured graphs hold the old launch shape
  if (p->done) HIPCHK(hipEventSynchronize(p->done));
  p->grid = workgroups ? workgroups : (uint32_t)default_grid();
  return p->nunits ? plan_queues(p) : HENTT_OK;
}

int hentt_batch_plan_set_schedule(hentt_batch_plan *p, uint32_t lookahead_pct, uint32_t group_units) {
  if (!p || lookahead_pct > 10000 || group_units == 0 || group_units > 4096) return HENTT_EINVAL;
  if (p->graphs.load() > 0) return HENTT_EBUSY;  // captured graphs read the tile list being rewritten
  if (p->done) HIPCHK(hipEventSynchronize(p->done));
  p->look_pct = lookahead_pct;
  p->group_max = group_units;
  return p->nunits ? plan_queues(p) : HENTT_OK;
}

int hentt_batch_plan_info(const hentt_batch_plan *p, uint32_t *units, uint32_t *tiles, uint32_t *grid) {
  if (!p) return HENTT_EINVAL;
  if (units) *units = p->nunits;
  if (tiles) *tiles = p->ntiles;
  if (grid) *grid = p->grid;
  return HENTT_OK;
}

int hentt_batch_plan_run(hentt_batch_plan *p, void *stream) {
  ApiRange range_("hentt_batch_plan_run");
  if (!p) return HENTT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  int rc = plan_launch(p, st);
  if (rc) return rc;
  HIPCHK(hipEventRecord(p->done, st));
  return HENTT_OK;
}

int hentt_batch_plan_status(hentt_batch_plan *p) {
  if (!p) return HENTT_EINVAL;
  return plan_status(p);
}

int hentt_batch_plan_destroy(hentt_batch_plan *p) {
  if (!p) return HENTT_EINVAL;
  if (p->graphs.load() > 0) return HENTT_EBUSY;
  plan_free(p);
  return HENTT_OK;
}

int hentt_batch_graph_create(hentt_batch_plan *p, hentt_graph **out) {
  if (!p || !out) return HENTT_EINVAL;
  hipStream_t cs = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hentt_graph *g = new (std::nothrow) hentt_graph();
  if (!g) {
    (void)hipStreamDestroy(cs);
    return HENTT_ENOMEM;
  }
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  int rc = HENTT_OK;
  if (e == hipSuccess) rc = plan_launch(p, cs);
  hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess && !rc) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess || rc) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    if (rc) return rc;
    return hip_fail(e);
  }
  g->plan = p;
  p->graphs.fetch_add(1);
  *out = g;
  return HENTT_OK;
}

int hentt_graph_launch(hentt_graph *g, void *stream) {
  ApiRange range_("hentt_graph_launch");
  if (!g) return HENTT_EINVAL;
  HIPCHK(hipGraphLaunch(g->exec, (hipStream_t)stream));
  HIPCHK(hipEventRecord(g->plan->done, (hipStream_t)stream));  // hentt_batch_plan_status waits for this replay
  return HENTT_OK;
}

int hentt_graph_destroy(hentt_graph *g) {
  if (!g) return HENTT_EINVAL;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->plan) g->plan->graphs.fetch_sub(1);
  delete g;
  return HENTT_OK;
}

int hentt_ntt_batch(const hentt_job *jobs, uint32_t njobs, int dir, void *stream) {
  ApiRange range_("hentt_ntt_batch");
  if (!jobs || njobs == 0 || (dir != 1 && dir != -1)) return HENTT_EINVAL;
  for (uint32_t j = 0; j < njobs; ++j)
    if (!jobs[j].t) return HENTT_EINVAL;
  const std::vector<uint64_t> key = plan_key(jobs, njobs, dir);
  std::shared_ptr<hentt_batch_plan> p = cached_plan(key);
  if (!p) {
    hentt_batch_plan *raw = nullptr;
    int rc = plan_build(jobs, njobs, dir, &raw);
    if (rc) return rc;
    p = std::shared_ptr<hentt_batch_plan>(raw, plan_free);
    std::shared_ptr<hentt_batch_plan> gone;  // freed outside the lock
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (g_plans.size() >= kPlanCacheMax) {
      gone = g_plans.begin()->second;
      g_plans.erase(g_plans.begin());
    }
    g_plans[key] = p;
  }
  return hentt_batch_plan_run(p.get(), stream);
}

int hentt_ntt_batch_status(const hentt_job *jobs, uint32_t njobs, int dir) {
  if (!jobs || njobs == 0 || (dir != 1 && dir != -1)) return HENTT_EINVAL;
  for (uint32_t j = 0; j < njobs; ++j)
    if (!jobs[j].t) return HENTT_EINVAL;
  std::shared_ptr<hentt_batch_plan> p = cached_plan(plan_key(jobs, njobs, dir));
  if (!p) return HENTT_EINVAL;
  return plan_status(p.get());
}

namespace {
int tune_count(int op, uint32_t log_n, uint32_t *count) {
  if (op < 0 || op >= kTuneOps || log_n < HENTT_LOG_N_MIN || log_n > HENTT_LOG_N_MAX) return HENTT_EINVAL;
  if (op == HENTT_OP_FWD || op == HENTT_OP_INV) *count = transform_candidates(log_n);
  else (void)prod_candidates(op == HENTT_OP_POLYMUL ? PROD_MUL : PROD_TENSOR, log_n, count);
  return HENTT_OK;
}
}  // namespace

int hentt_tune_count(int op, uint32_t log_n, uint32_t *count) {
  if (!count) return HENTT_EINVAL;
  return tune_count(op, log_n, count);
}

int hentt_tune_describe(int op, uint32_t log_n, uint32_t choice, char *buf, uint32_t len, uint32_t *column_stages) {
  uint32_t n = 0;
  if (!buf || len == 0 || tune_count(op, log_n, &n) || choice >= n) return HENTT_EINVAL;
  const char *d = nullptr;
  uint32_t cols = 0;
  if (op == HENTT_OP_FWD || op == HENTT_OP_INV) {
    d = transform_describe(log_n, choice);
    cols = transform_cols(log_n, choice);
  } else {
    const ProdCand &c = prod_candidates(op == HENTT_OP_POLYMUL ? PROD_MUL : PROD_TENSOR, log_n, &n)[choice];
    d = c.desc;
    cols = c.pec;
  }
  snprintf(buf, len, "%s", d);
  if (column_stages) *column_stages = cols;
  return HENTT_OK;
}

int hentt_tune_class(uint64_t units, uint32_t *cls) {
  if (!cls) return HENTT_EINVAL;
  *cls = tune_class(units);
  return HENTT_OK;
}

int hentt_tune_select(int op, uint32_t log_n, uint32_t cls, uint32_t choice) {
  uint32_t n = 0;
  if (tune_count(op, log_n, &n) || choice >= n || cls >= (uint32_t)kTuneClasses) return HENTT_EINVAL;
  g_choice[op][log_n][cls].store((uint8_t)choice);
  return HENTT_OK;
}

int hentt_tune_get(int op, uint32_t log_n, uint32_t cls, uint32_t *choice) {
  uint32_t n = 0;
  if (!choice || tune_count(op, log_n, &n) || cls >= (uint32_t)kTuneClasses) return HENTT_EINVAL;
  *choice = g_choice[op][log_n][cls].load();
  return HENTT_OK;
}

int hentt_pool_trim(void) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  pool_trim_locked();
  return HENTT_OK;
}

int hentt_pool_bytes(uint64_t *bytes) {
  if (!bytes) return HENTT_EINVAL;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  uint64_t n = 0;
  for (auto &e : g_pool) n += e.bytes;
  *bytes = n;
  return HENTT_OK;
}

int hentt_prof_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto &r : g_prof) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.clear();
  g_prof_agg.clear();
  g_prof_on.store(on != 0);
  return HENTT_OK;
}

int hentt_prof_count(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto &r : g_prof) {
    float ms = 0;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return hip_fail(e);
    bool found = false;
    for (auto &g : g_prof_agg)
      if (g.name == r.name) {
        g.ms += ms;
        g.n += 1;
        found = true;
      }
    if (!found) g_prof_agg.push_back({r.name, (double)ms, 1});
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.clear();
  return (int)g_prof_agg.size();
}

int hentt_prof_get(uint32_t i, char *name, uint32_t name_len, double *total_ms, uint32_t *launches) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (i >= g_prof_agg.size() || !name || name_len == 0) return HENTT_EINVAL;
  snprintf(name, name_len, "%s", g_prof_agg[i].name.c_str());
  if (total_ms) *total_ms = g_prof_agg[i].ms;
  if (launches) *launches = g_prof_agg[i].n;
  return HENTT_OK;
}

}  // extern "C"
