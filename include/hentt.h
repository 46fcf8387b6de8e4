/*
 * hentt -- batched negacyclic NTT over RNS limbs for AMD Instinct MI355X (gfx950).
 *
 * C ABI of libhentt.so.  The operations follow arXiv 2109.14704:
 *   - ring R_q = Z_q[x]/(x^N + 1), N = 2^log_n               (section II-A)
 *   - polynomial product through the psi-twisted NTT:
 *       a * b = INTT(NTT(a) (.) NTT(b))                       (section II-B)
 *   - RNS: each limb (modulus q_l) is an independent sub-task (section II-B)
 *   - ciphertext Mul tensor: (c0 d0, c0 d1 + c1 d0, c1 d1)    (section II-A, Mul)
 *   - lazy Harvey butterflies, Algorithm 1                     (section III-B)
 *   - fused multiply-add with one reduction (mad_mod)          (section III-A-1)
 *
 * Conventions.
 *   - Data are uint64 words, layout [batch][limbs][N] (coefficient fastest);
 *     ciphertexts are [batch][2][limbs][N], tensor outputs [batch][3][limbs][N].
 *   - psi is the smallest primitive 2N-th root of unity mod q_l.
 *   - NTT domain = bit-reversed order: NTT(a)[k] = sum_i a_i psi^(i (2 brv(k) + 1)).
 *   - INTT includes N^-1 and the psi^-i untwist, so INTT(NTT(a)) == a exactly.
 *   - Inputs must be canonical residues in [0, q_l); every output is canonical.
 *   - Moduli: prime, q = 1 (mod 2N), 2^7 < q < 2^60 (16 q < 2^64 is what the
 *     lazy butterflies need).
 *
 * Memory and streams.  Every data pointer is a DEVICE pointer owned by the
 * caller, who keeps it alive until the work queued on `stream` completes.
 * `stream` is a hipStream_t passed as void* (NULL = default stream).  Compute
 * calls only enqueue work: they never synchronise the host.  Tables are
 * owned by the library, immutable after creation, and may be shared across
 * streams and threads.
 *
 * Errors.  Every call returns HENTT_OK (0) or a negative status; nothing is
 * thrown across the ABI.  On HENTT_EHIP the HIP error code is available from
 * hentt_last_hip_error() (thread-local).
 */
#ifndef HENTT_H
#define HENTT_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HENTT_OK 0
#define HENTT_EINVAL (-1)    /* null pointer, zero batch/limbs, log_n out of range, bad flags */
#define HENTT_EMODULUS (-2)  /* modulus not prime, not 1 mod 2N, or out of (2^7, 2^60) */
#define HENTT_ENOMEM (-3)    /* host or device allocation failed */
#define HENTT_EHIP (-4)      /* a HIP runtime call failed; see hentt_last_hip_error() */
#define HENTT_ETIMEOUT (-5)  /* a persistent batch tile gave up waiting (reported by hentt_batch_plan_status) */
#define HENTT_EBUSY (-6)     /* a batch plan still has live graphs (hentt_batch_plan_set_grid / _destroy) */
#define HENTT_ENONCANON (-7) /* hentt_check_canonical found input words outside [0, q) */
#define HENTT_ESCRATCH (-8)  /* hentt_ct_tensor_noalloc: workspace beyond HENTT_NOALLOC_SCRATCH_WORDS */

#define HENTT_LOG_N_MIN 6
#define HENTT_LOG_N_MAX 17
#define HENTT_LIMBS_MAX 64

/* ct_tensor flags: domain of the inputs and of the output. */
#define HENTT_IN_COEFF 0u   /* c, d in the coefficient domain (forward transforms applied) */
#define HENTT_IN_NTT 1u     /* c, d already in the NTT domain */
#define HENTT_OUT_COEFF 0u  /* out in the coefficient domain (inverse transforms applied) */
#define HENTT_OUT_NTT 2u    /* out left in the NTT domain */

typedef struct hentt_tables hentt_tables;

/* Twiddle tables for one modulus chain at one N (section II-B; Algorithm 1's
 * root powers W and root power quotients W' = floor(W 2^64 / q)).
 * log_n in [HENTT_LOG_N_MIN, HENTT_LOG_N_MAX]; moduli_host: `limbs` host
 * words.  Builds on the host, uploads on `stream`, and waits for the upload.
 * Device footprint: 32 N bytes per limb plus 64 bytes per limb.
 * *out receives a handle the caller releases with hentt_tables_destroy. */
int hentt_tables_create(uint32_t log_n, uint32_t limbs, const uint64_t *moduli_host, void *stream,
                        hentt_tables **out);

/* Releases a handle (a table or a view).  Device memory is freed when the last
 * handle sharing it is released.  The caller makes sure no queued work still
 * reads the tables (e.g. synchronises the stream first). */
int hentt_tables_destroy(hentt_tables *t);

/* A handle on the first `limbs` moduli of `t` (a lower level of the chain),
 * sharing t's device memory.  Released with hentt_tables_destroy. */
int hentt_tables_view(const hentt_tables *t, uint32_t limbs, hentt_tables **view);

/* log_n and limb count of a handle. */
int hentt_tables_info(const hentt_tables *t, uint32_t *log_n, uint32_t *limbs);

/* Device pointers of the raw tables, read-only.  The twiddles form one
 * [limbs][2][N] array of (W, W') uint64 pairs, W' = floor(W 2^64 / q): fwd
 * points at limb 0's forward table (W = psi^brv(k)) and inv at limb 0's
 * inverse table (W = psi^-brv(k)); limb l's tables start 4 N l words later.
 * moduli points at [limbs] records of 12 uint64 words whose first word is q
 * (the rest are the library's reduction constants). */
int hentt_tables_device_ptrs(const hentt_tables *t, const uint64_t **fwd, const uint64_t **inv,
                             const uint64_t **moduli);

/* The library's psi for (q, N): smallest primitive 2N-th root of unity mod q.
 * Host-only helper, no device work. */
int hentt_psi(uint64_t q, uint32_t log_n, uint64_t *psi);

/* Debug check of the input precondition that every compute call assumes and
 * none checks: the words of x[batch][limbs][N] are canonical residues,
 * x[b][l][i] < q_l (the input range of Algorithm 1, whose last round brings
 * outputs back into [0, q); section III-B).  Enqueues a check kernel on
 * `stream` and then WAITS for the stream (debug use, not for the hot path).
 * Returns HENTT_OK when every word is canonical, HENTT_ENONCANON otherwise;
 * bad_words (optional) receives the number of non-canonical words and
 * first_bad (optional) the smallest flat word index of one (~0 if none).
 * HENTT_EINVAL for null x or t, batch 0, or more than 2^31 - 1 tiles of 2048
 * words. */
int hentt_check_canonical(const hentt_tables *t, const uint64_t *x, uint32_t batch, uint64_t *bad_words,
                          uint64_t *first_bad, void *stream);

/* Forward negacyclic NTT in place: x[batch][limbs][N], natural order ->
 * bit-reversed NTT domain (section II-B). */
int hentt_ntt_fwd(const hentt_tables *t, uint64_t *x, uint32_t batch, void *stream);

/* Rescale RS of section II-A: divide by the last prime qL of the level with
 * rounding and drop that limb, c' = round(c / qL) mod q_i (c the CRT value of
 * each coefficient).  t's limb count is the level (at least 2); c is
 * [batch][limbs][N], out [batch][limbs - 1][N]; out must not overlap c
 * (HENTT_EINVAL).  flags: 0 for coefficient-domain input and output;
 * HENTT_IN_NTT | HENTT_OUT_NTT for NTT-domain (bit-reversed) input and output,
 * where the last limb is inverse-transformed once and its correction
 * forward-transformed per remaining limb, with the reduction, subtraction and
 * scaling fused into that transform; other flags: HENTT_EINVAL.  Canonical
 * inputs, canonical outputs.  The per-level constants are made on the first
 * call for a level (a synchronous upload); later calls only enqueue. */
int hentt_rescale(const hentt_tables *t, const uint64_t *c, uint64_t *out, uint32_t batch, uint32_t flags,
                  void *stream);

/* Encrypted element-wise polynomial matrix product of section IV-E, NTT
 * domain: C (m x n) += A (m x k) * B (k x n) where every matrix element is a
 * ciphertext and every element product the Mul tensor of section II-A
 * (c0 d0, c0 d1 + c1 d0, c1 d1), accumulated over k with one modular
 * reduction per output term of every element product (the middle term's two
 * products summed first: mad_mod, section III-A-1).
 * A [m][k][2][limbs][N], B [k][n][2][limbs][N], C [m][n][3][limbs][N] with
 * limbs and N those of t; canonical inputs, canonical C.  C is updated in
 * place and must not overlap A or B.  HENTT_EINVAL for null pointers, a zero
 * dimension, overlap, or more than 2^31 - 1 workgroups (m n limbs N / 2048). */
int hentt_ct_matmul(const hentt_tables *t, const uint64_t *A, const uint64_t *B, uint64_t *C, uint32_t m, uint32_t n,
                    uint32_t k, void *stream);

/* Relinearization Relin of section II-A with the RNS digit key switch:
 * c' = (c0, c1) + round(P^-1 sum_j [c2]_{q_j} evk_j) mod q, NTT domain in and
 * out.  t holds l + 1 limbs: the ciphertext's primes q_0 .. q_{l-1} followed
 * by the special prime P (l >= 1).  c [batch][3][l][N] (the Mul tensor),
 * ksk [l][2][l + 1][N] (digit j, component s, prime: the key-switching key,
 * caller-owned), out [batch][2][l][N]; canonical inputs and outputs.  out must
 * not overlap c or ksk (HENTT_EINVAL).  The level's rescale and key-switching
 * constants are made on its first call (a synchronous upload); later calls
 * only enqueue. */
int hentt_relin(const hentt_tables *t, const uint64_t *c, const uint64_t *ksk, uint64_t *out, uint32_t batch,
                void *stream);

/* Kernel-design ladder of the forward transform (section III-B and the
 * NTT evaluation of section IV): the same result as hentt_ntt_fwd, computed
 * by reference kernel designs so that they can be timed against each other.
 * Not for production use.
 *   HENTT_VARIANT_LIBRARY    the library's kernels (hentt_ntt_fwd);
 *   HENTT_VARIANT_NAIVE      naive radix-2: one global-memory launch per
 *                            stage, one butterfly per lane, then a separate
 *                            reduction to [0, q); any supported log_n;
 *   HENTT_VARIANT_STAGED_R2  four naive global stages, then LDS blocks of
 *                            2048 coefficients with radix-2 rounds (one stage
 *                            per LDS exchange); log_n = 15 only;
 *   HENTT_VARIANT_SIMD1, _SIMD2, _SIMD4
 *                            staged radix-2 with the smallest gaps exchanged
 *                            between the lanes of a wavefront (the SIMD
 *                            shuffling of section III-B): four naive global
 *                            stages, LDS blocks of 2048 coefficients with one
 *                            radix-2 stage per LDS exchange down to a gap of
 *                            128 S, then the stages with gaps 64 S .. 1 inside
 *                            each wavefront, every lane holding S pairs
 *                            (S = 1, 2, 4: the paper's one-, two- and four-slot
 *                            SIMD variants on 64-wide wavefronts); log_n = 15
 *                            only;
 *   HENTT_VARIANT_STAGED_R4, _R8, _R16
 *                            one radix-8 column pass, then LDS blocks of 4096
 *                            coefficients with radix-4, -8 or -16 rounds;
 *                            log_n = 15 only (HENTT_EINVAL otherwise).
 * Arguments, layout and errors as hentt_ntt_fwd; HENTT_EINVAL for an unknown
 * variant. */
#define HENTT_VARIANT_LIBRARY 0
#define HENTT_VARIANT_NAIVE 1
#define HENTT_VARIANT_STAGED_R4 2
#define HENTT_VARIANT_STAGED_R8 3
#define HENTT_VARIANT_STAGED_R16 4
#define HENTT_VARIANT_STAGED_R2 5
#define HENTT_VARIANT_SIMD1 6
#define HENTT_VARIANT_SIMD2 7
#define HENTT_VARIANT_SIMD4 8
int hentt_ntt_fwd_variant(const hentt_tables *t, uint64_t *x, uint32_t batch, int variant, void *stream);

/* Inverse negacyclic NTT in place: bit-reversed NTT domain -> natural order,
 * including N^-1 and the psi^-i untwist (section II-B). */
int hentt_ntt_inv(const hentt_tables *t, uint64_t *x, uint32_t batch, void *stream);

/* Element-wise (dyadic) product out = a (.) b mod q_l over [batch][limbs][N]
 * (section II-B).  out may alias a or b exactly; a partial overlap returns
 * HENTT_EINVAL. */
int hentt_dyadic_mul(const hentt_tables *t, const uint64_t *a, const uint64_t *b, uint64_t *out,
                     uint32_t batch, void *stream);

/* Negacyclic products out = INTT(NTT(a) (.) NTT(b)) of coefficient-domain
 * a, b over [batch][limbs][N] (section II-B), fused so that the NTT-domain
 * values never leave the chip.  out must not overlap a or b (HENTT_EINVAL).
 * For N > 2^12 the forward column pass writes a workspace of 2 batch limbs N
 * words taken from the library's pool (allocated on first need, reused). */
int hentt_polymul(const hentt_tables *t, const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t batch,
                  void *stream);

/* Ciphertext tensor product (section II-A, Mul): c, d [batch][2][limbs][N],
 * out [batch][3][limbs][N] = (c0 d0, c0 d1 + c1 d0, c1 d1) per limb, the middle
 * term reduced once (mad_mod).  flags: HENTT_IN_COEFF | HENTT_IN_NTT combined
 * with HENTT_OUT_COEFF | HENTT_OUT_NTT.  c and d are not modified; out must
 * not overlap them (HENTT_EINVAL).  With coefficient-domain inputs and
 * N > 2^12 the forward column pass writes a workspace of 4 batch limbs N
 * words from the library's pool. */
int hentt_ct_tensor(const hentt_tables *t, const uint64_t *c, const uint64_t *d, uint64_t *out, uint32_t batch,
                    uint32_t flags, void *stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * product as hentt_ct_tensor, with the same arguments, layout, flags and
 * results, that allocates nothing.  The forward column pass of a two-pass
 * product (coefficient-domain inputs, N > 2^12) writes its workspace of
 * 4 batch limbs N words into a static device array of
 * HENTT_NOALLOC_SCRATCH_WORDS words (64 MiB) that every GPU the library runs
 * on holds until the process ends; a call needing more returns
 * HENTT_ESCRATCH before enqueuing anything (e.g. one ciphertext pair of
 * N = 2^16 at 32 limbs fits, two do not).  Every call on one GPU shares that
 * array: calls that overlap in time on one GPU (different streams, or
 * threads) race and must be serialised by the caller.  Kernel timing
 * (hentt_prof_enable) does not cover this call.  No hipMalloc, hipFree or
 * other allocating routine is called; the array's device address is looked
 * up once per device on the first call. */
#define HENTT_NOALLOC_SCRATCH_WORDS (8ull << 20)
int hentt_ct_tensor_noalloc(const hentt_tables *t, const uint64_t *c, const uint64_t *d, uint64_t *out,
                            uint32_t batch, uint32_t flags, void *stream);

/* One ciphertext tensor product of a grouped call: c, d [batch][2][limbs][N]
 * -> out [batch][3][limbs][N] with the moduli of t (a table or a level
 * view: limbs = its limb count, N = its ring dimension).  reserved: 0. */
typedef struct {
  const uint64_t *c;
  const uint64_t *d;
  uint64_t *out;
  const hentt_tables *t;
  uint32_t batch;
  uint32_t reserved;
} hentt_ct_job;

/* Many ciphertext tensor products (section II-A, Mul) of mixed levels and
 * ring dimensions in a few launches: the products of every job of one N run
 * in one launch per kernel of the product (forward column pass, fused block
 * kernel, inverse column pass), jobs of larger N first, at most 24 jobs per
 * launch sequence (more jobs: further sequences).  This is continuous
 * batching's device side: a step of many small requests fills the GPU
 * without gathering their operands into one buffer.  Each job's result
 * equals hentt_ct_tensor on the same job; flags as there and common to all
 * jobs.  jobs is a HOST array read before the call returns; the data are
 * DEVICE pointers owned by the caller.  HENTT_EINVAL: jobs NULL with
 * njobs > 0, a NULL pointer, batch 0, reserved != 0, batch x limbs >= 2^24,
 * or an output range that overlaps another job's output or any job's input.
 * njobs = 0 enqueues nothing.  With coefficient-domain inputs and N > 2^12
 * the forward column pass writes a workspace of 4 batch limbs N words per
 * job (one buffer of the largest launch sequence's total, from the pool).
 * The stage split at each N is the single-job product's default one. */
int hentt_ct_tensor_grouped(const hentt_ct_job *jobs, uint32_t njobs, uint32_t flags, void *stream);

/* One polynomial set of an uneven batch: data [batch][limbs][N] in place,
 * transformed with the first `limbs` moduli of `t` (limbs <= t's limbs). */
typedef struct {
  uint64_t *data;
  const hentt_tables *t;
  uint32_t limbs;
  uint32_t batch;
} hentt_job;

/* Transforms every job (dir = +1 forward, -1 inverse), each job at its own N
 * and limb count, in a single persistent kernel launch (section III-B: the
 * batch and RNS limbs give independent transforms).  jobs is a HOST array; it
 * is read before the call returns.  The first call with a given job list
 * builds a plan (tile list on the device, synchronous) and caches it (up to
 * 16 plans, keyed by the data pointers, the table storages, N, limb counts,
 * batch sizes and direction); later calls only enqueue.  A cached plan holds
 * a reference on every table storage it uses; hentt_tables_destroy evicts
 * the plans of the destroyed table's storage.  Jobs with N < 2^12 run as
 * ordinary launches in the same call. */
int hentt_ntt_batch(const hentt_job *jobs, uint32_t njobs, int dir, void *stream);

/* Status of the last hentt_ntt_batch call with this job list and direction:
 * waits for it, then HENTT_ETIMEOUT if one of its pass-2 tiles gave up
 * waiting (bounded spin) or a queue went unserved, else HENTT_OK.
 * HENTT_EINVAL if no cached plan matches. */
int hentt_ntt_batch_status(const hentt_job *jobs, uint32_t njobs, int dir);

/* Explicit plans for the same persistent launch (for autotuning and graphs).
 * create: validates the jobs and uploads the tile list (synchronous).
 * set_grid: number of persistent workgroups (0 = as many as the device
 *   holds at once: the kernel's occupancy per compute unit, 4 on gfx950,
 *   times the compute units);
 *   HENTT_EBUSY while graphs captured from the plan exist (they hold the
 *   old launch shape).
 * run: enqueues a counter reset kernel and the persistent kernel on stream.
 * status: waits for the last run or graph replay; HENTT_ETIMEOUT if a pass-2
 *   tile gave up waiting for its pass-1 tiles (bounded spin) or a queue went
 *   unserved, else HENTT_OK.
 * destroy: HENTT_EBUSY while graphs captured from the plan exist.
 * The plan holds a reference on every table storage it uses.  The job data
 * stay owned by the caller and must outlive every run. */
typedef struct hentt_batch_plan hentt_batch_plan;
int hentt_batch_plan_create(const hentt_job *jobs, uint32_t njobs, int dir, hentt_batch_plan **out);
int hentt_batch_plan_set_grid(hentt_batch_plan *p, uint32_t workgroups);
/* set_schedule: the tile order of each queue (tuning constants of the
 * staged transform's schedule, section III-B).  Units sharing a twiddle
 * table are taken in groups of at most group_units (default 8; 1 to 4096)
 * whose block tiles run block-major across the group, so that tiles reading
 * the same twiddles run together; a group's pass-2 tiles are queued at least
 * lookahead_pct % of the queue's workgroup count (default 200; at most
 * 10000) after its last pass-1 tile: smaller values keep pass-1 results
 * likelier in L2, larger values make dependency waits rarer.  HENTT_EBUSY
 * while graphs exist; HENTT_EINVAL out of range. */
int hentt_batch_plan_set_schedule(hentt_batch_plan *p, uint32_t lookahead_pct, uint32_t group_units);
int hentt_batch_plan_info(const hentt_batch_plan *p, uint32_t *units, uint32_t *tiles, uint32_t *grid);
int hentt_batch_plan_run(hentt_batch_plan *p, void *stream);
int hentt_batch_plan_status(hentt_batch_plan *p);
int hentt_batch_plan_destroy(hentt_batch_plan *p);

/* A plan's launch sequence captured once into a hipGraph (on a private
 * stream; the counter reset is a kernel, not a memset node) and replayed with
 * hentt_graph_launch on any stream; each replay records the plan's
 * completion event, so hentt_batch_plan_status reports on the last replay.
 * Destroy the graphs before the plan. */
typedef struct hentt_graph hentt_graph;
int hentt_batch_graph_create(hentt_batch_plan *p, hentt_graph **out);
int hentt_graph_launch(hentt_graph *g, void *stream);
int hentt_graph_destroy(hentt_graph *g);

/* Workspace pool (the memory cache of section III-C-1): device buffers for
 * the column passes of two-pass products, rescale and relinearization are
 * kept after use and reused by later calls on the same device and stream.
 * hentt_pool_bytes reports the bytes the pool holds; hentt_pool_trim waits
 * for the streams of the idle buffers and frees them (buffers of calls still
 * being enqueued by other threads are kept).  Environment: with
 * HENTT_POOL_MAX_BYTES=<bytes> (read once), a call that would grow the pool
 * past that many bytes first trims the idle buffers (a soft cap: a single
 * buffer larger than the cap is still allocated). */
int hentt_pool_bytes(uint64_t *bytes);
int hentt_pool_trim(void);

/* Kernel timing for benchmarks.  While enabled, every kernel the library
 * launches is bracketed by HIP events recorded on the launching stream.
 * hentt_prof_count() waits for the recorded events, folds them into per-kernel
 * totals and returns the number of distinct kernels (or a negative status);
 * hentt_prof_get() copies entry i: kernel name (with log_n), total milliseconds
 * and launch count.  hentt_prof_enable() clears all records. */
int hentt_prof_enable(int on);
int hentt_prof_count(void);
int hentt_prof_get(uint32_t i, char *name, uint32_t name_len, double *total_ms, uint32_t *launches);

/* Stage split of the default instances at N = 2^log_n: how many butterfly
 * stages the column pass of a plain transform (transform_cols) and of the
 * fused dyadic product (product_cols) performs; 0 means the transform runs
 * whole in one workgroup.  Tuned instances (hentt_tune_*) and the tensor
 * product may split differently.  Host-only, no device work. */
int hentt_stage_split(uint32_t log_n, uint32_t *transform_cols, uint32_t *product_cols);

/* Autotuning (the tuning constants of section III-B, chosen by measurement):
 * every operation has, per N, a list of compiled kernel instances -- the
 * stage split between the column pass and the block pass, and the words
 * held per lane (the radix of the register rounds) -- of which instance 0 is
 * the default.  A selection applies per (operation, N, shape class) to every
 * later call of the library in this process (all threads); the shape class
 * of a call groups its number of (batch entry, limb) units, batch * limbs:
 * class 0 below 64, class 1 below 1024, class 2 above.  Every instance gives
 * the same results (bit-exact); only its speed differs.  Products select
 * among their instances only in the fused coefficient-to-coefficient form
 * (the other forms run instance 0).  Host-only, no device work:
 *   count: number of instances of op at N = 2^log_n;
 *   describe: text of instance `choice` (copied into buf) and, if
 *     column_stages is not null, the stages of its column pass (0: the whole
 *     operation runs in one kernel per (batch entry, limb));
 *   class: the shape class of `units` units;
 *   select / get: the instance used for (op, N, class).
 * HENTT_EINVAL for an unknown op, log_n out of range, or choice >= count. */
#define HENTT_OP_FWD 0
#define HENTT_OP_INV 1
#define HENTT_OP_POLYMUL 2
#define HENTT_OP_TENSOR 3
int hentt_tune_count(int op, uint32_t log_n, uint32_t *count);
int hentt_tune_describe(int op, uint32_t log_n, uint32_t choice, char *buf, uint32_t len, uint32_t *column_stages);
int hentt_tune_class(uint64_t units, uint32_t *cls);
int hentt_tune_select(int op, uint32_t log_n, uint32_t cls, uint32_t choice);
int hentt_tune_get(int op, uint32_t log_n, uint32_t cls, uint32_t *choice);

/* Text for a status code (static storage). */
const char *hentt_status_str(int status);

/* HIP error code behind the last HENTT_EHIP returned on this thread. */
int hentt_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HENTT_H */
