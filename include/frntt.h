/*
 * frntt -- number-theoretic transforms over the BN254 scalar field Fr on
 * AMD MI355X (gfx950). C ABI of libfrntt.so.
 *
 * The operation (paper: Background, "Number Theory Transformation"): for a
 * vector x of N = 2^log_n field elements,
 *     X_k = sum_{n<N} x_n * w^(k*n)  mod r,     k in [0, N),
 * with r the 254-bit BN254 scalar-field prime and w = 5^((r-1)/N) a
 * primitive N-th root of unity (5 generates Fr^*). The inverse transform
 * uses w^-1 and scales by N^-1; the coset transform evaluates at g*w^k with
 * g = 5, i.e. it transforms x_n * g^n; the coset inverse undoes it.
 * Batching follows the paper's batch-size study (Ablation Study - Batch
 * Size): `batch` independent polynomials in one call.
 *
 * Data layout (all entry points): an element is 32 bytes, four 64-bit
 * little-endian limbs of a canonical integer in [0, r). A polynomial is
 * 2^log_n consecutive elements in natural order; `batch` polynomials are
 * consecutive. Transforms are in place, input and output in natural order.
 *
 * Memory ownership: the caller allocates and owns every data buffer (device
 * memory, e.g. hipMalloc or a torch tensor) and keeps it alive until the
 * stream has passed the call. The context owns its twiddle and limb tables
 * and its scratch space.
 *
 * Asynchrony: every transform call is enqueued on `stream` (a hipStream_t;
 * NULL means the null stream) and returns at once, with two exceptions that
 * happen at most once per context: the first transform of a (size, kind,
 * plan) builds that plan's pass-twiddle table (allocation plus a synchronous
 * device fill; frntt_prepare does it ahead of time), and the first transform
 * on a stream that needs more scratch than the stream has allocates it.
 * Inside a hipGraph stream capture neither may happen: such a call returns
 * FRNTT_ESTATE and enqueues nothing (call frntt_prepare and one transform of
 * that size on the stream before capturing). Argument errors are returned
 * synchronously before anything is enqueued. A failed HIP launch returns
 * FRNTT_EHIP and frntt_last_hip_error() gives the hipError_t.
 *
 * Preconditions: inputs must be canonical (< r). With the FRNTT_VALIDATE
 * context flag a device check runs before each transform; a violation is
 * reported by frntt_check_inputs(). Otherwise the output for inputs >= r is
 * unspecified (but the call never reads or writes out of bounds).
 *
 * Threads and streams: a context may be used from several host threads and
 * streams at once. Calls on different streams get separate scratch space.
 */
#ifndef FRNTT_H
#define FRNTT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct frntt_ctx frntt_ctx;
typedef struct frntt_server frntt_server;
typedef struct frntt_rns_field frntt_rns_field;

/* Status codes returned by every call. */
enum {
    FRNTT_OK = 0,
    FRNTT_EINVAL = -1, /* null pointer, bad kind/algorithm/flag, batch < 0     */
    FRNTT_ERANGE = -2, /* log_n outside [0, max_log_n] or above 28            */
    FRNTT_EALIGN = -3, /* data pointer not 32-byte aligned                    */
    FRNTT_ENOMEM = -4, /* device or host allocation failed                    */
    FRNTT_EHIP = -5,   /* a HIP runtime call failed (see frntt_last_hip_error) */
    FRNTT_EBUSY = -6,  /* server: over its memory budget or queue limit       */
    FRNTT_ESTATE = -7  /* object in the wrong state (e.g. unknown ticket)     */
};

/* Transform kinds. */
enum { FRNTT_FWD = 0, FRNTT_INV = 1, FRNTT_COSET = 2, FRNTT_COSET_INV = 3 };

/* Algorithms.
 * BUTTERFLY: radix-2/4 Cooley-Tukey stages with Montgomery twiddle products
 *   on the vector ALUs (the paper's butterfly NTT; Dataflow Optimizations).
 * FOURSTEP_MFMA: the matrix form (the paper's 3-step NTT and its recursive
 *   5-step refinement, Eq. 1): sub-DFTs as byte-limb x twiddle products on
 *   int8 matrix cores with 32-bit accumulators, then carry merge and
 *   reduction mod r (Alg. 1's ByteDecompose / einsum / ByteMerge pattern).
 * AUTO: the context's tuned choice per size (MFMA unless tuned otherwise). */
enum { FRNTT_ALGO_AUTO = 0, FRNTT_ALGO_BUTTERFLY = 1, FRNTT_ALGO_FOURSTEP_MFMA = 2 };

/* Context flags. */
enum {
    FRNTT_VALIDATE = 1u << 0,       /* check inputs < r on the device before transforming */
    FRNTT_SPLIT_TWIDDLES = 1u << 1  /* keep no N-entry pass-twiddle tables: every pass twiddle
                                     * (and coset factor) is formed from the two 2^14-entry
                                     * split tables with one more product. For contexts that
                                     * must keep their table memory small (a few MiB); slower. */
};

/* Create a context on HIP device `hip_device` for sizes up to 2^max_log_n
 * (1 <= max_log_n <= 28). Builds all twiddle and limb tables on the device.
 * *out is set only on success. Errors: EINVAL, ERANGE, ENOMEM, EHIP. */
int frntt_ctx_create(frntt_ctx **out, int hip_device, int max_log_n, unsigned flags);

/* Destroy a context (waits for the device). NULL is accepted. */
int frntt_ctx_destroy(frntt_ctx *ctx);

/* In-place transforms of `batch` consecutive polynomials of 2^log_n
 * elements at device pointer `data`. batch == 0 is a no-op; log_n == 0 is
 * the identity. Errors: EINVAL (ctx or data NULL, batch < 0), ERANGE,
 * EALIGN, ENOMEM (scratch), EHIP. */
int ntt_fwd(frntt_ctx *ctx, void *data, int log_n, int batch, void *stream);
int ntt_inv(frntt_ctx *ctx, void *data, int log_n, int batch, void *stream);
int ntt_coset(frntt_ctx *ctx, void *data, int log_n, int batch, void *stream);     /* g = 5 */
int ntt_coset_inv(frntt_ctx *ctx, void *data, int log_n, int batch, void *stream);
/* Same, with the kind as an argument (FRNTT_FWD .. FRNTT_COSET_INV). */
int ntt_transform(frntt_ctx *ctx, void *data, int log_n, int batch, int kind, void *stream);

/* As ntt_transform, with an explicit algorithm that overrides the context's
 * choice for this call only. */
int ntt_transform_algo(frntt_ctx *ctx, void *data, int log_n, int batch, int kind, int algo,
                       void *stream);

/* For callers that cannot allocate: code under hipGraph stream capture,
 * tight serving loops, harnesses that forbid hipMalloc. Same result as
 * ntt_transform (bit-identical), but nothing is allocated, built or waited
 * for on any call: the passes ping-pong through a static device array of
 * FRNTT_NOALLOC_MAX_ELEMS elements (32 MiB) that the library holds on each GPU
 * until the process ends, and every pass twiddle comes from the split tables
 * built at context creation (no N-entry tables; slower than ntt_transform).
 * batch << log_n must not exceed FRNTT_NOALLOC_MAX_ELEMS (ERANGE otherwise).
 * All calls on one GPU share that array: calls that overlap on one GPU (other
 * streams, other contexts, other threads) race and must be serialised by the
 * caller. Errors otherwise as ntt_transform. */
#define FRNTT_NOALLOC_MAX_ELEMS (1u << 20)
int ntt_transform_noalloc(frntt_ctx *ctx, void *data, int log_n, int batch, int kind, void *stream);

/* Choose the algorithm used by later calls (FRNTT_ALGO_*). */
int frntt_set_algo(frntt_ctx *ctx, int algo);
int frntt_get_algo(const frntt_ctx *ctx);

/* Override the decomposition of 2^log_n into HBM passes for one algorithm:
 * pass_logs[0..n_passes-1] are the log2 radices of the passes, in order,
 * each in [1, 12], summing to log_n. n_passes == 0 restores the default.
 * Any valid plan gives bit-identical results. Errors: EINVAL, ERANGE. */
int frntt_set_plan(frntt_ctx *ctx, int algo, int log_n, const int *pass_logs, int n_passes);
/* The plan in use; writes up to `cap` entries, returns the pass count (>= 0)
 * or an error. */
int frntt_get_plan(const frntt_ctx *ctx, int algo, int log_n, int *pass_logs, int cap);

/* The level split the matrix form uses inside HBM pass `pass` of a single
 * transform of 2^log_n elements with the plan in use (default, override or
 * tuned): writes up to `cap` log2 radices and returns how many levels there
 * are, or 0 if that pass runs on the butterfly engine (the algorithm is the
 * butterfly form, or the pass's tile is below 4096 elements). Errors: EINVAL,
 * ERANGE. */
int frntt_get_plan_levels(const frntt_ctx *ctx, int algo, int log_n, int pass, int *levels, int cap);

/* One job of an uneven batch: a polynomial of 2^log_n elements at `data`. */
typedef struct {
    void *data;
    int log_n;
    int kind;
} frntt_job;

/* Uneven batch (paper: Ablation Study - Batch Size): transform every job in
 * place with persistent kernel launches, one per pass stage (the first passes
 * of all jobs, then the second passes, ...). The descriptors are copied before
 * the call returns; the data buffers must stay alive until the stream passes
 * the call. Jobs must not overlap in memory. Errors as for ntt_transform,
 * per job, plus EINVAL for n_jobs < 0 or jobs == NULL with n_jobs > 0, and
 * ESTATE inside a stream capture (the descriptor upload waits on the host;
 * ntt_batch_graph is the capturable form). */
int ntt_batch(frntt_ctx *ctx, const frntt_job *jobs, int n_jobs, void *stream);

/* Graph form of ntt_batch for repeated identical batches: the first call for
 * a given job list captures the launches into a hipGraph; later calls with the
 * same list, whose jobs still resolve to the same form and plan (see
 * frntt_set_algo, frntt_set_plan, frntt_tune), replay it. Results are
 * identical to ntt_batch. */
int ntt_batch_graph(frntt_ctx *ctx, const frntt_job *jobs, int n_jobs, void *stream);

/* Autotuner: time forward transforms of one size and batch on `stream` for
 * every candidate plan: algorithm x split into HBM passes (one pass up to
 * 2^12, two passes of at least 2^4 each, three balanced passes from 2^15) x,
 * for the matrix form, the order of the level radices inside its 2^10 and
 * 2^11 passes ([4,3,3], [3,4,3], [3,3,4]; [4,4,3], [3,4,4], [4,3,4]). The
 * median of five runs decides. Keeps the fastest in the context (used by
 * transforms and batches of that size, every kind) and returns it through the
 * out-parameters (any may be NULL). Pass-twiddle tables that only losing
 * candidates built are freed again (after waiting for the device): do not
 * tune a size while other threads transform that size. Synchronous. */
int frntt_tune(frntt_ctx *ctx, int log_n, int batch, int *best_algo, int *best_passes,
               float *best_ms, void *stream);
/* Save / load the tuned choices as a small JSON file. */
int frntt_tune_save(const frntt_ctx *ctx, const char *path);
int frntt_tune_load(frntt_ctx *ctx, const char *path);

/* Fill `count` elements at `data` on the device with the seeded uniform
 * elements of [0, r) that the project's input generator defines (SplitMix64
 * counter stream `stream_id`, starting at element `start`). */
int frntt_generate(frntt_ctx *ctx, void *data, uint64_t seed, uint64_t stream_id, uint64_t start,
                   uint64_t count, void *stream);

/* With FRNTT_VALIDATE: waits for the device and returns EINVAL if any input
 * seen since the last check was >= r, else OK. Without the flag: OK. */
int frntt_check_inputs(frntt_ctx *ctx);

/* Scratch bytes a transform of this size needs (informational). */
size_t frntt_scratch_bytes(int log_n, int batch);

/* Build now the tables a transform of 2^log_n elements of this kind will use
 * (the twiddle table of every pass but the last, w^(rest*k) of the pass's
 * sub-problem: the pass twiddles of the 3-step / 5-step decomposition, Eq. 1,
 * which the paper generates offline), so that later calls allocate nothing
 * for them. Otherwise they are built on first use. The first pass of an
 * inverse kind reads a table whose entries also carry N^-1 (its last pass then
 * skips that product); that of a forward coset kind carries the per-line part
 * g^rest of the coset factor and ends with 2^l entries of its per-element part
 * for the pre-scale; that of a two-pass COSET_INV carries N^-1 g^-k and ends
 * with the factors of the last pass's epilogue. So each kind of one size has
 * its own table. Synchronous. Errors: EINVAL, ERANGE, ENOMEM, EHIP. */
int frntt_prepare(frntt_ctx *ctx, int log_n, int kind);

/* Device bytes held by the context's tables, including the pass-twiddle
 * tables built so far. */
size_t frntt_table_bytes(const frntt_ctx *ctx);

/* ---- RNS lazy modular product (paper: Arithmetic Optimizations, the
 * walk-through example and Alg. 1, "MXU RNS Lazy") ----
 * A field element x in [0, r) is carried in the extended non-prime ring Z_Q,
 * Q = q_0 ... q_16 > 2 r^2, as its residues x z mod q_i (z = 2^32,
 * "Montgomery form" of each residue). The product of two such elements is a
 * residue-wise 32-bit Montgomery product followed by Alg. 1's Main (one int8
 * matrix product of the residues' bytes with the BAT constant table, fused
 * with the overflow-count rows f; then per output residue the byte merge,
 * + k g_j and the reduction mod p_j), which leaves the lazily reduced product
 * W' (W' = a b mod r, |W'| < 2^15 r) in a second base P = p_0 ... p_8 as the
 * residues W' z mod p_j. The moduli are the 26 consecutive primes below
 * 2^31 - 2^24, the largest 17 forming Q, the next 9 forming P. Tables are
 * built at context creation.
 *
 * Layouts (device memory, 16-byte aligned, element-major):
 *   canonical: 8 little-endian 32-bit words per element (< r);
 *   base Q:    FRNTT_RNS_Q_WORDS words per element: residues 0..16, then zeros;
 *   base P:    FRNTT_RNS_P_WORDS words per element: residues 0..8, then zeros.
 * Every call is enqueued on `stream` and returns at once; n = 0 is a no-op.
 * Errors: EINVAL (null context or pointer, n < 0), EALIGN, EHIP. Inputs
 * outside the documented ranges give unspecified outputs. */
#define FRNTT_RNS_Q_WORDS 20
#define FRNTT_RNS_P_WORDS 12
/* The moduli q_0..q_16 and p_0..p_8 (host only; needs no device). */
int frntt_rns_moduli(uint32_t *q, uint32_t *p);
/* Canonical values -> base-Q residues x z mod q_i (the RNS decomposition,
 * itself one byte matrix product with the bytes of z 2^(8b) mod q_i). */
int frntt_rns_encode(frntt_ctx *ctx, const void *a, void *xq, int64_t n, void *stream);
/* Base-Q residues of a and b -> base-P residues of the lazily reduced
 * product (residue-wise Montgomery product, then Alg. 1 Main). */
int frntt_rns_mul(frntt_ctx *ctx, const void *xa, const void *xb, void *xp, int64_t n, void *stream);
/* Base-P residues W' z mod p_j (|W'| < P / 2) -> canonical W' mod r (the RNS
 * reconstruction: Alg. 1 Main once more, from base P into the 32 bytes of a
 * 256-bit word, with k rounded to the nearest integer). */
int frntt_rns_decode(frntt_ctx *ctx, const void *xp, void *out, int64_t n, void *stream);
/* The radix Montgomery product on the vector ALUs, the baseline of the
 * paper's arithmetic ablation: out = a b 2^-261 mod r for canonical a, b
 * (nine 29-bit limbs). */
int frntt_mont_mul(frntt_ctx *ctx, const void *a, const void *b, void *out, int64_t n, void *stream);

/* ---- the same product over other prime fields (the paper's 256/377/753-bit
 * precisions; Arithmetic Optimizations and the Ablation Study) ----
 * A field object holds the tables of one odd prime modulus M given as m_words
 * little-endian 32-bit words: 8 words for M below 2^254, 12 for M below
 * 2^377, 24 for M below 2^753 (and M above 2^32). The shape follows the width:
 *   M words | base Q (I residues, words/element) | base P (J, words) | Montgomery limbs
 *      8    |            17, 20                  |      9, 12        |  9
 *     12    |            25, 28                  |     13, 16        | 13
 *     24    |            49, 52                  |     25, 28        | 26
 * with the moduli q_i, p_j the first I + J primes below 2^31 - 2^24 and
 * |W'| < (4 I 255 + 1) M. Canonical elements take m_words words. Creation is
 * synchronous (tables are built on the host and copied); the calls below are
 * enqueued on `stream`; destroy waits for the device. Errors: EINVAL (null
 * pointer, n < 0, m_words not 8/12/24), ERANGE (M even, below 2^32 or too
 * wide for m_words), EALIGN (pointers not 16-byte aligned), ENOMEM, EHIP.
 * With M = r (8 words) the results equal those of the calls above. */
int frntt_rns_field_create(frntt_rns_field **out, frntt_ctx *ctx, const uint32_t *m, int m_words);
int frntt_rns_field_destroy(frntt_rns_field *f);
/* I, J and the words per element of base Q and base P. */
int frntt_rns_field_shape(const frntt_rns_field *f, int *n_q, int *n_p, int *q_words, int *p_words);
int frntt_rns_field_encode(frntt_rns_field *f, const void *a, void *xq, int64_t n, void *stream);
int frntt_rns_field_mul(frntt_rns_field *f, const void *xa, const void *xb, void *xp, int64_t n, void *stream);
int frntt_rns_field_decode(frntt_rns_field *f, const void *xp, void *out, int64_t n, void *stream);
/* out = a b 2^(-29 L) mod M (L = 9, 13, 26 limbs for 8, 12, 24 words). */
int frntt_rns_field_mont_mul(frntt_rns_field *f, const void *a, const void *b, void *out, int64_t n, void *stream);

/* ---- multi-scalar multiplication (Background, "Multi-Scalar
 * Multiplication"; Alg. 2, Layout Stationary Pippenger) ----
 * MSM = sum_n S_n P_n on the twisted Edwards curve
 * a x^2 + y^2 = 1 + d x^2 y^2 over Fr, a = 168700, d = 168696 (Baby Jubjub;
 * the zero point is (0, 1)), with c-bit windows: K = ceil(256 / c) windows of
 * 2^c buckets.
 *   scalars: device, n x 8 32-bit little-endian words (any value below
 *            2^256; not reduced), 16-byte aligned;
 *   points:  device, n x 16 words: x (8 words) then y (8 words), canonical
 *            or not (read mod r), 16-byte aligned; points must lie on the
 *            curve (not checked: other inputs give an unspecified point);
 *   out:     device, 16 words: the affine result x then y, canonical;
 *   window:  c in [1, 20], or 0 for frntt_msm_window(n).
 * n = 0 gives the zero point. The work is queued on `stream` (0: the null
 * stream) in the context's per-stream scratch (frntt_msm_workspace_bytes;
 * grown as needed, with a synchronisation of the stream when it grows). An
 * MSM cannot be captured into a hipGraph (its radix sort clears counters
 * with memset nodes): under a stream capture the call returns ESTATE and
 * enqueues nothing. Errors: EINVAL (null pointer, n < 0), ERANGE (n > 2^26,
 * window outside [0, 20]), EALIGN, ENOMEM, ESTATE (stream capture), EHIP. */
int frntt_msm(frntt_ctx *ctx, const void *scalars, const void *points, int64_t n, int window, void *out,
              void *stream);
/* Several independent MSMs in one call: MSM i reads scalars[i] and
 * points[i] (n[i] points) and writes out[i], with the layouts, window and
 * errors of frntt_msm. They run on up to three streams of the context's own
 * (default priority), and `stream` waits for all of them, so that one MSM's
 * latency-bound tail (small reduction levels, the one-wave window merge)
 * overlaps another's accumulation. Every argument is checked before
 * anything is enqueued; a later failure (e.g. ENOMEM for scratch) leaves
 * the MSMs before it enqueued. Each side stream holds its own scratch
 * (frntt_msm_workspace_bytes of the largest MSM it ran). Calls on one
 * context enqueue one batch at a time. ESTATE under a stream capture. */
int frntt_msm_batch(frntt_ctx *ctx, const void *const *scalars, const void *const *points, const int64_t *n,
                    int count, int window, void *const *out, void *stream);
/* The same MSM by the paper's dataflow baseline, Presort-PPG (Background,
 * "Presorting Pippenger"; Table 2): every window's points are first written
 * to HBM in bucket order (96 bytes per point and window) and the bucket
 * accumulation reads that copy, where frntt_msm reads the points through the
 * sorted index lists and never writes a presorted copy (the layout-stationary
 * dataflow of Alg. 2). Bit-identical result. Needs n K 96 bytes of scratch
 * more than frntt_msm_workspace_bytes reports. Arguments and errors as
 * frntt_msm. */
int frntt_msm_presort(frntt_ctx *ctx, const void *scalars, const void *points, int64_t n, int window, void *out,
                      void *stream);
/* Batch scalar multiplication on the same curve: out_i = S_i P_i, affine
 * (16 words per point: x then y, canonical), n points; the layouts, the
 * alignment and the on-curve requirement of frntt_msm. out may not overlap
 * the inputs. Used to produce curve points (multiples of a generator) for
 * MSM workloads, and as the per-term product of the MSM definition.
 * Errors: EINVAL, ERANGE (n > 2^26), EALIGN, EHIP. */
int frntt_ec_mul(frntt_ctx *ctx, const void *scalars, const void *points, int64_t n, void *out, void *stream);
/* Window width frntt_msm picks for n points: from 2^13 points on, the
 * width measured fastest on MI355X for floor(log2 n) (uniform 254-bit
 * scalars; 15 at 2^20, 16 at 2^22 and 2^24, 20 at 2^26); below, the c that
 * minimises K (n + 5 2^c) additions. */
int frntt_msm_window(int64_t n);
/* Scratch bytes of frntt_msm for (n, window); 0 for arguments it rejects. */
size_t frntt_msm_workspace_bytes(int64_t n, int window);

/* Last hipError_t seen by the context (0 if none). */
int frntt_last_hip_error(const frntt_ctx *ctx);
/* Static description of a status code. */
const char *frntt_strerror(int status);

/* ---- serving: continuous batching of requests (see frntt_server_*) ----
 * A server owns a worker thread, `slots` streams and a device memory pool
 * bounded by `hbm_budget_bytes` (twiddle tables included). Requests are
 * admitted in arrival order while their buffers fit the budget; admitted
 * requests are grouped into batches and launched on a free slot stream, so
 * work that arrives while other batches run overlaps with them.
 * Request data are generated on the device from (data_seed, request id),
 * using the same generator as frntt_generate with stream_id = request id.
 */
int frntt_server_create(frntt_server **out, frntt_ctx *ctx, size_t hbm_budget_bytes, int slots);
/* Queue a request; returns its ticket. EBUSY if the request alone exceeds
 * the budget. */
int frntt_server_submit(frntt_server *srv, int kind, int log_n, uint64_t data_seed,
                        uint64_t *ticket);
/* done = 1 once the result is on the device; latency_ms = completion time
 * minus submit time (host clock). ESTATE for an unknown ticket. */
int frntt_server_poll(frntt_server *srv, uint64_t ticket, int *done, double *latency_ms);
/* Copy a finished request's result (2^log_n elements) to host memory and
 * release its buffer. ESTATE if not finished or unknown. */
int frntt_server_result(frntt_server *srv, uint64_t ticket, void *host_out);
/* Release a finished request's buffer without copying. */
int frntt_server_release(frntt_server *srv, uint64_t ticket);
/* Wait up to timeout_s seconds until every submitted request is done.
 * EBUSY on time-out, or at once if the server is stalled: the queue head
 * does not fit the budget, nothing is running, and only releasing finished
 * results (frntt_server_result / frntt_server_release) can make room. */
int frntt_server_drain(frntt_server *srv, double timeout_s);
/* on != 0: return a request's buffer to the pool as soon as it completes
 * (poll still reports its latency; result() then returns ESTATE). For
 * clients that consume results on the device or only measure latency. */
int frntt_server_set_release_on_done(frntt_server *srv, int on);
/* Counters: requests completed, batches launched, peak bytes in flight. */
int frntt_server_stats(frntt_server *srv, uint64_t *completed, uint64_t *batches,
                       uint64_t *peak_bytes);
/* Largest number of batches (each one ntt_batch launch sequence on its own
 * slot stream) and of requests that were launched and not yet complete at the
 * same time: batches > 1 means launches were in flight together. */
int frntt_server_peak_inflight(frntt_server *srv, uint64_t *batches, uint64_t *requests);
/* Cancel requests not yet admitted, wait for running batches, stop the
 * worker and free everything. */
int frntt_server_destroy(frntt_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* FRNTT_H */
