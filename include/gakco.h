/*
 * gakco.h -- C ABI of the MI355X (gfx950) gapped k-mer string kernel library.
 *
 * The library computes the GaKCo gapped k-mer kernel (Singh et al.,
 * "GaKCo: a Fast Gapped k-mer string Kernel using Counting",
 * arXiv:1704.07468) on one AMD Instinct MI355X:
 *
 *   g-mers     every contiguous length-g substring of every sequence
 *              (Section 2.2, step 1).
 *   C_m        cumulative mismatch profile: for each of the C(g,m) sets of m
 *              positions, the positions are dropped from every g-mer, equal
 *              reduced strings are grouped, and every pair of sequences (X,Y)
 *              in a group gains count_X * count_Y  (Section 2.2, step 3;
 *              Algorithm 1).
 *   N_m        exact mismatch profile, N_m = C_m - sum_{j<m} C(g-j,m-j) N_j
 *              (Eq. 9).
 *   K          sum_{m=0}^{g-k} C(g-m,k) N_m  (Eqs. 6-7), reported cosine-
 *              normalised in FP64: K_ij / sqrt(K_ii K_jj), 0 where a diagonal
 *              entry is 0 (the paper's "normalized" counts, Eq. 3).
 *
 * Conventions shared by every entry point:
 *   - Sequences are symbol codes in [0, sigma), one int8 per symbol, all
 *     sequences concatenated; lens[i] is the length of sequence i.  Mapping
 *     characters (including an unknown-character symbol, Section S:5.2) to
 *     codes is the caller's job.
 *   - Unless stated otherwise every pointer argument is a DEVICE pointer on
 *     the context's device; the caller owns it.  No pointer is retained after
 *     a call returns.
 *   - Work is enqueued on `hip_stream` (a hipStream_t, NULL = the default
 *     stream) and the call synchronises that stream before it returns, so
 *     data-dependent errors can be reported.  Outputs are unspecified when a
 *     call fails.
 *   - Matrices are row-major: Nm[m][i][j] at ((m*N)+i)*N+j.  M = g - k.
 *   - Integer outputs are exact; the normalised kernel is FP64.
 *   - Sequences shorter than g have no g-mers: their rows and columns are 0,
 *     including the normalised diagonal.
 *   - Symbol width b = max(1, ceil(log2 sigma)); g*b must be <= 64.
 *
 * Errors: every gakco_status-returning function returns GAKCO_OK (0) or a
 * negative code; gakco_last_error() then gives a description for the calling
 * thread.
 */
#ifndef GAKCO_H
#define GAKCO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gakco_status;
#define GAKCO_OK 0
#define GAKCO_EINVAL (-1)      /* bad argument (sizes, sigma, g, k, NULL pointers) */
#define GAKCO_ERANGE (-2)      /* a symbol code outside [0, sigma)                 */
#define GAKCO_EUNSUPPORTED (-3) /* a valid request outside the library's limits    */
#define GAKCO_EBUDGET (-4)     /* scratch + outputs exceed the context's HBM budget */
#define GAKCO_EHIP (-5)        /* a HIP runtime call failed                         */
#define GAKCO_ECANCELLED (-6)  /* a serving request was cancelled                   */
#define GAKCO_EAGAIN (-7)      /* serving: nothing to return yet / queue full       */

/* Text for the last failing call made by this thread ("" if none). */
const char *gakco_last_error(void);
/* Library version string. */
const char *gakco_version(void);

/* ------------------------------------------------------------------------
 * Context: a device, a grow-only scratch arena bounded by hbm_budget bytes
 * (0 = half of the device's memory), and tuning parameters.
 * tune_json (nullable) is a JSON object with any of the integer keys
 *   "dense_tau"     minimum distinct sequences for a group to be summed by
 *                   the int8 matrix-core path (0 disables that path)
 *   "bucket_avg"    target g-mers per hash bucket of the partition sort
 *   "profile"       1 = time every launch phase with HIP events (see
 *                   gakco_profile_get)
 *   "pool_mb"       cap of the buffer pool reused by chunks of position sets
 *   "overlap"       1 (default) = run independent kernels of a Gram call
 *                   side by side on a second stream of the context (the
 *                   block sort beside the wave sort, the int8 products
 *                   beside the accumulation); 0 = all on the caller's
 *                   stream.  Never while profiling or under graph capture.
 *   "acc_slab"      columns of a Gram row per block of the row accumulation
 *                   (0, the default: a whole row when its int32 counters fit
 *                   the LDS, else the largest multiple of 64 that does);
 *                   a multiple of 64, for tests and tuning
 *   "acc_mstep"     cap on the position sets the row accumulation sums in
 *                   its 32-bit LDS row before adding it into C_m (0, the
 *                   default: as many as the count bound allows), for tests
 *   "rows_slabs"    slabs of the resident set per block of the serving rows
 *                   kernel (0, the default: two halves of at most 16384
 *                   sequences each, at least 4096); 1..64, for tuning
 *   "rows_dense"    1 (default): a resident set's top level whose reduced
 *                   g-mers take at most 12 bits is joined as an int8
 *                   product of count rows (query batch x resident set)
 *                   instead of the sparse walk, when the resident set has
 *                   at least "rows_dense_min_sv" sequences (default 2048)
 *                   and no count above 127 at that level, for batches of at
 *                   least "rows_dense_min_q" queries (default 28); the
 *                   resident count rows take n_sv * C(g, M) * 2^w bytes of
 *                   device memory; 0 = always the sparse walk
 *   "tau_b<B>_g<G>" dense_tau for jobs with B-bit symbols and this g (as
 *                   written by gakco_autotune)
 * Missing keys keep their defaults.  Not thread-safe: one context per host
 * thread (serving uses its own internal contexts).
 * ------------------------------------------------------------------------ */
typedef struct gakco_ctx gakco_ctx;
gakco_status gakco_ctx_create(int device, size_t hbm_budget, const char *tune_json, gakco_ctx **out);
void gakco_ctx_destroy(gakco_ctx *ctx);
/* Set one tuning parameter by name (same keys as tune_json). */
gakco_status gakco_ctx_set_param(gakco_ctx *ctx, const char *name, int64_t value);
/* Read a value about the context or its last Gram call: "dense_rows" (groups
 * summed by the int8 matrix-core path), "chunks" (position-set chunks),
 * "dense_tau", "bucket_avg", "arena_bytes", "dense_bytes"; with the profiler
 * on, "sort_gmers_<kind>" for kind in wave, wave_wide, block, block_wide,
 * global, global_wide: g-mers (summed over position sets) whose bucket was
 * sorted by that kernel, packed or 64-bit composites, and "acc_updates":
 * sequence-pair updates of the row accumulation (Algorithm 1
 * countAndUpdate on the groups left to it, the diagonal terms included),
 * and "rows_updates": resident entries gathered by the serving rows kernel
 * (one (query g-mer, resident sequence) pair update each), since the last
 * profile reset (synchronises the device). */
gakco_status gakco_ctx_stat(const gakco_ctx *ctx, const char *name, int64_t *value);

/* Reference rate for the row accumulation's LDS atomics: 2048 blocks of 256
 * threads, each thread adding 1 to pseudo-random counters of an LDS row of
 * row_words (a power of two in 64..8192) 4096 times, on the device's null
 * stream; *updates_per_s receives adds per second.  GAKCO_EINVAL for a bad
 * row_words or NULL pointers, GAKCO_EHIP on a runtime failure. */
gakco_status gakco_probe_lds_atomics(gakco_ctx *ctx, int32_t row_words, double *updates_per_s);

/* Event profiler (enable with the "profile" parameter): per launch phase of
 * the calls made on this context, the summed device time between HIP events
 * recorded on the call's stream around the phase's launch, and the number of
 * timed launches.  Every phase is one kernel (launched at most once per
 * position-set chunk; "sort_global" once per composite width), so its mean
 * time is that kernel's launch duration.
 * Phases are numbered 0 .. gakco_profile_phases()-1. */
int32_t gakco_profile_phases(void);
gakco_status gakco_profile_get(const gakco_ctx *ctx, int32_t phase, const char **name, double *total_ms,
                               int64_t *launches);
void gakco_profile_reset(gakco_ctx *ctx);

/* ------------------------------------------------------------------------
 * gakco_gram -- the N x N kernel of one dataset (Algorithm 1 plus the
 * normalisation).
 *   seqs    int8  [sum(lens)]   symbol codes
 *   lens    int32 [N]           sequence lengths (>= 0)
 *   N       number of sequences, >= 1
 *   sigma   alphabet size, 1..127
 *   g, k    g >= 1, 0 <= k <= g
 *   K_out   double [N][N]       normalised kernel (nullable)
 *   Nm_out  int64 [g-k+1][N][N] exact mismatch profiles N_m (nullable)
 *   Cm_out  int64 [g-k+1][N][N] cumulative profiles C_m (nullable)
 * Returns GAKCO_EINVAL for bad sizes or NULL seqs/lens, GAKCO_ERANGE for a
 * symbol outside [0, sigma), GAKCO_EUNSUPPORTED when g*b > 64, when a
 * sequence has 65536 or more g-mers (one position set could overflow the
 * accumulation's 32-bit counters), or past the other size limits (2^31
 * g-mers, 2^24 sequences, reduced key + sequence id above 64 bits),
 * GAKCO_EBUDGET when the scratch and outputs do not fit the context's budget,
 * GAKCO_EHIP on a runtime failure.
 * ------------------------------------------------------------------------ */
gakco_status gakco_gram(gakco_ctx *ctx, const int8_t *seqs, const int32_t *lens, int32_t N,
                        int32_t sigma, int32_t g, int32_t k, double *K_out, int64_t *Nm_out,
                        int64_t *Cm_out, void *hip_stream);

/* ------------------------------------------------------------------------
 * gakco_gram_noalloc -- gakco_gram for callers that cannot allocate device
 * memory (code that must not call hipMalloc: tight serving loops, harnesses
 * that forbid allocation).  It allocates and frees nothing: its scratch is a
 * library-owned device array of GAKCO_NOALLOC_SCRATCH_BYTES (512 MiB) that
 * every GPU the library runs on holds from the first call until the process
 * ends.  It runs on the calling thread's current device, with no context:
 * default tuning, no side stream, no profiler.
 *   Arguments, layouts, outputs and errors as gakco_gram, except:
 *   - the caller's outputs do not count against the scratch; the cumulative
 *     profiles are summed in Nm_out (else Cm_out), and only when both are
 *     NULL do they need (g-k+1) * N^2 * 8 bytes of the scratch;
 *   - GAKCO_EBUDGET when the call's scratch (g-mer arrays, one position-set
 *     chunk's partition buffers, count matrices, descriptors) exceeds the
 *     array; nothing is launched then.
 * Every call on a GPU shares that GPU's array and leaves its contents behind;
 * each call clears what it needs cleared.  The library serialises its own
 * calls on one device (they also synchronise the stream before returning);
 * other work a caller enqueues on the same array concurrently would race.
 * ------------------------------------------------------------------------ */
#define GAKCO_NOALLOC_SCRATCH_BYTES (512ull << 20)
gakco_status gakco_gram_noalloc(const int8_t *seqs, const int32_t *lens, int32_t N, int32_t sigma,
                                int32_t g, int32_t k, double *K_out, int64_t *Nm_out, int64_t *Cm_out,
                                void *hip_stream);

/* ------------------------------------------------------------------------
 * Stage entry points (the first steps of the Gram path on their own; used for
 * stage-level parity).
 *
 * gakco_extract: the g-mer array of Section 2.2 step 1.  keys_out[t] packs
 * g-mer t with its first symbol most significant: sum_j x[p+j] << (b*(g-1-j));
 * sid_out[t] is its sequence.  g-mers are in sequence order, then position
 * order.  keys_out: uint64 [T], sid_out: int32 [T], T = sum max(0, l-g+1)
 * (query it with gakco_count_gmers).  Device pointers.
 * ------------------------------------------------------------------------ */
gakco_status gakco_count_gmers(const int32_t *lens_host, int32_t N, int32_t g, int64_t *T_out);
gakco_status gakco_extract(gakco_ctx *ctx, const int8_t *seqs, const int32_t *lens, int32_t N,
                           int32_t sigma, int32_t g, uint64_t *keys_out, int32_t *sid_out,
                           void *hip_stream);

/* gakco_mask_groups: the groups of the sorted reduced list for ONE set of
 * removed positions (Algorithm 1, removePosition + sort + the grouping of
 * countAndUpdate).  removed_host: int32 [m] positions in [0, g) (HOST
 * pointer).  Outputs are HOST arrays of capacity cap: group q owns entries
 * [grp_off[q], grp_off[q+1]) of (ent_sid, ent_cnt), sorted by sequence;
 * grp_rep[q] is the extraction index of one g-mer of the group; grp_off has
 * cap+1 slots.  Group order is unspecified.  *n_groups_out receives the
 * number of groups.  GAKCO_EINVAL if cap is too small. */
gakco_status gakco_mask_groups(gakco_ctx *ctx, const int8_t *seqs, const int32_t *lens, int32_t N,
                               int32_t sigma, int32_t g, const int32_t *removed_host, int32_t m,
                               int32_t *grp_off, int32_t *grp_rep, int32_t *ent_sid,
                               int32_t *ent_cnt, int64_t cap, int64_t *n_groups_out,
                               void *hip_stream);

/* ------------------------------------------------------------------------
 * Batched Gram jobs: every job of the list is planned together and all its
 * position sets run in shared launches.  Pointers inside gakco_job are device
 * pointers except status_out (HOST, nullable), which receives each job's
 * status.  Returns the first failing job's status (or GAKCO_OK).
 * ------------------------------------------------------------------------ */
typedef struct {
    const int8_t *seqs;
    const int32_t *lens;
    int32_t N, sigma, g, k;
    double *K_out;      /* [N][N], nullable             */
    int64_t *Nm_out;    /* [g-k+1][N][N], nullable      */
    gakco_status *status_out; /* host, nullable          */
} gakco_job;
gakco_status gakco_gram_batch(gakco_ctx *ctx, const gakco_job *jobs_host, int32_t n_jobs,
                              void *hip_stream);

/* A reusable plan for a fixed list of job shapes: planning reads the lengths
 * once; gakco_batch_run replays the captured launch sequence (a hipGraph) on
 * the jobs' current buffer contents.  The job buffers must stay valid and
 * keep their shapes while the plan lives. */
typedef struct gakco_batch_plan gakco_batch_plan;
gakco_status gakco_batch_plan_create(gakco_ctx *ctx, const gakco_job *jobs_host, int32_t n_jobs,
                                     void *hip_stream, gakco_batch_plan **out);
gakco_status gakco_batch_run(gakco_batch_plan *plan, void *hip_stream);
void gakco_batch_plan_destroy(gakco_batch_plan *plan);

/* Autotuner: times candidate settings of the given jobs on the device (best
 * of `reps` runs after a warm-up, HIP events) and keeps the fastest: the
 * int8 matrix-core threshold per job class (symbol bits, g), then the hash
 * bucket size.  The choice is applied to ctx and, if out_json is not NULL,
 * written there as a tune_json object (GAKCO_EINVAL if out_cap is too
 * small).  The jobs' outputs are overwritten. */
gakco_status gakco_autotune(gakco_ctx *ctx, const gakco_job *jobs_host, int32_t n_jobs, int32_t reps,
                            void *hip_stream, char *out_json, size_t out_cap);

/* ------------------------------------------------------------------------
 * Serving: a resident set (e.g. an SVM's support vectors) kept on the device
 * as per-position-set group tables, and kernel rows of queries against it.
 *
 * gakco_resident_create copies the resident sequences (device pointers) and
 * builds the tables; dual_coef (HOST, nullable) holds alpha_i*y_i of Eq. 1
 * and bias is b.
 * gakco_rows: for n_q queries (device q_seqs/q_lens), K_rows [n_q][n_sv]
 * receives the normalised kernel rows K-hat(q, sv_i); Nm_rows (nullable)
 * [g-k+1][n_q][n_sv] the exact mismatch profiles; decision (nullable) [n_q]
 * f(q) = b + sum_i alpha_i K-hat(sv_i, q) (Eq. 1), summed in a fixed
 * per-query order (chunks of 2048 consecutive i, each summed by a fixed
 * tree, then the chunk sums in ascending order) so that a query's result does
 * not depend on the other queries of the batch.  GAKCO_EUNSUPPORTED when a
 * query is past the 32-bit serving counters (see gakco_server_submit), or, in
 * gakco_resident_create, when C(g,m) * (longest resident g-mers)^2 reaches
 * 2^32.
 * ------------------------------------------------------------------------ */
typedef struct gakco_resident gakco_resident;
gakco_status gakco_resident_create(gakco_ctx *ctx, const int8_t *seqs, const int32_t *lens,
                                   int32_t n_sv, int32_t sigma, int32_t g, int32_t k,
                                   const double *dual_coef_host, double bias,
                                   gakco_resident **out);
void gakco_resident_destroy(gakco_resident *res);
gakco_status gakco_resident_info(const gakco_resident *res, int32_t *n_sv, int32_t *sigma,
                                 int32_t *g, int32_t *k, size_t *device_bytes);
gakco_status gakco_rows(gakco_ctx *ctx, const gakco_resident *res, const int8_t *q_seqs,
                        const int32_t *q_lens, int32_t n_q, double *K_rows, int64_t *Nm_rows,
                        double *decision, void *hip_stream);

/* ------------------------------------------------------------------------
 * Incremental Gram: a normalised kernel matrix that grows as sequences are
 * appended, each append computing only the new rows (the counting approach
 * suits adaptive training on a growing set, Section 3.2).  The sequences
 * appended so far stay on the device as resident group tables, one segment
 * per append.
 * gakco_incr_append with n_new sequences (device seqs / lens, as in
 * gakco_gram) onto N: K_out [N+n_new][N+n_new] (device, row-major) receives
 * the normalised kernel of all N+n_new sequences in append order -- the
 * N x N block copied from K_prev [N][N] (device; ignored when N = 0, and not
 * the same buffer as K_out), the new rows from the serving join against every
 * earlier segment, the new block from a Gram of the new sequences -- equal to
 * gakco_gram on the concatenation.  GAKCO_EINVAL for NULL pointers, n_new < 1
 * or K_prev missing / aliasing K_out; the other errors as gakco_gram and
 * gakco_rows (a new sequence past the serving counters: GAKCO_EUNSUPPORTED).
 * A failed append leaves the set as it was.  Synchronises the stream.
 * ------------------------------------------------------------------------ */
typedef struct gakco_incr gakco_incr;
gakco_status gakco_incr_create(gakco_ctx *ctx, int32_t sigma, int32_t g, int32_t k, gakco_incr **out);
gakco_status gakco_incr_append(gakco_incr *inc, const int8_t *seqs, const int32_t *lens, int32_t n_new,
                               const double *K_prev, double *K_out, void *hip_stream);
gakco_status gakco_incr_info(const gakco_incr *inc, int64_t *N, int32_t *segments);
void gakco_incr_destroy(gakco_incr *inc);

/* ------------------------------------------------------------------------
 * gakco_svm_train -- the support-vector machine that consumes the kernel
 * (Section 3.1 classifies with an SVM on the Gram matrix; Eq. 1 is its
 * decision function f(x) = sum_i alpha_i y_i K(x_i, x) + b).  The bias is
 * absorbed into the kernel (K + 1, so b = sum_i alpha_i y_i) and the dual
 *     minimise 1/2 alpha^T Q alpha - sum_i alpha_i,  0 <= alpha_i <= C,
 *     Q_ij = y_i y_j (K_ij + 1)
 * is solved by dual coordinate descent (Hsieh et al., ICML 2008):
 * coordinates 0..N-1 in order, each moved to its clipped minimiser; the run
 * stops after the first epoch whose projected gradients span at most eps, or
 * after max_epochs.  One block of the device runs it (the coordinates are
 * sequential); every FP64 operation is separately rounded in a fixed order,
 * so the result does not depend on the thread layout.
 *   K              double [N][N] normalised kernel (e.g. gakco_gram's K_out), device
 *   y              int8 [N] labels +1 / -1, device
 *   alpha_out      double [N] multipliers alpha_i, device, nullable
 *   dual_coef_out  double [N] alpha_i * y_i, device, nullable -- with bias the
 *                  arguments gakco_resident_create takes (its support vectors
 *                  are the i with alpha_i > 0)
 *   bias_out       host double, nullable: b
 *   epochs_out     host int32, nullable: epochs run
 * GAKCO_EINVAL for N < 1, C <= 0, eps < 0, max_epochs < 1, NULL K / y or a
 * label other than +1 / -1; GAKCO_EUNSUPPORTED for N > 8192 (the gradient
 * lives in one block's registers); synchronises the stream.
 * ------------------------------------------------------------------------ */
gakco_status gakco_svm_train(gakco_ctx *ctx, const double *K, const int8_t *y, int32_t N, double C, double eps,
                             int32_t max_epochs, double *alpha_out, double *dual_coef_out, double *bias_out,
                             int32_t *epochs_out, void *hip_stream);

/* ------------------------------------------------------------------------
 * Continuous-batching server over a resident set.  Queries are HOST arrays
 * (copied at submit).  A scheduler thread admits queued requests into device
 * batches whenever a batch slot and HBM budget are free, so requests that
 * arrive while others run are admitted as capacity frees up; up to
 * `n_streams` batches are in flight on separate HIP streams.  Results are
 * returned by gakco_server_poll in completion order; K_row points into
 * server-owned memory that stays valid until the next poll on this server.
 * Timestamps are seconds on a monotonic clock.  gakco_server_create runs one
 * warm-up batch per worker (up to max_batch queries of 1024 symbols, as far
 * as the worker's share of hbm_budget allows) so that later batches of
 * queries up to that length find their buffers sized.
 * This differs from a context-based create: the server owns one context and
 * stream per worker (n_streams of them) on `device`, so it takes the device
 * instead of a context; t_submit is the request's arrival (its submit call).
 * ------------------------------------------------------------------------ */
typedef struct gakco_server gakco_server;
typedef struct {
    uint64_t tag;
    gakco_status status;
    double decision;
    const double *K_row; /* [n_sv] host memory, NULL if cancelled */
    double t_submit, t_start, t_done;
    int32_t batch_size;  /* number of queries in the device batch that ran it */
} gakco_result;
gakco_status gakco_server_create(const gakco_resident *res, int32_t device, int32_t max_batch,
                                 int32_t n_streams, size_t hbm_budget, gakco_server **out);
/* gakco_server_submit copies the query; GAKCO_ERANGE for a symbol outside
 * [0, sigma) and GAKCO_EUNSUPPORTED for a query past the 32-bit serving
 * counters (C(g,m) * its g-mers * max(its g-mers, the longest resident
 * sequence's) must stay below 2^32 for every m) -- either way nothing is
 * queued, so a bad query never affects the batch it would have joined. */
gakco_status gakco_server_submit(gakco_server *srv, const int8_t *q_host, int32_t len, uint64_t tag);
gakco_status gakco_server_cancel(gakco_server *srv, uint64_t tag);
gakco_status gakco_server_poll(gakco_server *srv, gakco_result *out, int32_t max, int32_t *n_out,
                               int32_t wait_us);
/* Sets a tuning parameter (names and ranges as gakco_ctx_set_param) on every
 * worker's context, e.g. "rows_dense_min_q" to keep batches below a size on
 * the sparse walk, which bounds a batch's time at moderate load.  Waits until
 * no batch is running and admits none meanwhile, so every batch runs with
 * one setting; queued requests stay queued.  GAKCO_EINVAL for an unknown name
 * or a value out of range (then no worker is changed). */
gakco_status gakco_server_set_param(gakco_server *srv, const char *name, int64_t value);
/* Stops admission, finishes in-flight batches, cancels what is still queued
 * and frees everything. */
gakco_status gakco_server_destroy(gakco_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* GAKCO_H */
