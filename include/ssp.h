/*
 * ssp.h -- sampled-compression-ratio structure prediction for SpGEMM on AMD
 * Instinct MI355X (gfx950).
 *
 * The method is that of Du et al., "Predicting the Output Structure of Sparse
 * Matrix Multiplication with Sampled Compression Ratio" (arXiv 2207.13848):
 * for C = A.B it counts the intermediate products of every output row
 * (Sec. V-A, Alg. 1), samples rows of A (Sec. IV-A), counts the distinct
 * output columns of the sampled rows exactly (Sec. IV-B, Alg. 2), forms the
 * sampled compression ratio r* = f* / z* and predicts every row as its product
 * count divided by r* (Sec. IV-D, Eq. (4)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Matrices are CSR, structure only (no values): int32 row pointers
 *    rpt[nrows+1] with rpt[0] = 0, non-decreasing, rpt[nrows] = nnz, and int32
 *    column indices col[nnz] in [0, ncols).  Rows may be unsorted and may
 *    repeat a column: product counts count stored entries, distinct counts
 *    count distinct columns.  nnz must fit in int32.
 *  - All array pointers in ssp_csr, all outputs and the optional ssp_stats
 *    are DEVICE pointers on the handle's device.  The caller owns them and
 *    keeps them alive until the work queued on `stream` has finished.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    The prediction, reference, exact and batch entry points enqueue their
 *    work and return once it is queued.  They block the host in two cases
 *    only: when the handle's workspace has to grow (hipDeviceSynchronize
 *    before the old workspace is freed), and, for calls of more than 8
 *    cases, when the pinned buffer that stages the case table is still being
 *    copied from by the previous such call (hipEventSynchronize on that
 *    copy).  Calls documented below as synchronous say so.
 *  - The library owns one device workspace per handle.  It grows on demand
 *    (hipMalloc) up to the handle's HBM budget; once a call of a given size
 *    has run, repeated calls of that size or smaller allocate nothing.  A
 *    handle serves one stream at a time: calls on one handle must not run
 *    concurrently on different streams.
 *  - Host-checkable problems return a negative status synchronously and queue
 *    nothing: null pointers, negative sizes, A.ncols != B.nrows, a rate that
 *    is NaN or outside [0, 1], nnz beyond int32, a workspace beyond the
 *    budget.  The CONTENTS of the CSR arrays are not checked on the compute
 *    path (out-of-range columns are undefined behaviour); ssp_validate_csr is
 *    the explicit check.  HIP failures return SSP_ERR_HIP; ssp_last_error()
 *    gives the HIP message.
 *  - Degenerate shapes are valid: M = 0 only clears the stats; K = 0 or N = 0 give
 *    zero counts.  A and B may alias (C = A.A).
 *  - All results are integers and are independent of launch configuration,
 *    thread timing and tuning: two calls with the same inputs give the same
 *    bytes.
 */
#ifndef SSP_H
#define SSP_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define SSP_API __attribute__((visibility("default")))
#else
#define SSP_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SSP_OK = 0,
    SSP_ERR_INVALID_ARG = -1,  /* null pointer, negative size, bad rate    */
    SSP_ERR_DIM_MISMATCH = -2, /* A.ncols != B.nrows                        */
    SSP_ERR_OVERFLOW = -3,     /* a size does not fit the int32 CSR format  */
    SSP_ERR_BUDGET = -4,       /* workspace would exceed the HBM budget     */
    SSP_ERR_OOM = -5,          /* hipMalloc failed                          */
    SSP_ERR_HIP = -6,          /* a HIP runtime call failed                 */
    SSP_ERR_NO_DEVICE = -7,    /* no such device / not a usable GPU         */
    SSP_ERR_INVALID_CSR = -8,  /* reserved for CSR validation results       */
    SSP_ERR_BUSY = -9,         /* a resource (slot, queue) is full          */
    SSP_ERR_NOT_READY = -10    /* asynchronous result not finished yet      */
} ssp_status;

typedef struct ssp_context* ssp_handle;

/* Structure-only CSR matrix in device memory. */
typedef struct {
    int64_t nrows;
    int64_t ncols;
    int64_t nnz;        /* = rpt[nrows]                                     */
    const int32_t* rpt; /* device, nrows + 1 entries                        */
    const int32_t* col; /* device, nnz entries, each in [0, ncols)          */
} ssp_csr;

/*
 * Statistics of one call, written to device memory (64 bytes).  Names follow
 * the paper: F = FLOP(C) (Alg. 1), n_s sampled rows, f* = sampled FLOP and
 * z* = sampled NNZ (Alg. 2).  The predicted total of Eq. (4) is the exact
 * rational Z2* = F z* / f*; the reference design's is Z1* = z* M / n_s.
 */
typedef struct {
    uint64_t total_flop;  /* F                                            */
    uint64_t n_sampled;   /* n_s (paper sampler: number of draws)         */
    uint64_t sample_flop; /* f*                                           */
    uint64_t sample_nnz;  /* z*                                           */
    uint64_t out_sum;     /* sum of the per-row output of this call       */
    uint64_t nrows;       /* M                                            */
    uint64_t flags;       /* SSP_FLAG_* bits                              */
    uint64_t a_sample_nnz; /* stored entries of A in the sampled rows     */
} ssp_stats;

/* f* = 0 (no sampled row has a product): the ratio is undefined and every
 * row falls back to its product count, the upper bound. */
#define SSP_FLAG_EMPTY_SAMPLE 1u
/* reserved (never set): every value of the reference design fits int64,
 * being at most M N < 2^62 */
#define SSP_FLAG_SATURATED 2u

/* Row sampler.  BERNOULLI: row i is sampled iff
 * (splitmix64(seed, i) >> 11) < floor(rate * 2^53), splitmix64(seed, i) being
 * the (i+1)-th output of the splitmix64 stream (Steele, Lea & Flood 2014)
 * whose state starts at seed.  PAPER: the fixed-count sampler of Alg. 2 and
 * Sec. V-B, min(floor(0.003 M), 300) draws with replacement, draw r picking
 * row (M * (splitmix64(seed, r) >> 11)) >> 53; `rate` is ignored. */
typedef enum { SSP_SAMPLER_BERNOULLI = 0, SSP_SAMPLER_PAPER = 1 } ssp_sampler;

/* ------------------------------------------------------------ lifetime */

/* Create a handle on HIP device `device`.  hbm_budget_bytes bounds the
 * workspace the handle may allocate (0 = no bound).  Allocates nothing yet. */
SSP_API ssp_status ssp_create(ssp_handle* h, int device, size_t hbm_budget_bytes);

/* Release the handle and its workspace.  Waits for the device first. */
SSP_API ssp_status ssp_destroy(ssp_handle h);

/* Workspace bytes the handle holds now. */
SSP_API size_t ssp_workspace_bytes(ssp_handle h);

/* ------------------------------------------------------ the hot path */

/*
 * Predicted nonzeros per row of C = A.B by the proposed method (Sec. IV-D,
 * Eq. (4); Alg. 2): with the Bernoulli sampler at `sample_rate` and `seed`,
 *     nnz_pred[i] = ceil(row_flop[i] * z* / f*)      (exact integers),
 * row_flop[i] being the intermediate products of row i (Alg. 1).  When
 * f* = 0 every row gets row_flop[i] and SSP_FLAG_EMPTY_SAMPLE is set.
 *   nnz_pred : device int64[A.nrows], written.
 *   row_flop : device int64[A.nrows] or NULL; if given, the per-row product
 *              counts (the upper-bound structure) are written too.
 *   stats    : device ssp_stats or NULL.
 */
SSP_API ssp_status ssp_predict_structure(ssp_handle h, const ssp_csr* A, const ssp_csr* B,
                                 double sample_rate, uint64_t seed, int64_t* nnz_pred,
                                 int64_t* row_flop, ssp_stats* stats, void* stream);

/* As ssp_predict_structure with an explicit sampler (see ssp_sampler). */
SSP_API ssp_status ssp_predict_structure_ex(ssp_handle h, const ssp_csr* A, const ssp_csr* B,
                                    ssp_sampler sampler, double sample_rate, uint64_t seed,
                                    int64_t* nnz_pred, int64_t* row_flop, ssp_stats* stats,
                                    void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * prediction as ssp_predict_structure_ex, same arguments, outputs and
 * statistics, bit-identical to it, but its workspace is a fixed array of
 * 256 MiB in the library's device code (one copy per device, taken when the
 * library loads and held until the process ends) instead of the handle's
 * workspace.  It calls no hipMalloc, hipFree or other allocating routine and
 * never blocks the host; it writes none of the handle's workspace and records
 * no timing events.  A product whose workspace plan does not fit the array
 * (about 88 bytes per row of A, 80 when row_flop is given, 2 per row of B,
 * and the bitmap windows of split long rows, 1024 of 128 KiB as in the
 * allocating call or, when the rows leave less room, down to 16: about 3
 * million rows at most) returns SSP_ERR_BUDGET, with the sizes in
 * ssp_last_error(), and queues nothing.  Every call on one device shares that
 * device's array, whatever the handle: calls whose work overlaps on the
 * device (different streams, handles or threads) race and give wrong
 * results; calls queued on one stream are ordered and safe.  Each call
 * clears what it needs cleared itself; the array keeps the last call's
 * contents.
 */
SSP_API ssp_status ssp_predict_structure_noalloc(ssp_handle h, const ssp_csr* A, const ssp_csr* B,
                                                 ssp_sampler sampler, double sample_rate,
                                                 uint64_t seed, int64_t* nnz_pred,
                                                 int64_t* row_flop, ssp_stats* stats,
                                                 void* stream);

/*
 * The reference design of the existing sampling estimator on the same sample
 * (Sec. IV-C, Eq. (2)): Z1* = z* / p with p = n_s / M, and every row gets
 *     nnz_ref[i] = ceil(row_flop[i] * z* * M / (n_s * F)),
 * not clamped (a value is at most M N; its numerator, up to 2^155, is
 * divided exactly).
 * Same fallback as above when f* = 0.
 *   nnz_ref : device int64[A.nrows], written.
 */
SSP_API ssp_status ssp_reference_estimate(ssp_handle h, const ssp_csr* A, const ssp_csr* B,
                                  ssp_sampler sampler, double sample_rate, uint64_t seed,
                                  int64_t* nnz_ref, ssp_stats* stats, void* stream);

/*
 * The precise method (Sec. I, the symbolic phase): the exact number of
 * distinct columns of every row of C = A.B.  stats->out_sum = Z = NNZ(C),
 * stats->total_flop = F; the sample fields are zero.
 *   nnz_exact : device int64[A.nrows], written.
 */
SSP_API ssp_status ssp_exact_structure(ssp_handle h, const ssp_csr* A, const ssp_csr* B,
                               int64_t* nnz_exact, ssp_stats* stats, void* stream);

/* ----------------------------------------------------------- batches */

/*
 * One product of a batch: the arguments of ssp_predict_structure_ex.  The
 * CSR descriptors are copied by value; the arrays they point to, and the
 * outputs, are device memory the caller owns (as above).
 */
typedef struct {
    ssp_csr A;
    ssp_csr B;
    int32_t sampler;      /* ssp_sampler                                   */
    int32_t reserved;     /* 0                                             */
    double sample_rate;
    uint64_t seed;
    int64_t* nnz_pred;    /* device int64[A.nrows], written                */
    int64_t* row_flop;    /* device int64[A.nrows] or NULL                 */
    ssp_stats* stats;     /* device ssp_stats or NULL                      */
} ssp_case;

/*
 * Predicts every case of a batch (the workload shape of the paper's 625
 * products, Sec. VI-A) with one launch sequence whose grids span all cases:
 * each stage (streaming FLOP pass, sampling, distinct counts, reduction,
 * prediction) is one kernel for the whole batch, the workgroups of a stage
 * shared among the cases in proportion to their work.  Every case's outputs
 * and statistics are bit-identical to ssp_predict_structure_ex on that case
 * alone.  n = 0 is a no-op.  Errors as for the single call (the first
 * failing case decides); nothing is queued on an error.
 */
SSP_API ssp_status ssp_predict_batch(ssp_handle h, int n, const ssp_case* cases, void* stream);

/*
 * A batch captured once as a HIP graph, replayed by ssp_batch_graph_launch.
 * Creation plans the batch, allocates the graph's own workspace (hipMalloc,
 * bounded by the handle's HBM budget), uploads the case table and captures
 * the launch sequence; it synchronises with the device.  A launch allocates
 * nothing and queues one graph on `stream`: the outputs named at creation
 * are rewritten from the current contents of the inputs, whose sizes and
 * addresses are fixed at creation.  Launches of one graph must not overlap
 * (they share its workspace).  Destroy waits for the device and frees the
 * graph and its workspace; the handle must outlive its graphs.
 */
typedef struct ssp_batch_graph_s* ssp_batch_graph;
SSP_API ssp_status ssp_batch_graph_create(ssp_handle h, int n, const ssp_case* cases,
                                          ssp_batch_graph* graph);
SSP_API ssp_status ssp_batch_graph_launch(ssp_batch_graph graph, void* stream);
SSP_API size_t ssp_batch_graph_workspace_bytes(ssp_batch_graph graph);
SSP_API ssp_status ssp_batch_graph_destroy(ssp_batch_graph graph);

/* ------------------------------------------------------------ tuning */

/*
 * Launch parameters of the distinct-count stage, per handle (a server copies
 * its handle's at creation).  Outputs never depend on them (every count is
 * exact); only speed does.
 *   bin_max[3]  : rows of up to bin_max[0] products are counted by one
 *                 wavefront each, up to bin_max[1] by 256 threads, up to
 *                 bin_max[2] by 512 threads, longer ones by the 1024-thread
 *                 long-row kernel.  Defaults 128, 1024, 8192.
 *   hash_mult   : LDS hash tables hold at least hash_mult times a row's
 *                 distinct bound (2, 4 or 8; default 2).  Limits:
 *                 bin_max[0..2] * hash_mult <= 256, 2048, 16384.
 *   long_len    : the long-row kernel walks B rows of at least long_len
 *                 columns in 256-column units by wavefront, shorter ones
 *                 flattened over the workgroup (8..1024; default 16).
 *   big3        : 1 (default): when one 2^20-column bitmap covers all of B's
 *                 columns but bin 3 would hash, bin-3 rows go to the long-row
 *                 kernel; 0: never.
 *   split_target: long rows above this many products are split into parts
 *                 (2^12..2^40; default 2^19).
 *   est_max_rf  : the prediction's per-row ceiling ceil(rf z* / f*) takes a
 *                 double-precision estimate corrected in integers for rows
 *                 of fewer than est_max_rf products, a 128-bit division for
 *                 the others (0..2^48; default 2^48, the largest value for
 *                 which the estimate is exact).
 */
typedef struct {
    uint32_t bin_max[3];
    uint32_t hash_mult;
    uint32_t long_len;
    int32_t big3;
    uint64_t split_target;
    uint64_t est_max_rf;
} ssp_tuning;

/* Defaults, current value, and change (SSP_ERR_INVALID_ARG outside the limits). */
SSP_API void ssp_default_tuning(ssp_tuning* t);
SSP_API ssp_status ssp_get_tuning(ssp_handle h, ssp_tuning* t);
SSP_API ssp_status ssp_set_tuning(ssp_handle h, const ssp_tuning* t);

/*
 * Picks the tuning for a representative batch (n >= 1 cases, as for
 * ssp_predict_batch) by coordinate descent from the handle's current tuning:
 * each parameter in turn is tried at a few values, every candidate timed as
 * the mean of `reps` batch calls (HIP events on `stream`, after a warm-up);
 * a change is kept when it is at least 2% faster.  Sets the handle's tuning
 * to the result and returns it in *chosen, with its time and the default
 * tuning's time in *best_ms and *default_ms (either may be NULL).  The cases'
 * outputs are written by every trial.  Synchronises with the device.
 */
SSP_API ssp_status ssp_autotune(ssp_handle h, int n, const ssp_case* cases, int reps,
                                ssp_tuning* chosen, double* best_ms, double* default_ms,
                                void* stream);

/* ----------------------------------------------------------- serving */

/*
 * A request server with continuous batching over device-resident matrices.
 * A worker thread owns `nslots` slots (a stream, a workspace of slot_bytes
 * and a pinned staging buffer each; nslots * slot_bytes is allocated at
 * creation and counts against the handle's HBM budget).  Submitted requests
 * queue in arrival order; whenever a slot is free the worker admits the
 * oldest requests whose workspaces fit the slot together (at most max_batch)
 * and launches them as one batch (ssp_predict_batch semantics) on the slot's
 * stream, so batches on different slots overlap on the device and requests
 * arriving meanwhile join the next free slot.  A request's result is
 * bit-identical to ssp_predict_structure_ex on the same inputs, alone or in
 * any mix.  Latency is the time from submission to the worker seeing the
 * request's batch complete.
 *
 *  create   : slot_bytes 0 = 1 GiB; SSP_ERR_BUDGET beyond the handle's budget.
 *             The handle must outlive the server (the server uses its device).
 *  register : keeps a copy of the descriptor; the arrays stay the caller's
 *             and must stay alive and unchanged while requests use them.
 *             Returns the matrix id in *id.
 *  submit   : C = mats[a] . mats[b]; nnz_pred (device int64[nrows of a]) and
 *             stats (device or NULL) must stay alive until the request is done.
 *             The slots' streams do not wait for the caller's: work the caller
 *             queued on the output buffers (a fill, an earlier use of the
 *             memory) must have finished before submit.  Host-checkable errors
 *             return at once; SSP_ERR_BUDGET if the request alone does not fit
 *             a slot.  Thread-safe.
 *  poll     : SSP_OK when done, SSP_ERR_NOT_READY while queued or running,
 *             the failure status otherwise, SSP_ERR_INVALID_ARG for an
 *             unknown ticket.
 *  wait     : as poll, blocking up to timeout_s seconds (< 0: no limit).
 *  destroy  : finishes every submitted request, then frees the slots.
 */
typedef struct ssp_server_s* ssp_server;

typedef struct {
    int32_t a, b;          /* registered matrix ids: C = A.B               */
    int32_t sampler;       /* ssp_sampler                                   */
    int32_t reserved;      /* 0                                             */
    double sample_rate;
    uint64_t seed;
    int64_t* nnz_pred;     /* device int64[rows of a], written              */
    ssp_stats* stats;      /* device ssp_stats or NULL                      */
} ssp_request;

typedef struct {
    uint64_t submitted, completed, batches, max_batch_seen, queued;
    uint64_t max_slots_busy; /* most slots running batches at once        */
    double elapsed_s;      /* since creation or the last reset             */
    double latency_p50_ms, latency_p99_ms, latency_mean_ms, latency_max_ms;
} ssp_server_stats;

SSP_API ssp_status ssp_server_create(ssp_handle h, int nslots, size_t slot_bytes, int max_batch,
                                     ssp_server* server);
SSP_API ssp_status ssp_server_register_matrix(ssp_server s, const ssp_csr* m, int32_t* id);
SSP_API ssp_status ssp_server_submit(ssp_server s, const ssp_request* r, uint64_t* ticket);
SSP_API ssp_status ssp_server_poll(ssp_server s, uint64_t ticket);
SSP_API ssp_status ssp_server_wait(ssp_server s, uint64_t ticket, double timeout_s);
SSP_API ssp_status ssp_server_info(ssp_server s, ssp_server_stats* out);
SSP_API ssp_status ssp_server_reset_stats(ssp_server s);
SSP_API ssp_status ssp_server_destroy(ssp_server s);

/*
 * Explicit CSR check (the compute entry points do not check contents):
 * counts the violations of rpt[0] = 0, rpt[i] <= rpt[i+1], rpt[nrows] = nnz
 * and 0 <= col < ncols, and writes the count to the device int64 *n_bad.
 */
SSP_API ssp_status ssp_validate_csr(ssp_handle h, const ssp_csr* M, int64_t* n_bad, void* stream);

/* ------------------------------------- the consumer: numeric product */

/*
 * Numeric C = A.B (float64 values) whose memory is sized by a per-row
 * capacity, normally the prediction: the output structure is predicted so
 * that C can be allocated, and the numeric phase balanced, without a symbolic
 * pass (Sec. I).  The paper stops at the prediction; this consumer is one way
 * to use it.  Two calls:
 *
 * ssp_spgemm_compute.  Row i of C gets a slot of
 *     s_i = min(N, c + ceil(c * margin_pct / 100)),  c = row_cap[i] clamped to [0, N],
 * in a slot area of S = sum(s_i) entries (12 bytes each) that the handle
 * allocates, and the rows share an overflow area of ceil(S * spill_pct / 100)
 * entries (12 bytes each, plus 24 bytes per record of where its runs go).
 * One numeric pass accumulates every row once (rows of at most 2048 products
 * in an LDS hash table, longer rows in a dense accumulator), counts its
 * nonzeros and writes the row, columns increasing, into its slot when it
 * fits.  A row with more nonzeros than its slot keeps them in the overflow
 * area while the area lasts: a row of more than 2048 products the entries
 * past its first s_i (B's rows sorted), a shorter row all of them when it
 * completes within half its hash table (with spill_pct > 0 a row's table is
 * sized for all its products, so the row does, unless the table sized by
 * its slot fits the one-wave kernel's 512 slots and a table for all its
 * products would not).  The other overflowing rows are recomputed.  C_rpt then receives
 * C's row offsets from the exact counts.  Waits for `stream` twice (the slot
 * area's size and the results are read on the host) and fills *info.
 *   A_val, B_val : device double[A.nnz], double[B.nnz]; duplicate entries add.
 *   row_cap      : device int64[A.nrows], any values (clamped as above).
 *   margin_pct   : 0 .. 10000.
 *   spill_pct    : 0 .. 10000 (0: no overflow area).
 *   C_rpt        : device int64[A.nrows + 1], written (C_rpt[0] = 0).
 *   info         : host, written.
 * Which overflowing rows the area holds depends on the order in which rows
 * finish when it runs short (spill_rows, spill_nnz); C does not.
 *
 * ssp_spgemm_copy.  Writes C_col / C_val (device, capacity >= info.nnz
 * entries, else SSP_ERR_INVALID_ARG): rows that fitted are copied from their
 * slots, rows held in the overflow area from their slot and the area, the
 * other rows with more nonzeros than their slot (an under-prediction) are
 * recomputed straight into their final place.  Asynchronous on `stream`.  A,
 * B and their values must be unchanged since the compute call; the next
 * compute call on the handle waits for this copy and replaces its state.
 *
 * C keeps every structural entry (terms that cancel leave an explicit 0.0):
 * C's structure is exactly the structure the prediction estimates
 * (ssp_exact_structure).  Values are sums of the products in an unspecified
 * order.  Errors: those of the other calls; SSP_ERR_BUDGET when the slot area,
 * the overflow area and the accumulators exceed the handle's budget.
 */
typedef struct {
    int64_t nnz;           /* NNZ(C)                                                */
    int64_t total_flop;    /* F                                                     */
    int64_t slot_entries;  /* sum of the slot sizes s_i                             */
    int64_t overflow_rows; /* rows with more nonzeros than their slot               */
    int64_t overflow_nnz;  /* their nonzeros                                        */
    int64_t slot_bytes;    /* bytes of the slot area                                */
    int64_t spill_rows;    /* overflowing rows the overflow area holds (the rest of
                              the overflowing rows are recomputed by ssp_spgemm_copy) */
    int64_t spill_nnz;     /* their nonzeros held in the area                       */
    int64_t spill_bytes;   /* bytes of the overflow area and its records            */
} ssp_spgemm_info;

SSP_API ssp_status ssp_spgemm_compute(ssp_handle h, const ssp_csr* A, const double* A_val,
                                      const ssp_csr* B, const double* B_val,
                                      const int64_t* row_cap, int32_t margin_pct,
                                      int32_t spill_pct, int64_t* C_rpt,
                                      ssp_spgemm_info* info, void* stream);
SSP_API ssp_status ssp_spgemm_copy(ssp_handle h, int32_t* C_col, double* C_val,
                                   int64_t capacity, void* stream);

/* ----------------------- the existing sampling estimator (related work) */

/*
 * Amossen et al.'s k-minimum-values estimate of NNZ(C) with BHash's sampling
 * (Sec. III), the comparison the paper's reference design stands for: rows of
 * A and columns of B are each kept with probability `sample_rate`, every
 * intermediate product (i, j) of C' = A'B' is hashed to [0, 1), the k-th
 * smallest distinct hashed value v gives NNZ(C') = k / v, and
 * NNZ(C) = NNZ(C') / (p_r p_c) with the realised proportions p_r = rows kept / M,
 * p_c = columns kept / N (the paper's p^2).  Definitions (splitmix64 as for the
 * row sampler, T = floor(sample_rate * 2^53)):
 *   row i kept     iff (splitmix64(seed,     i) >> 11) < T
 *   column j kept  iff (splitmix64(seed + 1, j) >> 11) < T
 *   hash of (i, j) = (splitmix64(seed + 2, i * N + j) >> 11) / 2^53.
 * With fewer than k distinct values the sample's NNZ is their number (exact).
 * Synchronous: waits for `stream`, fills *out (host).  k in 1 .. 4096.
 */
typedef struct {
    uint64_t rows_kept;     /* rows of A'                                        */
    uint64_t cols_kept;     /* columns of B'                                     */
    uint64_t products;      /* intermediate products of C' = A'B'                */
    uint64_t distinct_kept; /* distinct hashes below the final threshold         */
    uint64_t kth_hash;      /* k-th smallest distinct 53-bit hash, 0 if < k      */
    uint64_t k;
    uint64_t threshold;     /* the final threshold on the 53-bit hashes          */
    double nnz_sample;      /* NNZ(C') estimate: k / v, or the distinct count    */
    double nnz_estimate;    /* NNZ(C) estimate; -1 when no row or column is kept */
} ssp_kmv_result;

SSP_API ssp_status ssp_kmv_estimate(ssp_handle h, const ssp_csr* A, const ssp_csr* B,
                                    double sample_rate, uint32_t k, uint64_t seed,
                                    ssp_kmv_result* out, void* stream);

/* ------------------------------------------------ diagnostics, strings */

/* Per-phase device timing.  While enabled, every phase a call enqueues is
 * bracketed by two hipEvents on the call's stream.  Phases: "tiles" (the
 * merge-path tile partition), "flop" (the streaming row-FLOP kernel alone),
 * "flop_fixup" (rows spanning tiles, F), "sample_bin" (sampling and
 * binning), "sym_bins" (distinct counts of short and medium rows), "sym_long"
 * (the long-row kernel alone), "sym_merge" (OR of split rows' parts),
 * "finalize" (z* or the exact total, the divisor of f*, and the reference
 * design's constants), "pred_rows" and
 * "ref_rows" (the per-row outputs); for the numeric product "num_scan" (slot
 * and row offsets), "num_hash" and "num_dense" (the numeric pass by bin),
 * "num_copy" and "num_fallback" (the copy call).  ssp_timing_read waits for the recorded
 * events, writes up to `max` aggregated entries (one per phase seen) and
 * clears them; it returns the number written, -1 on a bad argument.  Timing
 * serialises nothing but adds two event records per phase. */
typedef struct {
    char name[24];
    uint64_t launches;
    double total_ms;
} ssp_phase_time;

SSP_API ssp_status ssp_timing_enable(ssp_handle h, int enable);
SSP_API int ssp_timing_read(ssp_handle h, ssp_phase_time* out, int max);

SSP_API const char* ssp_status_string(ssp_status s);
/* Message of the last failing HIP call made through this handle ("" if none). */
SSP_API const char* ssp_last_error(ssp_handle h);
/* Library version string. */
SSP_API const char* ssp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SSP_H */
