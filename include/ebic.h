/*
 * ebic.h -- C ABI of the EBIC fitness evaluation on MI355X (gfx950).
 *
 * EBIC (Orzechowski & Moore, "EBIC: an open source software for
 * high-dimensional and big data biclustering analyses") is an evolutionary
 * biclustering method whose search is driven by counting rows (Methods,
 * "Handling missing values"). An individual of its population is an ordered
 * list of column indices c_0 .. c_{k-1}. A row supports the individual when
 * its values along that order stand in the greater-or-equal relation:
 *
 *   P(row) = AND_{j=1..k-1} X[row, c_j] >= X[row, c_{j-1}]   (positive trend)
 *   N(row) = AND_{j=1..k-1} X[row, c_j] <= X[row, c_{j-1}]   (negative trend,
 *                                                  only with EBIC_NEG_TRENDS)
 *   matched  = #rows with P or N
 *   negative = #rows with N and not P  (a row on both trends -- constant along
 *                                       the individual -- counts as positive)
 *
 * Comparisons are IEEE-754 single precision, ordered, exact: -0 == +0,
 * denormals are ordinary values, +-inf are ordinary values, NaN is missing.
 *
 * Missing values (Methods, "Handling missing values"), two modes:
 *   EBIC_NAN_EXCLUDE: a row with a missing value in any of the individual's
 *                     columns is not counted.
 *   EBIC_NAN_INCLUDE: the legacy behaviour; a missing value takes the
 *                     matrix's fill value and joins the ordinary comparison.
 * A cell is missing when it is NaN, or, if a sentinel was given at upload,
 * when it compares equal to that sentinel (the paper's "predefined value",
 * e.g. 0 or 999).
 *
 * Rows: up to 2^31-1 per matrix on one GPU (Methods, "Support for Big
 * Data"); there is no cap on the population size beyond int32.
 *
 * Conventions shared by every call:
 *   - Every function returns an ebic_status (0 = EBIC_OK, < 0 = error) except
 *     ebic_last_error and ebic_mask_words. On error, ebic_last_error() returns
 *     a message (thread-local, valid until the calling thread's next call).
 *     No C++ exception crosses this boundary.
 *   - Host-checkable errors (NULL required pointer, unknown handle, bad
 *     flags, bad sizes) return before anything is enqueued.
 *   - `hip_stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Device pointers (d_*) are caller-owned device memory of the context's
 *     device; they are borrowed until the work enqueued on `hip_stream`
 *     completes.
 *   - The context is thread-safe. Evaluations on different streams may run
 *     concurrently; matrix upload and release are serialised internally.
 */
#ifndef EBIC_H
#define EBIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ebic_ctx ebic_ctx;  /* opaque; one per HIP device */
typedef int32_t ebic_status;

enum {
    EBIC_OK = 0,
    EBIC_EINVAL = -1,   /* bad argument */
    EBIC_ENOMEM = -2,   /* device or host allocation failed */
    EBIC_EHIP = -3,     /* a HIP runtime call failed */
    EBIC_ENOENT = -4,   /* unknown matrix handle */
    EBIC_EBUSY = -5,    /* resource in use */
    EBIC_EBUDGET = -6,  /* request exceeds a memory budget */
    EBIC_ECANCELED = -7 /* a serving request was cancelled before it ran */
};

/* Evaluation flags. */
#define EBIC_NAN_EXCLUDE 0u   /* bit 0 clear: exclude rows with missing values */
#define EBIC_NAN_INCLUDE 1u   /* bit 0 set: missing values take the fill value */
#define EBIC_NEG_TRENDS 2u    /* also count rows on the reversed (<=) chain */

/* Upload-only flags. */
#define EBIC_SRC_DEVICE 4u       /* `src` is device memory (default: host) */
#define EBIC_SRC_COL_MAJOR 8u    /* `src` is column-major (default: row-major) */
#define EBIC_KEEP_FILL_COPY 16u  /* also keep a fill-substituted copy resident */

/* Create a context on HIP device `hip_device`. *out receives the handle. */
ebic_status ebic_create(int32_t hip_device, ebic_ctx **out);

/* Wait for the device, free every resident matrix and the context. */
ebic_status ebic_destroy(ebic_ctx *ctx);

/*
 * Route the library's device allocations (resident matrices, descriptor
 * tables) through `alloc`/`release` (e.g. a framework's caching allocator).
 * `alloc(bytes, user)` returns device memory of the context's device aligned
 * to at least 256 bytes, or NULL. Pass NULLs to restore hipMalloc/hipFree.
 * Only allowed while no matrix is resident (else EBIC_EBUSY).
 */
ebic_status ebic_set_allocator(ebic_ctx *ctx, void *(*alloc)(size_t bytes, void *user),
                               void (*release)(void *ptr, void *user), void *user);

/* Message of the calling thread's last failed call ("" if none). */
const char *ebic_last_error(void);

/*
 * Make a matrix resident on the device (rows x cols, FP32).
 *   src:      host (default) or device (EBIC_SRC_DEVICE) memory; row-major
 *             with row stride ld_src >= cols (default) or column-major with
 *             column stride ld_src >= rows (EBIC_SRC_COL_MAJOR), in elements.
 *   rows:     1 .. 2^31-1.       cols: >= 1.
 *   flags:    EBIC_SRC_DEVICE | EBIC_SRC_COL_MAJOR | EBIC_KEEP_FILL_COPY.
 *   missing_sentinel: cells equal (IEEE ==) to it become missing; NaN = none.
 *   missing_fill:     value a missing cell takes in EBIC_NAN_INCLUDE mode;
 *                     must not be NaN.
 *   out_matrix: receives a handle (>= 0).
 * The resident copy is column-major with a leading dimension padded to a
 * multiple of 64 rows (missing cells stored as NaN). A matrix of at most 384
 * columns also keeps its rank codes (per cell, the number of smaller cells
 * of its row, as FP16; half the bytes of the values, and of the fill copy
 * if kept), which stage twice the rows in LDS and compare exactly as the
 * values do. A matrix of at most 128 columns also keeps byte rank codes of
 * its fill-substituted values (one byte per cell, rows padded to a multiple
 * of 256), which let one 32-bit lane word hold four rows; exclude mode uses
 * them only if the matrix has no missing cell. Returns after the copy has
 * completed on `hip_stream`.
 */
ebic_status ebic_upload_matrix(ebic_ctx *ctx, const float *src, int64_t rows, int32_t cols,
                               int64_t ld_src, uint32_t flags, float missing_sentinel,
                               float missing_fill, void *hip_stream, int32_t *out_matrix);

/* Shape and resident bytes of a matrix. Any output pointer may be NULL. */
ebic_status ebic_matrix_info(ebic_ctx *ctx, int32_t matrix, int64_t *rows, int32_t *cols,
                             int64_t *device_bytes);

/* Code sets a resident matrix may hold (ebic_matrix_stats.code_sets, from ebic_matrix_get_stats). */
enum {
    EBIC_SET_FILL_COPY = 1u,   /* FP32 copy with missing cells replaced by the fill */
    EBIC_SET_FP16 = 2u,        /* FP16 rank codes of the values (missing = NaN) */
    EBIC_SET_FP16_FILL = 4u,   /* FP16 rank codes of the fill copy */
    EBIC_SET_U8 = 8u,          /* byte rank codes of the fill-substituted values */
    EBIC_SET_U16 = 16u,        /* 16-bit rank codes of the fill-substituted values */
    EBIC_SET_U10 = 32u,        /* 10-bit rank codes (three per 32-bit word) of the same */
    EBIC_SET_PAIRS = 64u,      /* pairwise order bitmaps of the values */
    EBIC_SET_PAIRS_FILL = 128u /* pairwise order bitmaps of the fill-substituted values */
};

/*
 * What a resident matrix holds and what its upload cost (for reports and
 * tests; the values are stated as of this call).
 *   value_bytes:     the FP32 matrix, plus its fill copy if kept.
 *   code_bytes:      every rank-code set resident now, with its flags.
 *   swar_chunks:     512-row chunks of the byte or 16-bit codes (0 without).
 *   swar_tie_chunks: of those, the chunks in which some row holds two equal
 *                    (code-equal) cells; the evaluation runs the first
 *                    pair's tie handling only on these.
 *   has_missing:     1 if a cell is missing, 0 if none, -1 if not known
 *                    (no SWAR code set was built).
 *   upload_ms:       host wall time of the ebic_upload_matrix call.
 * Copies a few bytes per 512 rows back from the device (synchronous).
 */
typedef struct {
    int64_t rows;
    int32_t cols;
    uint32_t code_sets;        /* EBIC_SET_* */
    int64_t value_bytes;
    int64_t code_bytes;
    int64_t swar_chunks;
    int64_t swar_tie_chunks;
    int32_t has_missing;
    int32_t reserved;
    double upload_ms;
} ebic_matrix_stats;
ebic_status ebic_matrix_get_stats(ebic_ctx *ctx, int32_t matrix, ebic_matrix_stats *out);

/*
 * Free a resident matrix. Waits for the device to finish the work already
 * enqueued. Returns EBIC_EBUSY, freeing nothing, while a call on another
 * thread is between reading the matrix and enqueuing its kernels, or while
 * a serving engine holds requests on it that have not completed.
 */
ebic_status ebic_release_matrix(ebic_ctx *ctx, int32_t matrix);

/* Number of uint64 mask words per individual: ceil(rows / 64). */
int64_t ebic_mask_words(int64_t rows);

/*
 * Evaluate one population against a resident matrix (the fitness evaluation
 * of one EBIC generation; Methods, "Handling missing values" and "Support
 * for Big Data").
 *   n_ind:     number of individuals (0 is a valid no-op).
 *   d_offsets: int32[n_ind + 1], non-decreasing; individual i is
 *              d_cols[d_offsets[i] .. d_offsets[i+1]).
 *   d_cols:    int32[d_offsets[n_ind]] column indices.
 *   flags:     EBIC_NAN_EXCLUDE or EBIC_NAN_INCLUDE, | EBIC_NEG_TRENDS.
 *   d_matched:       int32[n_ind] (required).
 *   d_negative:      int32[n_ind] or NULL.
 *   d_matched_mask:  uint64[n_ind * ebic_mask_words(rows)] or NULL; bit
 *                    (r % 64) of word (r / 64) of individual i's row is set
 *                    when row r is matched. Bits past `rows` are 0.
 *   d_negative_mask: same layout for the negative-trend rows, or NULL.
 * Outputs are fully overwritten. An individual of length < 1 or with a
 * column outside [0, cols) gets matched = negative = -1 and zero mask words;
 * the call still returns EBIC_OK. Asynchronous on `hip_stream`.
 */
ebic_status ebic_eval_population(ebic_ctx *ctx, int32_t matrix, int32_t n_ind,
                                 const int32_t *d_offsets, const int32_t *d_cols,
                                 uint32_t flags, int32_t *d_matched, int32_t *d_negative,
                                 uint64_t *d_matched_mask, uint64_t *d_negative_mask,
                                 void *hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * evaluation as ebic_eval_population, with the same arguments, outputs and
 * errors, that allocates nothing. It calls no hipMalloc or hipFree and no
 * allocator hook; the per-individual headers that ebic_eval_population keeps
 * in stream scratch go to a fixed device buffer instead, which each device
 * holds from ebic_create until the process ends.
 *   Limit: n_ind <= 65,536 (4 MiB of 64-byte headers per device); a larger
 *   population returns EBIC_EINVAL and enqueues nothing.
 *   Sharing: every call on one device uses the same buffer, and it keeps
 *   the last call's headers (the prep kernel rewrites every header a call
 *   reads, so nothing has to start at zero). Calls in order on one stream
 *   are safe; calls that overlap on one device (other streams, other
 *   threads, other contexts) race on the buffer and must be serialised by
 *   the caller.
 *   No profiling events are recorded for these launches.
 */
ebic_status ebic_eval_population_noalloc(ebic_ctx *ctx, int32_t matrix, int32_t n_ind,
                                         const int32_t *d_offsets, const int32_t *d_cols, uint32_t flags,
                                         int32_t *d_matched, int32_t *d_negative,
                                         uint64_t *d_matched_mask, uint64_t *d_negative_mask,
                                         void *hip_stream);

/* One population-evaluation request of a batch (same meaning as above). */
typedef struct ebic_request {
    int32_t matrix;
    int32_t n_ind;
    const int32_t *d_offsets;
    const int32_t *d_cols;
    uint32_t flags;
    int32_t *d_matched;
    int32_t *d_negative;
    uint64_t *d_matched_mask;
    uint64_t *d_negative_mask;
} ebic_request;

/*
 * Evaluate many populations -- of uneven sizes, with individuals of uneven
 * lengths, from many concurrent EBIC runs, over one or several resident
 * matrices -- in one replay of a captured HIP graph: requests on matrices
 * that take the pair bitmaps (staging 6, built here on first use) in one
 * fixed-grid kernel, the others in one persistent tiled kernel. Each
 * request's outputs equal those of ebic_eval_population on the same inputs.
 * `reqs` is a host array of n_reqs entries (read before the call returns).
 * Asynchronous on `hip_stream`.
 */
ebic_status ebic_eval_batch(ebic_ctx *ctx, const ebic_request *reqs, int32_t n_reqs,
                            void *hip_stream);

/*
 * Time the candidate launch shapes on `sample` (a representative batch whose
 * outputs are overwritten) and store the fastest for the sample's shape class
 * in the context; if cache_path is not NULL, also merge it into that JSON
 * file, which later contexts read at creation when EBIC_TUNE_CACHE names it.
 * Synchronises the device.
 */
ebic_status ebic_autotune(ebic_ctx *ctx, const ebic_request *sample, int32_t n_reqs,
                          const char *cache_path);

/*
 * Force the launch shape of later evaluations on this context (tests and
 * tuning experiments); waves_per_block = 0 restores the automatic choice.
 *   tiles_per_wave:        64-row tiles one wave evaluates together (1, 2, 4;
 *                          3 or 6 with the 10-bit codes; 8 or 16 with the
 *                          byte codes, 16 for counts only)
 *   waves_per_block:       1 .. 16
 *   individuals_per_group: individuals that share one block's staged tiles
 *   staging:               0 = column tiles staged in LDS, 1 = direct reads,
 *                          2 = the rank codes staged in LDS (2 or 4 sub-tiles;
 *                              include mode needs EBIC_KEEP_FILL_COPY),
 *                          3 = the byte rank codes staged in LDS (4, 8 or 16
 *                              sub-tiles; matrices of at most 128 columns;
 *                              exclude mode needs a matrix without missing
 *                              cells),
 *                          4 = the 16-bit rank codes staged in LDS (2 or 4
 *                              sub-tiles; 129 .. 384 columns; the same
 *                              condition for exclude mode),
 *                          5 = the 10-bit rank codes staged in LDS (3 or 6
 *                              sub-tiles; 129 .. 512 columns; the same
 *                              condition); 3, 4 and 5 select whichever kind
 *                              the matrix has when it lacks the one asked
 *                              for; without codes for the request's mode the
 *                              launch takes another staging. Batches stage
 *                              byte codes at 4 sub-tiles, 10-bit codes at 3
 *                              and 16-bit codes at 2.
 *                          6 = the pairwise order bitmaps (one bit per row
 *                              for every ordered pair of columns, built on
 *                              first use: cols^2 x ceil(rows / 2048) x 256
 *                              bytes plus 512 bytes per 2,048 rows, at most
 *                              1,024 columns, 1,073,725,440 rows and 32
 *                              GiB); nothing staged,
 *                              tiles_per_wave and blocks ignored, at most
 *                              64 individuals per wave (individuals_per_group
 *                              0 with a shape of this staging: chosen from
 *                              the work); without them (too large, or the
 *                              allocation-free entry point before they are
 *                              built) the launch takes the rank codes the
 *                              matrix has.
 *   blocks:                grid size per group, 0 = from occupancy
 * Shapes that do not fit the device are reduced at launch (fewer tiles per
 * wave, then direct reads). Results never depend on the shape.
 */
ebic_status ebic_set_launch_shape(ebic_ctx *ctx, int32_t tiles_per_wave, int32_t waves_per_block,
                                  int32_t individuals_per_group, int32_t staging, int32_t blocks);

/*
 * The launch shape an evaluation of n_ind individuals (nnz columns in all,
 * or -1 if unknown) on `matrix` would use now: the forced shape if one is
 * set, else the tuned one for its shape class, else the default, reduced to
 * what the device fits. Any output may be NULL. Staging: 0 = LDS, 1 = direct,
 * 2 = rank codes in LDS, 3 = byte rank codes in LDS, 4 = 16-bit rank codes in
 * LDS, 5 = 10-bit rank codes in LDS, 6 = the pair bitmaps (the staging
 * planned for exclude mode; for staging 6, blocks reports the 2,048-row
 * chunks).
 */
ebic_status ebic_plan_shape(ebic_ctx *ctx, int32_t matrix, int32_t n_ind, int64_t nnz,
                            int32_t *tiles_per_wave, int32_t *waves_per_block,
                            int32_t *individuals_per_group, int32_t *staging, int32_t *blocks);

/*
 * The launch shape ebic_eval_batch would use now for `reqs` (the same
 * validation, no launch): tiles per wave, waves per block, individuals per
 * group, the grid size, and, if `stagings` is not NULL, the staging of each
 * request (n_reqs entries, numbered as for ebic_plan_shape). The shape is
 * the tiled kernel's when any request is on it, else the pairs kernel's.
 * Any output may be NULL.
 */
ebic_status ebic_plan_batch_shape(ebic_ctx *ctx, const ebic_request *reqs, int32_t n_reqs,
                                  int32_t *tiles_per_wave, int32_t *waves_per_block,
                                  int32_t *individuals_per_group, int32_t *stagings,
                                  int32_t *blocks);

/*
 * Measurement diagnostics. `mode` bit 0: record a HIP event pair on the
 * caller's stream around every evaluation kernel this context launches;
 * bit 1: count executed predicate steps (one step = one column of one
 * individual compared on one 64-row tile), using a counting variant of the
 * kernel that is slower and meant for an untimed run. 0 turns both off.
 */
ebic_status ebic_set_profiling(ebic_ctx *ctx, int32_t mode);

/*
 * Synchronise the device, then report what was recorded since the previous
 * read and reset it: evaluation kernels timed, their summed duration in
 * milliseconds, and executed predicate steps. Any output may be NULL.
 */
ebic_status ebic_read_profile(ebic_ctx *ctx, int64_t *launches, double *kernel_ms,
                              int64_t *executed_steps);

/* ------------------------------------------------------------------------
 * Serving: evaluations submitted by many concurrent EBIC runs (each run's
 * evolutionary loop on the host asks for the counts of one population per
 * generation, EBIC paper, Introduction and Methods), batched continuously
 * onto one GPU. Host buffers in, host buffers out.
 * ------------------------------------------------------------------------ */
typedef struct ebic_server ebic_server;

typedef struct ebic_server_stats {
    int64_t submitted;        /* requests accepted (after the last reset) */
    int64_t completed;        /* requests completed */
    int64_t batches;          /* batched launches */
    int64_t pending;          /* requests waiting for a slot or memory */
    int64_t reserved_bytes;   /* device bytes held by batches in flight */
    int64_t high_water_bytes; /* largest reserved_bytes seen */
    int64_t budget_bytes;     /* the HBM budget */
    int64_t nominal_checks;   /* rows x sum of lengths over completed requests */
    double latency_p50_ms;    /* submission to completion */
    double latency_p99_ms;
    double mean_batch;        /* requests per batched launch */
    double latency_max_ms;
    int64_t graph_captures;   /* batch graphs the context has captured in all */
    int64_t staging_grows;    /* pinned staging buffers enlarged */
    double queue_p99_ms;      /* submission to the enqueue of the request's batch */
    int64_t cancelled;        /* requests cancelled before they ran */
} ebic_server_stats;

/*
 * Device bytes one request holds while in flight (its CSR and outputs,
 * 256-byte aligned): the quantity admission compares with the budget.
 * masks != 0: both mask arrays (the negative one only with
 * EBIC_NEG_TRENDS) are returned.
 */
ebic_status ebic_server_request_bytes(ebic_ctx *ctx, int32_t matrix, int32_t n_ind, int64_t nnz,
                                      uint32_t flags, int32_t masks, int64_t *out_bytes);

/*
 * Start a server on `ctx`: a device arena of hbm_budget_bytes (from the
 * context's allocator; it bounds the bytes of all batches in flight),
 * `slots` streams (1..16, each with a pinned staging buffer and a completion
 * thread) and a scheduler thread that launches waiting requests, in
 * arrival order, as one ebic_eval_batch per idle slot: at most max_batch of
 * them, and at most an equal share (rounded up) of those waiting per idle
 * slot, so that a backlog is spread over the idle slots. The matrices stay owned by the
 * context and must outlive the requests that use them.
 */
ebic_status ebic_server_create(ebic_ctx *ctx, int64_t hbm_budget_bytes, int32_t slots,
                               int32_t max_batch, ebic_server **out);

/*
 * Complete every submitted request (their outputs are written), stop the
 * threads and free the server's memory. Tags not yet polled are dropped.
 */
ebic_status ebic_server_destroy(ebic_server *srv);

/*
 * Queue one population evaluation. offsets (n_ind + 1 entries) and cols
 * (max(offsets) entries) are host arrays, copied before the call returns.
 * matched (n_ind), negative (n_ind, or NULL), matched_mask and
 * negative_mask (n_ind * ebic_mask_words(rows) words each, or NULL; the
 * negative mask needs `negative`) are host buffers that the server writes
 * when the request completes: they must stay valid until ebic_server_poll
 * returns `tag`. flags: EBIC_NAN_INCLUDE, EBIC_NEG_TRENDS. Results equal
 * those of ebic_eval_population on the same inputs. From submission until
 * the request completes (or is cancelled) it holds its matrix:
 * ebic_release_matrix returns EBIC_EBUSY meanwhile. Errors: EBIC_EINVAL
 * (arguments, negative offsets), EBIC_ENOENT (unknown matrix), EBIC_EBUDGET
 * (the request alone exceeds the budget), EBIC_EBUSY (shutting down).
 */
ebic_status ebic_server_submit(ebic_server *srv, int32_t matrix, int32_t n_ind,
                               const int32_t *offsets, const int32_t *cols, uint32_t flags,
                               int32_t *matched, int32_t *negative, uint64_t *matched_mask,
                               uint64_t *negative_mask, uint64_t tag);

/*
 * Wait up to timeout_us microseconds for completed requests and return up to
 * max_tags of their tags (and, if `statuses` is not NULL, each request's
 * status: EBIC_OK, or the error of its batch's launch) in completion order.
 */
ebic_status ebic_server_poll(ebic_server *srv, uint64_t *tags, ebic_status *statuses,
                             int32_t max_tags, int32_t timeout_us, int32_t *n_done);

/*
 * Cancel a request that has not been launched yet: it leaves the queue, its
 * outputs are not written, it releases its matrix, and ebic_server_poll
 * returns its tag with status EBIC_ECANCELED. Returns EBIC_EBUSY if the
 * request's batch is already on the device (it will complete normally) and
 * EBIC_ENOENT if no submitted, uncompleted request has this tag.
 */
ebic_status ebic_server_cancel(ebic_server *srv, uint64_t tag);

/*
 * paused != 0: launch no new batch (submissions still queue; batches on the
 * device complete); 0: resume. For draining and for deterministic tests.
 */
ebic_status ebic_server_set_paused(ebic_server *srv, int32_t paused);

/* Counters and latency percentiles; reset != 0 starts a new window. */
ebic_status ebic_server_get_stats(ebic_server *srv, ebic_server_stats *out, int32_t reset);

/* ------------------------------------------------------------------------
 * A stand-in evolutionary driver (host code). The paper gives EBIC's search
 * only as evolutionary and driven by row counts (Introduction; Methods,
 * "Handling missing values"), not its operators or fitness formula, so these
 * are a stand-in of the same shape: tournament selection with elitism on
 * fitness = matched * 2^(k-2) (invalid individuals last), one-point
 * crossover, and one mutation (insert, delete, swap or substitute a column).
 * Every random choice comes from SplitMix64 seeded with `seed`, so a run is
 * a function of its parameters and the counts it is given.
 * ------------------------------------------------------------------------ */
typedef struct ebic_ea ebic_ea;

typedef struct ebic_ea_params {
    int32_t n_cols;      /* columns of the matrix the individuals index */
    int32_t pop_size;    /* individuals per generation (>= 2) */
    int32_t k_min;       /* individual length bounds, 1 <= k_min <= k_max <= n_cols */
    int32_t k_max;
    int32_t elite;       /* best individuals carried over unchanged, [0, pop_size) */
    double p_crossover;  /* probability that a child comes from crossover */
    double p_mutation;   /* probability that a child is mutated once */
    uint64_t seed;
} ebic_ea_params;

/* A driver with a random first generation (distinct columns per individual). */
ebic_status ebic_ea_create(const ebic_ea_params *params, ebic_ea **out);

ebic_status ebic_ea_destroy(ebic_ea *ea);

/*
 * The current generation as host CSR (pop_size + 1 offsets, then the
 * columns), owned by the driver and valid until the next ebic_ea_step or
 * ebic_ea_destroy; any output may be NULL.
 */
ebic_status ebic_ea_population(ebic_ea *ea, const int32_t **offsets, const int32_t **cols,
                               int32_t *n_ind, int64_t *generation);

/*
 * Score the current generation from its matched counts (pop_size entries,
 * as returned by an evaluation of the CSR above; -1 marks an invalid
 * individual), report its best individual, and replace it by the next
 * generation.
 */
ebic_status ebic_ea_step(ebic_ea *ea, const int32_t *matched, int32_t *best_index,
                         double *best_fitness);

/*
 * The same breeding on the device: the generation after (d_offsets,
 * d_cols), a population of n_ind = params->pop_size individuals in device
 * memory, from its matched counts d_matched (n_ind, device; -1 marks an
 * invalid individual), written as CSR to d_next_offsets (n_ind + 1) and
 * d_next_cols (capacity n_ind * k_max int32), all device memory of the
 * context's device, caller-owned and borrowed until the stream work
 * completes. `generation` is the index of the generation being bred (>= 1;
 * generation 0 is the driver's random first one): with the driver's
 * parameters and the same counts, generation g equals what the g-th
 * ebic_ea_step produces, column for column. d_best (nullable, device)
 * receives the index of the current generation's best individual.
 * Asynchronous on hip_stream (evaluation and breeding can alternate on one
 * stream without the population leaving the device); the input and output
 * populations must not overlap. A parent longer than k_max is read as its
 * first k_max columns; a parent without columns is replaced by a random
 * individual. Errors: EBIC_EINVAL (parameters as for ebic_ea_create,
 * n_ind != pop_size, generation < 1, a NULL required pointer), EBIC_ENOMEM,
 * EBIC_EHIP; nothing is enqueued on error.
 */
ebic_status ebic_ea_breed(ebic_ctx *ctx, const ebic_ea_params *params, int64_t generation, int32_t n_ind,
                          const int32_t *d_offsets, const int32_t *d_cols, const int32_t *d_matched,
                          int32_t *d_next_offsets, int32_t *d_next_cols, int32_t *d_best,
                          void *hip_stream);

/* ------------------------------------------------------------------------
 * Ingest and export (host code).
 * ------------------------------------------------------------------------ */
typedef struct ebic_text_matrix {
    int64_t rows;
    int32_t cols;
    char delimiter;     /* the one used (given or detected) */
    float *values;      /* column-major: values[c * rows + r]; missing = NaN */
    char **row_names;   /* rows entries, or NULL when the file has none */
    char **col_names;   /* cols entries, or NULL when the file has no header */
} ebic_text_matrix;

/*
 * Read a delimited text matrix, genes in rows and samples in columns (EBIC
 * paper, Methods, "Different input file formats support"): values separated
 * by ',', '\t' or ';' (delimiter 0: the one of those most frequent on the
 * first line); an optional header row (header -1: detected, a non-numeric
 * field past the first; 0: none; 1: present) whose upper-left cell may be
 * absent; optional row names in the first field (row_names -1: detected,
 * 0, 1). Empty fields and NA, NaN, nan, na, ? are missing (NaN); other
 * fields are decimal numbers, read as double and rounded to float. Blank
 * lines are skipped; CR LF is accepted. `threads` (>= 1) parse lines in
 * parallel. The result is ready for ebic_upload_matrix(src = values,
 * ld_src = rows, flags = EBIC_SRC_COL_MAJOR); free it with
 * ebic_free_text_matrix. Errors: EBIC_ENOENT (cannot open), EBIC_EINVAL
 * (ragged lines, non-numeric values, with the line and field in
 * ebic_last_error()).
 */
ebic_status ebic_read_delimited(const char *path, char delimiter, int32_t header,
                                int32_t row_names, int32_t threads, ebic_text_matrix *out);

/* Free what ebic_read_delimited allocated and zero the struct. */
ebic_status ebic_free_text_matrix(ebic_text_matrix *m);

/*
 * Write the biclusters of the chosen individuals (EBIC paper, Methods,
 * "Compatibility with R and Bioconductor") as text: a comment line, then
 * per bicluster three tab-separated lines,
 *   bicluster <b> <number of rows> <number of columns>
 *   rows <row> <row> ...      (the set bits of its matched mask)
 *   cols <col> <col> ...      (its columns in the individual's order)
 * with 1-based indices, or the names when row_names / col_names are given.
 *   offsets, cols: the population's host CSR (n_ind individuals).
 *   matched_mask:  host copy of the evaluation's matched mask,
 *                  n_ind x ebic_mask_words(rows) words.
 *   which:         n_out individual indices in [0, n_ind).
 */
ebic_status ebic_write_biclusters(const char *path, int64_t rows, int32_t n_ind,
                                  const int32_t *offsets, const int32_t *cols,
                                  const uint64_t *matched_mask, int32_t n_out,
                                  const int32_t *which, const char *const *row_names,
                                  const char *const *col_names);

#ifdef __cplusplus
}
#endif

#endif /* EBIC_H */
