/*
 * repro.h -- C interface of librepro: reproducible GroupBy-SUM over
 * floating-point columns into the accumulator type repro<T,L> on AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Mueller, Arteaga, Hoefler, Alonso, "Reproducible Floating-Point
 * Aggregation in RDBMSs" (arXiv 1802.09883).  The problem statement is
 * Sec. II-A (GroupBy turns <key,value> pairs into <key,aggregate> pairs; the
 * aggregate must have the same bits for every execution); the accumulator is
 * the repro<ScalarT,L> type of Sec. IV, built on RSum (Sec. III-C, Alg. 2)
 * with its operator+=(ScalarT), operator+=(repro), resumable state and the
 * finalisation equation of Sec. III-C.
 *
 * Conventions for every entry point:
 *   - All buffers are DEVICE pointers owned by the caller (except the job
 *     and plan records of the batch calls, which live in host memory).  The
 *     library allocates no device memory; scratch memory is the caller's
 *     `workspace`.
 *   - Work is enqueued asynchronously on `stream` (0 = the null stream);
 *     results are visible after the stream is synchronised.
 *   - Host return value: REPRO_OK, or REPRO_EINVAL for invalid arguments
 *     (checked synchronously; nothing is enqueued), or REPRO_EHIP when a
 *     kernel launch fails.
 *   - Calls on different streams are independent; calls that touch the same
 *     states or workspace must be ordered by the caller.
 *
 * Accumulator formats (paper: W = 18 for float, 40 for double; m = fraction
 * bits; extractor exponents on the fixed lattice E_j = B + j*W, B = emin):
 *   T = double: m = 52, W = 40, B = -1022, top index j in [L-1, 51],
 *               value domain |b| < 2^1005.
 *   T = float:  m = 23, W = 18, B = -126,  top index j in [L-1, 14],
 *               value domain |b| < 2^120.
 *
 * State layout (num_groups = G), "canonical" at every call boundary:
 *   S[l][g]  : T,       l = 0..L-1 (level 0 = first, largest level),
 *                       S in [1.5, 1.75) * 2^E_l with E_l = E_top - l*W;
 *   C[l][g]  : int64_t, the carry-bit counts, starting at the next
 *                       multiple of 8 bytes after the S block.
 * The exact value of level l is (S - 1.5*2^E_l) + 0.25*2^E_l*C (Sec. III-C).
 * An empty group has E_top = E_{L-1} and all C = 0.  Canonical states are
 * unique, so two states can be compared bit for bit.
 */
#ifndef REPRO_H
#define REPRO_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* host-side return codes */
typedef enum { REPRO_OK = 0, REPRO_EINVAL = -1, REPRO_EHIP = -2 } repro_status_t;

/* device status bits, OR-ed into the caller's status word */
enum {
    REPRO_ERR_KEY = 1u,       /* key outside [0, num_groups): row skipped      */
    REPRO_ERR_NONFINITE = 2u, /* NaN or +-Inf value: row skipped              */
    REPRO_ERR_RANGE = 4u      /* |value| beyond the domain of T: row skipped   */
};

typedef enum { REPRO_F32 = 0, REPRO_F64 = 1 } repro_scalar_t;
typedef enum { REPRO_I32 = 0, REPRO_I64 = 1 } repro_key_t;

/* value columns of one multi-column call or served query, at most */
#define REPRO_MAX_COLS 8

/*
 * Bytes of a state buffer for G groups (layout above).  Returns 0 for
 * invalid arguments (G < 1, L outside 1..4).
 */
size_t repro_state_bytes(int64_t num_groups, repro_scalar_t T, int L);

/*
 * Bytes of scratch memory repro_groupby_sum needs for these sizes (may be
 * 0).  Depends only on the arguments, never on the data.
 */
size_t repro_workspace_bytes(int64_t n, int64_t num_groups, repro_key_t kt, repro_scalar_t vt,
                             repro_scalar_t T, int L);

/* Writes the empty state of every group (the initialised state Alg. 2 loads). */
int repro_state_init(void* states, int64_t num_groups, repro_scalar_t T, int L, hipStream_t stream);

/*
 * GroupBy-SUM (Sec. II-A; the repro type's operator+=(ScalarT), Sec. IV):
 * adds rows i = 0..n-1, value values[i] into group keys[i], to `states`
 * (accumulated into: pass freshly initialised states for a plain GroupBy,
 * or earlier results to resume, as Alg. 2's load/store of state allows).
 *
 *   keys       int32 or int64 (kt), dense group ids in [0, num_groups)
 *              (identity hashing, Sec. VI-A); others set REPRO_ERR_KEY.
 *   values     float or double (vt).  vt = F32 with T = F64 widens exactly;
 *              vt = F64 with T = F32 is REPRO_EINVAL.
 *   n          rows, >= 0 (n = 0 enqueues nothing).
 *   num_groups 1 .. 2^31-1.  Groups that do not fit one workgroup's LDS are
 *              partitioned first (Alg. 4); beyond 2^24 groups (2^23 at
 *              L = 4) a second partitioning level runs, and the call waits
 *              once for its stream to read the first level's partition
 *              sizes (so such calls cannot be captured in a HIP graph).
 *   L          levels, 1..4.
 *   workspace  >= repro_workspace_bytes(...) bytes, 256-byte aligned device
 *              memory (may be NULL if that size is 0); contents on entry are
 *              ignored.
 *   status     device uint32, OR-ed with REPRO_ERR_* bits; may be NULL.
 *
 * Result bits depend only on the multiset of (key, value) rows deposited
 * into each group since initialisation: not on the row order, the split
 * into calls, the stream or the launch configuration.  Groups that saw a
 * skipped row hold the sum of their other rows.
 */
int repro_groupby_sum(const void* keys, repro_key_t kt, const void* values, repro_scalar_t vt, int64_t n,
                      int64_t num_groups, repro_scalar_t T, int L, void* states, void* workspace,
                      size_t workspace_bytes, uint32_t* status, hipStream_t stream);

/*
 * dst[g] += src[g] for every group (operator+=(repro), Sec. IV; the merge
 * phase of Alg. 4, Sec. V-B): the larger top wins, the other state's levels
 * move down by the difference (its lowest levels drop off), level sums add
 * exactly, carries renormalise.  dst and src may not overlap.
 */
int repro_merge(void* dst, const void* src, int64_t num_groups, repro_scalar_t T, int L, hipStream_t stream);

/*
 * out[g] = the finalised sum of group g, type T (equation of Sec. III-C):
 * each level's exact value is rounded once to T, then the levels are added
 * in T from the last one to the first.  Empty groups give +0.0.
 */
int repro_finalize(const void* states, int64_t num_groups, repro_scalar_t T, int L, void* out,
                   hipStream_t stream);

/*
 * Baseline, NOT reproducible: out[g] += values[i] for keys[i] == g with
 * plain double-precision adds (the built-in floating-point SUM the paper
 * compares against, Sec. VI).  out is double[num_groups], accumulated into;
 * status as above (bad keys and non-finite values are skipped).
 *
 * Groups that fit one workgroup's LDS are summed with LDS double atomics,
 * then one global atomic per group and workgroup.  Beyond that the same
 * algorithm as the reproducible path runs on doubles (PartitionAndAggregate
 * on built-in types, as Sec. VI-C compares): partition on the key's high
 * bits, LDS double atomics per partition; this needs a workspace of
 * repro_plain_workspace_bytes(...) bytes (256-byte aligned).  Without one
 * (workspace NULL or too small), those groups take direct global double
 * atomics instead.
 */
size_t repro_plain_workspace_bytes(int64_t n, int64_t num_groups, repro_key_t kt, repro_scalar_t vt);
int repro_plain_groupby_sum(const void* keys, repro_key_t kt, const void* values, repro_scalar_t vt, int64_t n,
                            int64_t num_groups, double* out, void* workspace, size_t workspace_bytes,
                            uint32_t* status, hipStream_t stream);

/*
 * Several SUM aggregates over one GROUP BY (Sec. V-D: a query's aggregates
 * per group; Sec. VI-E's TPC-H Q1 has several SUMs over one key): for every
 * column c = 0..ncols-1, states[c] += the GroupBy-SUM of values[c] over
 * keys, with exactly the bits repro_groupby_sum gives for that column
 * alone.  The key column is read once for up to four columns whose groups
 * fit one workgroup's LDS together (T = double); other shapes run column by
 * column.
 *
 *   ncols      1 .. REPRO_MAX_COLS.
 *   values     HOST array of ncols device pointers, each n entries of type
 *              vts[c] (HOST array).  Fusion needs keys aligned to two keys
 *              and each column to two of its elements; otherwise the call
 *              still works, column by column.
 *   states     HOST array of ncols distinct device state buffers.
 *   workspace  >= repro_workspace_bytes_cols(...) bytes, 256-byte aligned.
 *   other arguments and errors as for repro_groupby_sum; REPRO_EINVAL is
 *   returned before anything is enqueued.
 */
size_t repro_workspace_bytes_cols(int64_t n, int64_t num_groups, repro_key_t kt, int ncols,
                                  const repro_scalar_t* vts, repro_scalar_t T, int L);
int repro_groupby_sum_cols(const void* keys, repro_key_t kt, int ncols, const void* const* values,
                           const repro_scalar_t* vts, int64_t n, int64_t num_groups, repro_scalar_t T, int L,
                           void* const* states, void* workspace, size_t workspace_bytes, uint32_t* status,
                           hipStream_t stream);

/*
 * Baseline of the multi-column call, NOT reproducible: outs[c][g] +=
 * values[c][i] for keys[i] == g with plain double atomics, the key column
 * read once for up to four columns.  outs is a HOST array of ncols device
 * double[num_groups] buffers, accumulated into.
 */
int repro_plain_groupby_sum_cols(const void* keys, repro_key_t kt, int ncols, const void* const* values,
                                 const repro_scalar_t* vts, int64_t n, int64_t num_groups, double* const* outs,
                                 uint32_t* status, hipStream_t stream);

/*
 * Ungrouped reproducible sum (RSum over a whole column, Sec. III-C/III-D):
 * state (a one-group state buffer, repro_state_bytes(1, T, L)) += the sum
 * of values[0..n).  Bits equal those of repro_groupby_sum with every key 0
 * and one group; no keys are read.  values as for repro_groupby_sum;
 * workspace >= repro_sum_workspace_bytes(n, L) bytes, 256-byte aligned.
 * REPRO_EINVAL also for n beyond 2^35.
 */
size_t repro_sum_workspace_bytes(int64_t n, int L);
int repro_sum(const void* values, repro_scalar_t vt, int64_t n, repro_scalar_t T, int L, void* state,
              void* workspace, size_t workspace_bytes, uint32_t* status, hipStream_t stream);

/*
 * Exact row counts per group (COUNT(*) of the GroupBy, Sec. II-A):
 * counts[g] += number of rows with key g (int64, accumulated into; integer
 * additions, so order-free).  Bad keys set REPRO_ERR_KEY.
 */
int repro_groupby_count(const void* keys, repro_key_t kt, int64_t n, int64_t num_groups, int64_t* counts,
                        uint32_t* status, hipStream_t stream);

/*
 * Aggregates derived from reproducible sums (AVG, VAR, STDDEV computed from
 * SUM, as Sec. I notes they can be): from the finalised SUM(x), SUM(x*x)
 * (float64) and COUNT of every group, in a fixed order of IEEE operations,
 * no fused multiply-add:
 *   avg = s / c;  var_samp = (q - s * avg) / (c - 1);  stddev = sqrt(var).
 * NaN where c = 0 (avg) or c < 2 (var, stddev).  Any output may be NULL.
 */
int repro_derive_stats(const double* sum, const double* sumsq, const int64_t* count, int64_t num_groups, double* avg,
                       double* var_samp, double* stddev_samp, hipStream_t stream);

/*
 * Expression columns for aggregates such as SUM(a * b) (RSum(expression,
 * L), Sec. V-D) or the SUM(x * x) behind a variance (Sec. I):
 * out[i] = a[i] * b[i] in double precision, one IEEE rounding to nearest
 * even, no fused multiply-add.  a and b are float (at/bt = F32, widened
 * exactly) or double columns of n entries; out is double[n] (may be a or b
 * when that column is double).  n = 0 enqueues nothing.
 */
int repro_mul(const void* a, repro_scalar_t at, const void* b, repro_scalar_t bt, int64_t n, double* out,
              hipStream_t stream);

/*
 * ------------------------------------------------------------ batches
 *
 * Many independent GroupBy-SUMs (jobs) in one persistent kernel launch.
 * Each job is what repro_groupby_sum computes for its own rows, groups and
 * level count (Sec. II-A; operator+=(ScalarT) and, across the pieces of a
 * job, operator+=(repro) of Sec. IV); its result bits are the same as
 * those of repro_groupby_sum on the same rows, whatever the batch, the
 * configuration or the schedule.  All jobs of a batch share kt, vt and T.
 *
 * Work is cut into items (job, row chunk, group slice).  A job whose groups
 * do not fit one workgroup's LDS is cut into group slices.  By default
 * (split 0) one item per chunk sorts the chunk's rows by slice into a copy
 * in the workspace and then aggregates each slice from its own rows (the
 * chunk-local partitioning of Alg. 4); with split 1, or beyond 64 slices,
 * every item of a slice reads the whole chunk and keeps only its slice's
 * groups.  Items are taken from a queue in order of decreasing size; the
 * last item of a (job, slice) to finish folds that slice's partial sums
 * into the states (and finalises them into `out`, when given).
 *
 * Use: repro_batch_workspace_bytes -> repro_batch_prepare (host planning,
 * uploads the plan into the workspace and waits for that copy) ->
 * repro_batch_launch (kernels only: may be captured into a HIP graph and
 * replayed; every launch recomputes the whole batch).  The plan stays valid
 * while the workspace and the jobs' buffers do.
 */
typedef struct {
    const void* keys;    /* device, kt, n entries                                  */
    const void* values;  /* device, vt, n entries                                  */
    int64_t n;           /* rows, >= 0                                             */
    int64_t num_groups;  /* 1 .. 2^31-1                                            */
    int L;               /* levels, 1..4                                           */
    int accumulate;      /* 1: add into `states`; 0: overwrite them with this batch */
    void* states;        /* device state buffer of the job (layout above)          */
    void* out;           /* device T[num_groups] finalised sums, or NULL           */
} repro_batch_job;

/* Tuning knobs.  None of them changes a result bit.  Zero fields take the
 * defaults (chunk_rows 131072, max_slice_groups as large as LDS allows,
 * order 0, merge 0, split 0). */
typedef struct {
    int64_t chunk_rows;   /* rows per item (rounded up to a multiple of 8192)  */
    int max_slice_groups; /* cap on the groups of one slice (bins per LDS)     */
    int order;            /* 0: largest items first, 1: job order              */
    int merge;            /* merge schedule of jobs cut into several chunks:
                             0: the last chunk to finish merges (in the
                             persistent launch), 1: a merge launch after it   */
    int split;            /* jobs cut into group slices: 0: each chunk's rows
                             are sorted by slice once (workspace holds the
                             sorted copy, 2 + sizeof(vt) bytes per row), 1:
                             every slice reads the whole chunk              */
} repro_batch_config;

/* Plan handle filled by repro_batch_prepare (host memory, plain data). */
typedef struct {
    void* workspace;
    int64_t items;
    int grid, lds_bytes;
    int kt, vt, T;
    int reserved[4];
} repro_batch_plan;

/* Workspace bytes for this batch and configuration (cfg may be NULL);
 * 0 for invalid arguments. */
size_t repro_batch_workspace_bytes(const repro_batch_job* jobs, int njobs, repro_key_t kt, repro_scalar_t vt,
                                   repro_scalar_t T, const repro_batch_config* cfg);

/* Validates the jobs (host array) and the configuration, plans the items
 * and copies the plan into `workspace` on `stream` (then waits for the
 * stream).  REPRO_EINVAL for invalid jobs (a NULL pointer a job needs, L
 * outside 1..4, num_groups out of range, vt = F64 with T = F32, more than
 * 2^31 rows in a job) or a workspace too small or not 256-byte aligned. */
int repro_batch_prepare(const repro_batch_job* jobs, int njobs, repro_key_t kt, repro_scalar_t vt, repro_scalar_t T,
                        const repro_batch_config* cfg, void* workspace, size_t workspace_bytes,
                        repro_batch_plan* plan, hipStream_t stream);

/* Runs a prepared batch on `stream`: a reset kernel, then the persistent
 * kernel (and the merge kernel under merge schedule 1).  status as for repro_groupby_sum (may be NULL).  Jobs that
 * accumulate must see their states' previous contents, so two launches of
 * the same plan add the batch twice; jobs that overwrite give the same
 * states every launch. */
int repro_batch_launch(const repro_batch_plan* plan, uint32_t* status, hipStream_t stream);

/* Autotuner: times the candidate configurations (chunk rows, slice cap,
 * order, merge schedule, split) on this batch and writes the fastest to *best (and its time in ms
 * to *best_ms, if not NULL).  It runs the batch many times: the jobs'
 * states and outputs hold unspecified values afterwards.  Candidates whose
 * workspace exceeds workspace_bytes are skipped.  Blocks until done. */
int repro_batch_tune(const repro_batch_job* jobs, int njobs, repro_key_t kt, repro_scalar_t vt, repro_scalar_t T,
                     void* workspace, size_t workspace_bytes, repro_batch_config* best, float* best_ms,
                     hipStream_t stream);

/*
 * ------------------------------------------------------------ serving
 *
 * A request loop for GroupBy queries with several reproducible SUM
 * aggregates (RSum(expression, L), Sec. V-D; the expression is a column or
 * the IEEE product of two columns, rounded once, no fused multiply-add).
 * Queries are admitted in arrival order when a slot and device memory are
 * free; an admitted query's states live in the server's arena and take its
 * rows chunk by chunk (the resumable state of Alg. 2: each chunk is added to
 * the resident states), then are finalised into the caller's outputs.
 * Admitted queries run on separate streams, so their work overlaps on the
 * device.  Every result is bit-identical to repro_groupby_sum of the same
 * expression column alone: admission order, concurrency, chunking and the
 * execution path do not change a bit.  The server allocates pinned host
 * memory for plan uploads (a few KiB per slot), no device memory.
 */
#define REPRO_MAX_AGGS 4

typedef struct {
    const int32_t* keys;                 /* device, n entries, dense ids           */
    const double* cols[REPRO_MAX_COLS];  /* device f64 columns, n entries (or NULL) */
    int64_t n;                           /* rows, >= 0                              */
    int64_t num_groups;                  /* 1 .. 2^31-1                             */
    int L;                               /* levels of every aggregate, 1..4         */
    int naggs;                           /* 1 .. REPRO_MAX_AGGS                     */
    int agg_a[REPRO_MAX_AGGS];           /* SUM(cols[agg_a]) ...                    */
    int agg_b[REPRO_MAX_AGGS];           /* ... * cols[agg_b] when agg_b >= 0       */
    double* out[REPRO_MAX_AGGS];         /* device f64[num_groups] finalised sums   */
    uint32_t* status;                    /* device status word (OR-ed), or NULL     */
} repro_query;

typedef struct {
    int slots;           /* queries on the GPU at once (one stream each), 1..64 */
    int64_t chunk_rows;  /* rows added to a query's states per call (0: 16M)   */
    int no_batch_path;   /* 0: a query whose groups fit one workgroup's LDS runs
                            its aggregates as jobs of one persistent batch launch
                            (its plan uploaded from pinned host memory); 1: every
                            query uses repro_groupby_sum chunk by chunk          */
    int query_workgroups;  /* on the batch path, persistent workgroups per query
                              (0: as many as the GPU holds).  Fewer let queries
                              of other slots run beside a long one           */
    int max_bypass;      /* a queued query whose memory does not fit yet may be
                            passed by later queries that fit, at most this many
                            times; then admission waits for it (0: strict
                            arrival order)                                    */
} repro_server_config;

typedef struct repro_server repro_server;

/* Arena bytes a query needs while admitted (0 for an invalid query). */
size_t repro_query_bytes(const repro_query* q, const repro_server_config* cfg);

/* A server over a caller-owned device arena (256-byte aligned), which it
 * sub-allocates for admitted queries.  Creates its streams (default
 * priority). */
int repro_server_create(void* arena, size_t arena_bytes, const repro_server_config* cfg, repro_server** srv);

/* Queues a query (host record copied; device buffers must stay valid until
 * the query completes).  *ticket numbers queries from 0 in submission order.
 * REPRO_EINVAL for an invalid query or one larger than the whole arena. */
int repro_server_submit(repro_server* srv, const repro_query* q, int64_t* ticket);

/* Makes progress without blocking: retires finished queries (freeing their
 * memory and slot), then admits queued queries in arrival order while slots
 * are free and their memory fits (a query that does not fit may be passed by
 * later ones up to max_bypass times).
 * Writes up to `cap` completed tickets and their completion times (seconds
 * on the host's monotonic clock); a finished query beyond `cap` stays in its
 * slot and is reported by a later call.  Always writes the counts of
 * completed (in this call, <= cap), queued and running queries, also when it
 * returns an error.  If enqueueing an admitted query's work fails, that query
 * is dropped: its slot and memory are freed once what was enqueued has
 * finished, its ticket is written to *dropped (otherwise -1), admission stops
 * for this call and REPRO_EHIP is returned.  Any output pointer may be NULL. */
int repro_server_poll(repro_server* srv, int64_t* tickets, double* times, int cap, int* ndone, int* nqueued,
                      int* nrunning, int64_t* dropped);

/* The host's monotonic clock (seconds) used for completion times. */
double repro_server_clock(void);

/* Waits for the running queries, then destroys the server (queued queries
 * are dropped). */
int repro_server_destroy(repro_server* srv);

/*
 * Profiling aid.  repro_profile_arm(k) makes the next k measured launches
 * of repro_groupby_sum calls issued by the calling host thread record a
 * pair of HIP events on their stream, right before and right after the
 * launch: the aggregation kernel (the one pass over the rows) on the LDS
 * path; the partition scatter and then the partition aggregation (two
 * measured launches per call) on the partitioned path.  The multi-column
 * call measures its fused pass.  repro_profile_read(ms, cap, &count) waits for
 * the recorded events and writes the elapsed milliseconds of each measured
 * launch, in call order (at most cap), then disarms.  k <= 4096.  Events are
 * created on first use, per thread; no device memory is involved.
 */
int repro_profile_arm(int max_launches);
int repro_profile_read(float* ms, int cap, int* count);

/*
 * Measurement aid: reads `bytes` (a multiple of 16, 16-byte aligned device
 * memory) once with 16-byte loads on a grid of `workgroups` x `threads`
 * (threads a multiple of 64, at most 1024), folding the words so that the
 * loads are kept; adds to *sink (device uint64) the number of workgroups
 * that read nonzero data.  Its rate is the read-stream ceiling of the chip.
 */
int repro_read_probe(const void* data, size_t bytes, int workgroups, int threads, unsigned long long* sink,
                     hipStream_t stream);

/*
 * Measurement aid: one 64-bit device-scope atomic add per index,
 * table[idx[i]] += 1 for i < n (idx: device int32; table: device uint64 of
 * table_words entries; an index outside [0, table_words) is skipped), on a
 * grid of `workgroups` x 256 threads.  Its rate is that of global atomics
 * on a working set of table_words * 8 bytes (e.g. the Infinity Cache), the
 * bound of aggregating level words with global atomics instead of
 * partitioning into LDS.
 */
int repro_atomic_probe(const int32_t* idx, int64_t n, unsigned long long* table, int64_t table_words,
                       int workgroups, hipStream_t stream);

/* Library version string. */
const char* repro_version(void);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * GroupBy-SUM as repro_groupby_sum, with the same arguments, status bits and
 * result bits, but with no workspace argument.  Its scratch memory is a
 * static device array of REPRO_NOALLOC_SCRATCH_BYTES inside the library;
 * every GPU the library runs on holds its own copy until the process ends.
 * The call allocates nothing (no hipMalloc, no hipFree).
 *
 *   - REPRO_EINVAL when repro_workspace_bytes(...) for these sizes exceeds
 *     REPRO_NOALLOC_SCRATCH_BYTES (it covers every call whose groups fit one
 *     workgroup's LDS up to 2^31 rows, and small high-cardinality calls),
 *     and for every argument repro_groupby_sum rejects.
 *   - The scratch array belongs to the device that is current on the calling
 *     thread; `stream` must belong to that device.  Its address is looked up
 *     once per device (REPRO_EHIP if that fails).
 *   - All calls on one GPU share that GPU's array and it keeps the last
 *     call's contents: two calls that may overlap on one GPU (different
 *     streams, or host threads without ordering) race on it and give wrong
 *     results.  Order them on one stream or with events.
 */
#define REPRO_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int repro_groupby_sum_noalloc(const void* keys, repro_key_t kt, const void* values, repro_scalar_t vt, int64_t n,
                              int64_t num_groups, repro_scalar_t T, int L, void* states, uint32_t* status,
                              hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* REPRO_H */
