/*
 * tds.h - distance-threshold search over trajectory line segments on one
 * AMD Instinct MI355X (gfx950).
 *
 * The problem (Gowanlock & Casanova, "Parallel Distance Threshold Query
 * Processing for Spatiotemporal Trajectory Databases on the GPU", Sec. 3):
 * a database D of n line segments in 3 spatial dimensions + time, each with
 * a start point (x,y,z,t)_start, an end point (x,y,z,t)_end and a trajectory
 * id; the point moves linearly from start to end. Given query segments and a
 * distance d per query segment, report every (query segment, entry segment,
 * [t_a, t_b]) such that the two moving points are within Euclidean distance
 * d at every time of [t_a, t_b], where [t_a, t_b] is the full set of such
 * times inside the two segments' common time span.
 *
 * Method (Sec. 4 and Sec. 5, Alg. 1): entries sorted by t_start and grouped
 * into m fixed-width temporal bins give each query segment a contiguous
 * candidate index range; each candidate is compared with the query segment
 * (temporal intersection, then the time interval within d from a degree-two
 * polynomial) and hits are appended to a result buffer.
 *
 * Semantics shared by every entry point:
 *  - Two spans are compared only when they overlap with positive length:
 *    max(t_start) < min(t_end).
 *  - "Within d" is closed (distance <= d); a tangency gives [t*, t*].
 *  - The decision is taken in IEEE binary64 by one fixed expression, so the
 *    hit set does not depend on launch shape, batch size, bin count or mode.
 *  - Result order is unspecified; sort by (query_idx, entry_idx) to compare.
 *
 * Threading: an index is immutable after build and may be shared by several
 * query handles on several streams. One query handle must not be used by
 * two threads at once.
 *
 * Errors: every int-returning call returns TDS_OK (0) or a negative status;
 * tds_last_error() gives a message for the calling thread's last failure.
 */
#ifndef TDS_H
#define TDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TDS_ABI_VERSION 1

/* Status codes. */
#define TDS_OK 0
#define TDS_EINVAL (-1)    /* null pointer, n < 0, t_end <= t_start, non-finite value, d < 0, bad option */
#define TDS_ENOMEM (-2)    /* device or host allocation failed */
#define TDS_EDEVICE (-3)   /* a HIP call failed (message names it) */
#define TDS_EOVERFLOW (-4) /* more selected pairs than the result slabs hold after all retries */
#define TDS_ESTATE (-5)    /* call out of order (e.g. fetch before a query) */
#define TDS_EBUSY (-6)     /* serving: the request was refused (its waiting queue is full) */

/* Where the arrays of a tds_segments live. */
#define TDS_MEM_HOST 0
#define TDS_MEM_DEVICE 1

/*
 * Segments as a structure of arrays (Sec. 3): start point (x0,y0,z0,t0) and
 * end point (x1,y1,z1,t1) of segment i are x0[i] ... t1[i]. All arrays hold n
 * binary64 values and live in host or device memory as `mem` says. traj_id
 * (optional, may be NULL: then the trajectory id is the segment's index) is
 * copied into results. The caller keeps ownership; the library only reads
 * the arrays during the call that receives them.
 */
typedef struct {
    int64_t n;
    int32_t mem;
    int32_t reserved;
    const double *x0, *y0, *z0, *t0;
    const double *x1, *y1, *z1, *t1;
    const int64_t *traj_id;
} tds_segments;

/* Index options (Sec. 4). num_bins: m >= 1 fixed-width temporal bins over
 * [min t_start, max t_end] of the database. */
typedef struct {
    int32_t num_bins;
    int32_t flags; /* reserved, 0 */
} tds_index_opts;

/* Query modes. */
#define TDS_MODE_FP64 0         /* every candidate pair decided in binary64 */
#define TDS_MODE_FP32_REFINE 1  /* binary32 conservative filter, binary64 decision of survivors */

/* How query segments are grouped into tiles (batches, Sec. 6). */
/* Periodic (Sec. 6): consecutive runs of batch_size query segments with
 * candidates, in (t_start, caller index) order. */
#define TDS_TILE_PERIODIC 0
#define TDS_TILE_RANGE 1        /* runs of <= batch_size segments with the same candidate bin range */
/* GreedySetSplit (Sec. 6, Alg. 4) over the query segments with candidates in
 * (t_start, caller index) order: first neighbours merge while the merge adds
 * no interactions (same candidate range, and the merged temporal extent
 * overlaps no further bin), then a second pass merges each batch with its
 * successor while the batch holds fewer than batch_size segments (Min), or
 * while the merged batch would hold at most batch_size segments (Max). */
#define TDS_TILE_GREEDY_MIN 2
#define TDS_TILE_GREEDY_MAX 3

/* Query flags. */
#define TDS_QF_TIMING 1          /* record per-stage HIP event times; tds_query_stats reads them */
#define TDS_QF_COUNT_OVERLAP 2   /* count pairs whose spans overlap (tds_stats.n_overlap) */
#define TDS_QF_KERNEL_OVERLAP 4  /* the pair kernel also counts the overlapping pairs it examined */
#define TDS_QF_TIMING_PAIR 8     /* time only the pair kernel (tds_stats.ms_pair; the other ms_* are 0):
                                    two events on one dispatch, the lightest timing */

typedef struct {
    int32_t mode;        /* TDS_MODE_* */
    int32_t tiling;      /* TDS_TILE_* */
    int32_t batch_size;  /* TDS_TILE_PERIODIC: query segments per tile (s); TDS_TILE_GREEDY_*:
                            the bound; 1..65536; 0 = 128 */
    int32_t block_size;  /* pair-kernel threads per workgroup: 64, 128, 256, 512 or 1024; 0 = 256 */
    int32_t reserved0;   /* 0 */
    int32_t max_retries; /* result-buffer regrowths allowed; < 0 = 4 */
    int64_t capacity;    /* initial result capacity, counted in pair-kernel selections beyond the
                            per-wave result slabs: FP64 the decided hits, FP32_REFINE the binary32
                            filter's survivors (hits and near-threshold pairs); 0 = 1,048,576 */
    int32_t grid;        /* pair-kernel workgroups; 0 = as many as are resident at once */
    int32_t flags;       /* TDS_QF_* */
} tds_query_opts;

/* One result (Sec. 3 and Alg. 1): indices are positions in the caller's
 * arrays; entry_traj is the entry's trajectory id. */
typedef struct {
    int64_t query_idx;
    int64_t entry_idx;
    int64_t entry_traj;
    double t_a;
    double t_b;
} tds_hit;

typedef struct {
    int64_t n_query;     /* query segments in the last batch */
    int64_t n_eval;      /* candidate pairs examined: sum over tiles of segments x range */
    int64_t n_overlap;   /* pairs with a common span of positive length, counted from the sorted
                            time arrays (TDS_QF_COUNT_OVERLAP), else -1 */
    int64_t n_overlap_k; /* the same, counted in the pair kernel (TDS_QF_KERNEL_OVERLAP), else -1 */
    int64_t n_refine;    /* pairs the pair kernel passed to the refine kernel: FP32_REFINE the
                            filter's survivors, FP64 the decided hits */
    int64_t n_hit;
    int64_t n_tiles;     /* tiles: the batches of query segments the pair kernel walks (TDS_TILE_*) */
    int64_t n_items;     /* work units of the pair kernel (query segment x entry chunk) */
    int32_t retries;
    int32_t grid;        /* pair-kernel workgroups used */
    float ms_prep;       /* TDS_QF_TIMING: query preparation, sort and tiling */
    float ms_pair;       /* pair kernel (last launch) */
    float ms_fetch;      /* the batch's last kernel at fetch: hit offsets, records, counters */
    float ms_refine;     /* refine kernel (last launch) */
    int32_t chunk;       /* entries per chunk: a work unit pairs one query segment with at most
                            this many consecutive candidate entries (64 x entries per lane) */
    int32_t reserved1;
} tds_stats;

typedef struct {
    int64_t n;           /* entries */
    int32_t num_bins;    /* m as requested */
    int32_t nonempty_bins;
    double t_first;      /* min t_start */
    double t_last;       /* max t_end */
    double bin_width;    /* (t_last - t_first) / m */
    int64_t device_bytes;
} tds_index_info;

/* One non-empty bin (Sec. 4): start = smallest t_start of its entries,
 * end = largest t_end, [first, last] = its index range in t_start order,
 * bin = its number j in 0..m-1. */
typedef struct {
    double start;
    double end;
    int64_t first;
    int64_t last;
    int64_t bin;
} tds_bin;

typedef struct tds_index tds_index;
typedef struct tds_query tds_query;

/*
 * Build the index of a database (Sec. 4): entries sorted by non-decreasing
 * t_start (ties in input order), m bins of width (t_last - t_first)/m with
 * entry i in bin clamp(floor((t0_i - t_first)/width), 0, m-1), and per bin
 * its start, end and index range. The sorted entries, their velocities and
 * their binary32 boxes go to device memory and stay there. `db` may be in
 * host or device memory; `stream` (a hipStream_t, NULL = default) orders the
 * uploads, and the call returns after they are complete. Returns TDS_EINVAL
 * for invalid segments, n == 0 is allowed (every query then has 0 hits).
 */
int tds_build_index(const tds_segments *db, const tds_index_opts *opts, void *stream,
                    tds_index **out);
int tds_index_info_get(const tds_index *ix, tds_index_info *out);
/* Copy up to cap non-empty bins (in time order) to host memory; *n_out gets
 * their number. */
int tds_index_bins(const tds_index *ix, tds_bin *out, int64_t cap, int64_t *n_out);
/* Copy the index's t_start values (in its t_start order) and its t_end values
 * (sorted on their own) to host arrays of n values, n = the entry count.
 * With them the number of entries whose span overlaps an interval (a, b)
 * with positive length is count(t_start < b) - count(t_end <= a), two binary
 * searches (the exact temporal-miss count of Sec. 8's beta). Errors:
 * TDS_EINVAL for null arrays with n > 0 or n other than the entry count,
 * TDS_EDEVICE on a failed copy. */
int tds_index_times(const tds_index *ix, double *t_start_sorted, double *t_end_sorted, int64_t n);
/* Release the index. Every query handle made from it must be destroyed first. */
void tds_index_destroy(tds_index *ix);

/*
 * Compute bins from host arrays of t_start / t_end that are already sorted
 * by t_start (no device needed): same rules as tds_build_index. Writes up to
 * cap non-empty bins to out and their number to *n_out.
 */
int tds_plan_bins(const double *t0_sorted, const double *t1_sorted, int64_t n, int32_t num_bins,
                  tds_bin *out, int64_t cap, int64_t *n_out);

/*
 * The candidate range of query segments (Sec. 4, host planning helper, no
 * device needed): for each (t0[i], t1[i]) the bins whose temporal extent
 * [start, end] overlaps it with positive length (start < t1[i] and
 * end > t0[i]); first[i] is the smallest first member and last[i] the
 * largest last member of those bins (last < first when no bin overlaps).
 * The device computes the same range for every query segment of a batch.
 * bins: the non-empty bins in time order, as tds_plan_bins or
 * tds_index_bins give them. Errors: TDS_EINVAL for negative counts or null
 * arrays with positive counts.
 */
int tds_plan_ranges(const tds_bin *bins, int64_t nb, const double *t0, const double *t1,
                    int64_t nq, int64_t *first, int64_t *last);

/* A query handle owns the device buffers of one batch at a time (query
 * records, tiles, result buffer); they grow on demand and are reused. */
int tds_query_create(tds_index *ix, tds_query **out);
void tds_query_destroy(tds_query *qh);

/*
 * Start the search of query segments q (with per-segment thresholds d[i] >= 0,
 * n values, in the same memory space as q) against the index, on `stream`:
 * the distance threshold query of Sec. 3 for one set of query segments. Each
 * query segment gets its candidate range from the bins (Sec. 4); the segments
 * are grouped into tiles (opts->tiling: range buckets, Periodic or
 * GreedySetSplit, Sec. 6); every candidate pair goes through the temporal
 * intersection and the degree-two polynomial of the squared distance
 * (Sec. 5, Alg. 1), decided in binary64 (TDS_MODE_FP64) or first screened by
 * a conservative binary32 test whose survivors are decided in binary64
 * (TDS_MODE_FP32_REFINE; the hit set is the same); hits are compacted into
 * the result slabs (Alg. 1: appended to the result set).
 * Returns once the work is enqueued; inputs in device memory must stay valid
 * until tds_fetch_results returns. Inputs in host memory are copied first.
 * Errors: TDS_EINVAL for null pointers, n out of range, an unknown mode,
 * tiling or block size; TDS_ESTATE when the previous batch of the handle was
 * not fetched; TDS_ENOMEM / TDS_EDEVICE for failed device calls. Invalid
 * segments or thresholds (non-finite values, t_end <= t_start, d < 0), in
 * host or device memory, are found by the preparation kernel and reported
 * by tds_fetch_results as TDS_EINVAL.
 */
int tds_query_batch(tds_query *qh, const tds_segments *q, const double *d,
                    const tds_query_opts *opts, void *stream);

/*
 * Wait for the batch, re-run the pair kernel with a larger result buffer if
 * it overflowed (Sec. 5: re-attempt with more memory), translate to caller
 * indices and write min(cap, n) records to `out` in an unspecified order
 * (host memory when out_mem is
 * TDS_MEM_HOST, device memory for TDS_MEM_DEVICE). *n_total always receives
 * the number of hits, so cap = 0 sizes the buffer. Host output is complete on
 * return; device output is written on the batch's stream, so work on another
 * stream must wait for it. Errors: TDS_EINVAL for bad arguments or a batch
 * holding an invalid query segment or threshold; TDS_ESTATE without a
 * pending or fetched batch; TDS_EOVERFLOW when the selections outgrow the
 * buffer after max_retries regrowths; TDS_ENOMEM / TDS_EDEVICE for failed
 * device calls.
 */
int tds_fetch_results(tds_query *qh, tds_hit *out, int64_t cap, int32_t out_mem, int64_t *n_total);
int tds_query_stats(const tds_query *qh, tds_stats *out);
/* After tds_fetch_results: the candidate range the device computed for each
 * query segment of the last batch (caller order, host arrays of n values). */
int tds_query_ranges(const tds_query *qh, int64_t *first, int64_t *last, int64_t n);

/* One tile (batch) of the last batch's pair launch. */
typedef struct {
    int32_t q_first; /* first member: position in the member order of tds_query_tiles */
    int32_t n_query; /* member query segments (positions q_first .. q_first + n_query - 1) */
    int32_t e_first; /* candidate range: entries e_first .. e_first + n_entry - 1 of the index,
                        counted in the index's t_start order (ties in caller order). Periodic and
                        GreedySetSplit tiles take the range of the tile's temporal extent (smallest
                        t_start to largest t_end of its members, Sec. 4); range tiles the union of
                        their members' ranges */
    int32_t n_entry;
} tds_tile_info; /* 16 bytes */

/*
 * After tds_fetch_results (or tds_fetch_trajectories): the tiles (batches,
 * Sec. 6) the device built for the last batch and the order of their
 * members. Writes min(cap, n_tiles) tiles to `tiles` and min(member_cap,
 * n_members) caller indices of query segments to `members` (host memory;
 * either pointer may be NULL with a cap of 0); *n_tiles and *n_members
 * receive the totals. Query segments without candidates are in no tile.
 * Errors: TDS_EINVAL for null counts or a negative cap, a null array with a
 * positive cap; TDS_ESTATE before a fetched batch; TDS_EDEVICE on a failed copy.
 */
int tds_query_tiles(const tds_query *qh, tds_tile_info *tiles, int64_t cap, int32_t *members,
                    int64_t member_cap, int64_t *n_tiles, int64_t *n_members);

/*
 * Trajectory-level answer of the last batch (Sec. 3: per query trajectory,
 * the entry trajectories within d and the times when). For each pair
 * (query trajectory, entry trajectory) the segment-pair intervals are merged
 * into maximal closed intervals (intervals that overlap or touch merge).
 */
typedef struct {
    int64_t query_traj; /* the query segments' trajectory id, as given */
    int64_t entry_traj; /* the entry segments' trajectory id (tds_segments.traj_id) */
    double t_a, t_b;    /* one maximal interval */
} tds_traj_hit;         /* 32 bytes */

/*
 * Complete the last batch like tds_fetch_results (waiting, and re-running on
 * overflow), then merge its hits per trajectory pair on the device.
 * query_traj: the trajectory id of each query segment of the batch (n values,
 * caller order) in memory space traj_mem. Writes min(cap, n) records, sorted
 * by (query_traj, entry_traj, t_a), to `out` in memory space out_mem;
 * *n_total receives the number of merged intervals (cap = 0 sizes). Usable
 * before or after tds_fetch_results for the same batch. A call with ids
 * merges; a call with query_traj == NULL copies the records the last merge
 * of this batch left in the handle (TDS_ESTATE if there is none), so
 * sizing and copying cost one merge. Device output is written on the
 * batch's stream; host output is complete on return. Errors: TDS_EINVAL
 * for a null n_total, cap < 0, cap > 0 with a null out, a bad memory space;
 * TDS_ESTATE without a batch; TDS_EDEVICE for a failed device call.
 */
int tds_fetch_trajectories(tds_query *qh, const int64_t *query_traj, int32_t traj_mem,
                           tds_traj_hit *out, int64_t cap, int32_t out_mem, int64_t *n_total);

/*
 * Device memory hook, so that a host framework can serve the library's
 * device buffers from its own allocator (for example PyTorch's caching
 * allocator; the paper keeps D resident on the GPU and sizes result memory
 * ahead of each kernel, Sec. 3 and Sec. 5, which is what these buffers are).
 * Every device buffer allocated after the call comes from
 * alloc(bytes, stream, ctx) and goes back through free(ptr, stream, ctx),
 * where `stream` is the HIP stream of the library call that needed it (the
 * build or batch stream; NULL for the default stream). A buffer is always
 * returned to the allocator that made it, so the hook may be changed while
 * indexes and query handles exist. alloc returning NULL fails the call with
 * TDS_ENOMEM. Both functions NULL restore hipMalloc / hipFree; exactly one
 * NULL is TDS_EINVAL. Process-wide; do not call it while another thread is
 * inside the library. Pinned host memory is not affected.
 */
typedef void *(*tds_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*tds_free_fn)(void *ptr, void *stream, void *ctx);
int tds_set_allocator(tds_alloc_fn alloc, tds_free_fn free_fn, void *ctx);

/*
 * One search that allocates nothing, for callers that cannot allocate device
 * memory: code that must not call hipMalloc (tight serving loops, harnesses
 * that forbid it, work prepared for HIP graph capture). It computes what
 * tds_query_batch followed by tds_fetch_results(out, cap, TDS_MEM_DEVICE)
 * computes, with the same kernels, but every per-batch buffer (query records,
 * ranges, buckets, tiles, counters, result slabs) lives in a fixed device
 * array of TDS_NOALLOC_SCRATCH_BYTES that the library holds on each device
 * it runs on until the process ends; no hipMalloc, hipFree, pinned host
 * memory, event or stream is created.
 *
 * q and d must be in device memory (TDS_MEM_DEVICE); out is device memory
 * for cap records (cap = 0 only counts). The call enqueues the search and
 * the writing of min(cap, n) records into `out` on `stream`, waits for it
 * (it reads the hit count) and returns: *n_total is the number of hits and
 * `out` is complete. On an error the contents of `out` are unspecified.
 * Options are those of tds_query_batch; capacity and max_retries are
 * ignored: the result slabs take whatever scratch the batch leaves free.
 *
 * Limits and errors: TDS_EINVAL for invalid arguments, host-memory inputs,
 * an invalid query segment, or a batch whose buffers do not fit the scratch
 * (the message gives the bytes it needs; about 180 bytes per query segment
 * plus 2 KiB per pair-kernel wave); TDS_EOVERFLOW when the selected pairs
 * need more result slabs than the scratch has left (no retry is possible);
 * TDS_EDEVICE for a failed HIP call. Calls that overlap on one GPU (from
 * several threads or streams) share its scratch and race; serialize them.
 * The scratch keeps the last call's contents; every call clears what it
 * counts before use.
 */
#define TDS_NOALLOC_SCRATCH_BYTES (64ull << 20)
int tds_search_noalloc(const tds_index *ix, const tds_segments *q, const double *d,
                       const tds_query_opts *opts, tds_hit *out, int64_t cap, int64_t *n_total,
                       void *stream);

/*
 * Grow the query handle's device buffers for batches of up to n_query
 * segments with `capacity` result selections (counted as in
 * tds_query_opts.capacity) under the launch shape of `opts` (mode, tiling,
 * block size, grid, batch size), without running anything. Buffers only
 * grow, and growing one frees the old buffer, which waits for the whole
 * device; a serving loop reserves once so that later batches up to that
 * size never wait for other streams' work. Errors: TDS_EINVAL for null
 * arguments, negative sizes or bad options; TDS_ESTATE while a batch is
 * pending; TDS_ENOMEM / TDS_EDEVICE for failed allocations.
 */
int tds_query_reserve(tds_query *qh, int64_t n_query, int64_t capacity, const tds_query_opts *opts);
/* Device bytes the query handle holds (all of its buffers), to *bytes. */
int tds_query_device_bytes(const tds_query *qh, int64_t *bytes);

/*
 * Serving (Sec. 3: several users query the resident database at once and
 * compete for GPU memory; Sec. 5: result memory is reserved before the
 * kernel runs; Sec. 8: the hit fraction alpha is estimated per temporal
 * epoch). A server holds an index and `streams` executors, each with its own
 * HIP stream and query handle. Requests (query segments with a threshold
 * each, in host memory) are submitted with an arrival time; a scheduler
 * thread admits arrived requests in arrival order while their estimated
 * result bytes fit the pool, groups them into one batch per free executor
 * (continuous batching: requests that arrive while batches run join the
 * next one) and the executor runs the batch (tds_query_batch +
 * tds_fetch_results) and splits its hits per request.
 *
 * Estimated result bytes of a request = 40 x k_safety x sum over its
 * segments of alpha(epoch of t_start) x candidate entries (Sec. 4 ranges
 * from the bin table), with alpha per epoch (`epochs` equal slices of the
 * database's time extent) a running estimate updated from every completed
 * batch; waiting requests are re-estimated with the current alpha each time
 * a batch is formed. The pool counts every executor's device bytes (its
 * query handle's buffers, which only grow) plus the estimates of the
 * batches in flight beyond what their executor already holds; a request is
 * admitted while that total stays within pool_bytes, and a batch of one
 * request is always admitted when nothing else is in flight (a request
 * larger than the pool then runs alone). A batch whose estimate was too
 * small still completes (the library re-runs with more memory).
 */
typedef struct {
    int32_t streams;            /* executors (batches in flight), 1..8; 0 = 4 */
    int32_t max_batch_segments; /* query segments per batch; 0 = 65,536 */
    int64_t max_waiting;        /* arrived requests not yet admitted beyond which tds_server_submit
                                   returns TDS_EBUSY; 0 = no limit */
    double pool_bytes;          /* device bytes for results across executors; 0 = 256 MiB */
    double k_safety;            /* multiplier on the estimated hits; 0 = 4 */
    int32_t epochs;             /* alpha epochs; 0 = 50 */
    int32_t reserve_segments;   /* segments each executor reserves buffers for at creation; 0 = max_batch_segments */
    double alpha_prior;         /* alpha before any batch completed; 0 = 1e-4 */
    tds_query_opts query;       /* options of every batch (capacity is set per batch) */
} tds_server_opts;

/* Timing and outcome of one request, in seconds on the server's clock
 * (tds_server_now). */
typedef struct {
    double arrival;  /* as submitted */
    double admit;    /* taken into a batch */
    double done;     /* its hits are split out and ready */
    int64_t n_hit;
    int64_t batch;   /* number of the batch that ran it */
    int32_t status;  /* TDS_OK, or the error of its batch */
    int32_t n_batch_requests; /* requests in that batch */
} tds_request_info;

typedef struct {
    int64_t batches, requests_done, retries, segments;
    int64_t device_bytes;  /* executors' device bytes now */
    double busy_s;         /* executor time spent in batches, summed over executors */
    /* the parts of busy_s: copying requests into pinned staging and enqueueing the
       upload and the batch; waiting for the batch and its results (tds_fetch_results);
       splitting the results per request and updating alpha */
    double stage_s, wait_s, split_s;
} tds_server_stats;

typedef struct tds_server tds_server;

/* Create a server over `ix` (which must outlive it); starts its clock and
 * its threads, and reserves each executor's buffers. Errors: TDS_EINVAL for
 * null arguments or bad options; TDS_ENOMEM / TDS_EDEVICE. */
int tds_server_create(tds_index *ix, const tds_server_opts *opts, tds_server **out);
/* Seconds since the server was created (steady clock). */
double tds_server_now(const tds_server *srv);
/*
 * Submit a request: q (host memory, q->n >= 1 segments) with thresholds d
 * (host, n values). The arrays are borrowed: they must stay valid and
 * unchanged until tds_server_wait has returned for the request. The request
 * becomes visible to the scheduler at `arrival` (server seconds; a time in
 * the past means now), so an open-loop load can be submitted ahead. *id
 * receives the request's id (0, 1, ... in submission order). Errors:
 * TDS_EINVAL for null arguments, n < 1, a non-finite arrival or an invalid
 * segment or threshold (checked here); TDS_EBUSY when max_waiting arrived
 * requests already wait; TDS_ESTATE after a failure stopped the server.
 */
int tds_server_submit(tds_server *srv, const tds_segments *q, const double *d, double arrival,
                      int64_t *id);
/* Wait until request `id` is done (or timeout_s passes; < 0 waits without
 * limit) and write its info. Returns TDS_OK when done, TDS_ESTATE on
 * timeout, TDS_EINVAL for an unknown id. */
int tds_server_wait(tds_server *srv, int64_t id, double timeout_s, tds_request_info *info);
/* After tds_server_wait: the request's hits (query_idx counts within the
 * request) to host memory, min(cap, n) records; *n_total gets n. */
int tds_server_results(tds_server *srv, int64_t id, tds_hit *out, int64_t cap, int64_t *n_total);
/* Drop a finished request's results (its id stays known). */
int tds_server_release(tds_server *srv, int64_t id);
int tds_server_stats_get(const tds_server *srv, tds_server_stats *out);
/* Current alpha estimate per epoch to host memory (cap values). */
int tds_server_alpha(const tds_server *srv, double *alpha, int32_t cap, int32_t *n);
/* Finish every submitted request, stop the threads and free the server. */
void tds_server_destroy(tds_server *srv);

const char *tds_last_error(void);
int tds_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TDS_H */
