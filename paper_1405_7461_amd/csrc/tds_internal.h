// Internal layouts shared by the host runtime (tds_api.cpp) and the HIP
// kernels (tds_kernels.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tds.h"

namespace tds {

// Query segment as the binary64 pair test reads it: start point, span,
// velocity and squared threshold (80 bytes, read wave-uniformly).
struct QRec64 {
    double t0, t1;
    double x0, y0, z0;
    double vx, vy, vz;
    double dd;
    double pad;
};

// Conservative binary32 region of a query segment: the ball of radius r
// about (cx, cy, cz) (relative to the index origin) that contains every point
// within d + band of the segment, with the slack the binary32 test needs
// (16 bytes).
struct alignas(16) QCube32 {
    float cx, cy, cz, r;
};

// A tile: sorted query segments [q0, q0 + nq) against entries [e0, e0 + ne).
// The entries are cut into nchunk chunks of echunk entries (a multiple of 64,
// the last chunk shorter); one work unit is one query segment against one
// chunk, so a tile holds nchunk * nq units, query-fastest.
struct Tile {
    int32_t q0, nq;
    int32_t e0, ne;
    int32_t nchunk, echunk;
    int32_t pad0, pad1;
};

// Entries per chunk when ne entries are cut into nchunk chunks: as even as
// possible, rounded up to whole waves of 64.
__host__ __device__ inline int chunk_entries(int ne, int nchunk) {
    int per = (ne + nchunk - 1) / (nchunk > 0 ? nchunk : 1);
    return (per + 63) & ~63;
}

// ------------------------------------------------ bins of an interval (Sec. 4)
// The candidate bins of an interval (a, b) are those whose temporal extent
// [start, end] overlaps it with positive length: start < b and end > a. The
// range runs from the first member of the first such bin to the last member
// of the last one. Bin starts are non-decreasing (bins are in t_start order)
// but bin ends are not, so three searches find them: j1 = the first bin whose
// running maximum end exceeds a (that bin itself ends after a); the last bin
// starting before b; and from there back to the last bin that also ends
// after a, found by descending a max-tree of the bin ends.
//
// The tree: P = the smallest power of two >= the number of bins; node k in
// [1, P) holds the largest end of its two children 2k and 2k+1, leaf P + j
// holds the end of bin j (-inf beyond the last bin).

// Largest j' <= j with end_j' > a, or -1.
__host__ __device__ inline int bins_last_end_above(const double *tree, int P, int j, double a) {
    int v = P + j;
    if (tree[v] > a) return j;
    while (v > 1) {
        if ((v & 1) && tree[v - 1] > a) {  // the left sibling holds one: its rightmost
            v -= 1;
            while (v < P) {
                v = 2 * v + 1;
                if (!(tree[v] > a)) v -= 1;
            }
            return v - P;
        }
        v >>= 1;
    }
    return -1;
}

// Smallest j' >= j with end_j' > a, or nb.
__host__ __device__ inline int bins_first_end_above(const double *tree, int P, int nb, int j, double a) {
    if (j >= nb) return nb;
    int v = P + j;
    if (tree[v] > a) return j;
    while (v > 1) {
        if (!(v & 1) && tree[v + 1] > a) {  // the right sibling holds one: its leftmost
            v += 1;
            while (v < P) {
                v = 2 * v;
                if (!(tree[v] > a)) v += 1;
            }
            return v - P;
        }
        v >>= 1;
    }
    return nb;
}

// First k in [0, n) with a[k] > x (a non-decreasing), n if none.
__host__ __device__ inline int first_above(const double *a, int n, double x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] > x) hi = mid; else lo = mid + 1;
    }
    return lo;
}
// Number of leading elements < x of a non-decreasing array.
__host__ __device__ inline int count_below(const double *a, int n, double x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// The candidate bins j1..j2 of (a, b); false when no bin overlaps it.
// bstart / bpend: bin starts and running maximum ends (searched, may be
// copies in LDS); tree: the max-tree of bin ends.
__host__ __device__ inline bool bins_of_interval(const double *bstart, const double *bpend,
                                                 const double *tree, int P, int nb, double a,
                                                 double b, int *j1, int *j2) {
    *j1 = first_above(bpend, nb, a);
    const int hi = count_below(bstart, nb, b) - 1;
    if (*j1 > hi) return false;
    *j2 = bins_last_end_above(tree, P, hi, a);  // >= j1: bin j1 ends after a
    return true;
}

// Segments of one t_start bin sorted in LDS by the bin sort; larger bins are
// ranked by counting over global memory.
constexpr int kSortLds = 2048;

// Unsigned bits of a binary64 value that order as the value does (-0 as +0).
__device__ __forceinline__ unsigned long long start_bits(double x) {
    x = x + 0.0;
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// The pair kernel splits a batch over its waves by cost rather than by work
// units (query segment x entry chunk): a pass over one chunk of a tile costs
// its nq segments plus a fixed overhead (loading the chunk and staging the
// first segments) and a further one per extra stage of 64 segments. Tiles of
// few segments are then no longer cheap for the waves that draw many of them.
#ifndef TDS_PASS_COST32
#define TDS_PASS_COST32 24
#endif
#ifndef TDS_STAGE_COST32
#define TDS_STAGE_COST32 4
#endif
#ifndef TDS_PASS_COST64
#define TDS_PASS_COST64 2
#endif
#ifndef TDS_STAGE_COST64
#define TDS_STAGE_COST64 0
#endif

// Overhead of one pass of a tile with nq segments, in work units.
__host__ __device__ inline long long pass_overhead(int nq, int pass_cost, int stage_cost) {
    return (long long)pass_cost + (long long)stage_cost * ((nq + 63) / 64 - 1);
}

// Cost of a whole tile: nchunk passes (0 for a tile without work).
__host__ __device__ inline long long tile_cost(int nq, int nchunk, int pass_cost, int stage_cost) {
    if (nq <= 0 || nchunk <= 0) return 0;
    return (long long)nchunk * ((long long)nq + pass_overhead(nq, pass_cost, stage_cost));
}

// A pair selected by the pair kernel: the query segment's caller index and
// the entry's sorted position.
struct Cand {
    uint32_t q, e;
};

// Device result record: the query segment's caller index, the entry's
// sorted position, the interval.
struct Hit24 {
    uint32_t q, e;
    double ta, tb;
};

// Selected pairs and hits live in slabs of kSlab records. Slab w < nwaves
// belongs to wave w of the pair launch, which fills it without atomics; a
// wave whose next selections do not fit its current slab takes a whole new
// slab from the spill slabs after the wave slabs (one atomic per 64 records
// at most) and leaves the old one partly filled. Every slab carries its own
// record count. Hit slab s holds the hits among selected-pair slab s, and
// the offsets k_emit writes give the position of each slab's hits in the
// dense output.
constexpr int kSlab = 64;
struct Slabs {
    Cand *cand;                    // nslabs * kSlab
    Hit24 *hits;                   // nslabs * kSlab
    int32_t *slab_n;               // selected pairs in each slab [nslabs]
    int32_t *slab_h;               // hits in each slab [nslabs]
    long long *hit_off;            // exclusive scan of slab_h [nslabs]
    unsigned long long *wave_ovl;  // overlapping pairs counted by each wave [nwaves]
    int32_t nwaves;                // waves of the pair launch (= wave slabs)
    int32_t pad;
    long long nslabs;              // slabs allocated (> nwaves)
};

// Device counters of one batch (zeroed at the start of the batch).
struct Counters {
    unsigned long long hits;
    unsigned long long cand;     // pairs selected by the pair kernel
    unsigned long long overlap;
    unsigned long long n_eval;
    unsigned long long n_overlap_exact;
    unsigned long long n_units;  // work units of the pair kernel
    unsigned int err;            // bit 0: invalid query segment
    unsigned int n_tiles;
    unsigned int n_sorted;       // query segments placed in tiles
    unsigned int big_bins;       // t_start bins with more than kSortLds segments (sorted tilings)
    unsigned long long spill;    // spill slabs taken by the pair kernel (may exceed nslabs - nwaves)
    unsigned long long n_slabs;  // slabs in use after the refine
};

// Index arrays in device memory (sorted by t_start).
struct DevIndex {
    int64_t n;
    int32_t nb;  // non-empty bins
    int32_t m;   // bins as requested
    double t_first, width;
    const double *t0, *t1, *x0, *y0, *z0, *vx, *vy, *vz;
    const float4 *ecen;   // entry ball in binary32 relative to the origin: centre c
                          // (the segment's midpoint) and e2 = |c|^2 (rounded)
    const float *erad;    // entry ball radius: half the segment's length plus the
                          // entry's share of the error band and of c's rounding
    const int32_t *orig;  // caller index of each sorted entry
    const int64_t *traj;  // trajectory id of each sorted entry
    const double *t1s;    // t_end, sorted independently (overlap counts)
    const double *bstart, *bpend;  // per non-empty bin: min t_start, prefix max of t_end
    const int32_t *bfirst, *blast;
    const double *btree;  // max-tree of the bin ends (2 * bleaf values)
    int32_t bleaf;        // leaves of btree: the smallest power of two >= nb
    int32_t pad_b;
    double ox, oy, oz;    // origin of the binary32 coordinates (per-axis median of
                          // the database's end points)
};

// Error band of the binary32 filter. A binary64 hit of a pair implies that
// the exact distance is within d + 8 sqrt(eps) (d + ext_q + ext_e) at some
// common time (ext: |dx| + |dy| + |dz| of a segment; eps = 2^-52, so the
// factor is 2^-23); kBandRel = 2^-20 is 8 times that. Positions carry a few
// ulps of their coordinates' magnitude, covered by kBandAbs per unit of
// magnitude. The band of a pair is split between its two sides: the query
// cube is widened by kBandRel (d + ext_q) + kBandAbs (1 + d + mag_q + ext_q),
// each entry's stored half-width by kBandRel ext_e + kBandAbs (mag_e +
// ext_e), so the band follows the entries of each chunk rather than the
// largest entry of the database. The binary32 comparison itself rounds by at
// most 2^-23 (r + H) near the threshold; both sides carry kCmpSlack = 2^-20
// of their half-width for it.
constexpr double kBandRel = 0x1p-20;
constexpr double kBandAbs = 0x1p-40;
constexpr double kCmpSlack = 0x1p-20;
// The binary32 test of a query ball (centre C, radius r) against the entries
// of a chunk (centres c, radii at most H) passes a pair when
//   s = e2 + (-2C).c <= T = (r + H)^2 - |C|^2 + kDotSlack (e2max + |C|^2),
// s evaluated as one multiply-add per axis; |C - c|^2 = |c|^2 - 2C.c + |C|^2,
// and the rounding of e2 and of the three multiply-adds is at most
// 4 * 2^-24 (|c|^2 + 2|c||C|) <= 2^-21 (e2max + |C|^2) (with e2max the largest
// e2 of the chunk), half of kDotSlack. T is evaluated in binary64 and rounded
// up to binary32, so balls that meet always pass.
constexpr double kDotSlack = 0x1p-20;
// Coordinates relative to the origin (and radii) up to this magnitude take
// part in the binary32 test (|c|^2 and 2|C||c| stay far below the binary32
// range); beyond it an entry or query passes every pair.
constexpr double kSphereLimit = 0x1p60;

// Range buckets per first candidate bin: spans of 0, 1, 2 and >= 3 bins.
constexpr int kSpanClasses = 4;
// Each bucket may count its query segments on kBucketSub counters (segment i
// on counter i % kBucketSub) to spread atomics on one bucket over several
// addresses; the bucket's segments stay contiguous in the sorted order. One
// counter measured fastest on MI355X (the histogram is not bound by them).
constexpr int kBucketSub = 1;

// Query-side buffers of one batch (device).
struct DevBatch {
    int32_t nq;
    int32_t s;            // periodic tile size
    int32_t chunk;        // entries per chunk (at most)
    int32_t tiling;
    int32_t nbuckets;
    int32_t ntiles_cap;
    int32_t count_overlap;      // exact overlap count in the query preparation
    int32_t pass_cost;          // pair-kernel cost of a chunk pass beyond its segments
    int32_t stage_cost;         // ... and of each further stage of 64 segments
    int32_t pad;
    QRec64 *rec;          // caller order
    QCube32 *box;         // caller order
    int32_t *first, *last;      // caller order candidate range (last < first: empty)
    int32_t *first_s, *last_s;  // sorted order
    int32_t *key;               // caller order bucket (-1: no candidates)
    int32_t *perm;              // perm[sorted position] = caller index (+2 spare slots)
    int32_t *qrank;             // caller order rank within its bucket
    int32_t *bcount, *bq_off;   // per bucket and sub-counter (kBucketSub each)
    int32_t *bj2;               // per bucket
    Tile *tiles;
    long long *units;           // per tile (periodic)
    long long *unit_off;        // exclusive scan of units per tile (+ total)
    long long *cost_off;        // exclusive scan of tile costs (+ total)
    // Sorted tilings (Periodic, greedy): the counting sort writes each
    // segment's order key here by bucket position instead of perm, and the
    // bin sort places it exactly; null for range tiling.
    unsigned long long *skey;   // order bits of t_start [nq]
    int32_t *sidx;              // caller index [nq]
    unsigned long long *tkey;   // pieces of bins too large for LDS, sorted [nq]
    int32_t *tidx;              // ... their caller indices [nq]
    Counters *ctr;
};

// Work arrays of the trajectory merge (n hits each).
// One hit of the trajectory merge as a whole sort key (small merges).
struct TrajKey {
    int64_t qt, et;
    double ta, tb;
};

// Merges of at most this many hits sort TrajKey records once with a
// comparison merge sort; larger ones use three stable radix sorts.
constexpr long long kTrajOneSortMax = 1LL << 16;
// Merges of at most this many hits rank each key by counting the keys that
// precede it (n^2 comparisons spread over the whole GPU), scatter, and merge
// in one workgroup: four launches instead of a dozen.
constexpr long long kTrajRankMax = 8192;

// t_b with a pair-start flag: the element of the segmented running maximum.
struct SegMax {
    double v;
    int32_t f, pad;
};

struct TrajBufs {
    int64_t *qt, *et;                  // trajectory ids, hit order
    double *ta, *tb;                   // interval, hit order
    unsigned long long *key_a, *key_b; // radix-sort keys
    int32_t *idx_a, *idx_b;            // permutations
    int32_t *flag, *start, *mid;       // sorted order: pair start, run start, record no.
    double *sta;                       // sorted order: t_a
    SegMax *seg_in, *seg_out;          // sorted order: (t_b, pair start), running maximum of t_b
    TrajKey *kin, *kout;               // small merges: hit order, sorted order
};

enum : int { kModeFP64 = 0, kModeFP32Refine = 1 };
enum : int { kTilePeriodic = 0, kTileRange = 1, kTileGreedyMin = 2, kTileGreedyMax = 3 };

// Work arrays of the GreedySetSplit tiling (nq = query segments of the batch).
struct GreedyBufs {
    unsigned long long *kin;         // DevBatch::skey [nq]
    int32_t *vout;                   // DevBatch::sidx [nq]
    unsigned long long *tkey;        // DevBatch::tkey [nq]
    int32_t *tidx;                   // DevBatch::tidx [nq]
    uint8_t *flag;                   // run start by sorted position [nq rounded up to 16]
    int32_t *gpos;                   // first sorted position of each run (group) [nq + 1]
    int32_t *jump;                   // levels x stride: the 2^k-th next batch start
    int32_t *mark;                   // level at which a group was found a batch start [nq + 1]
    int32_t *gb;                     // first group of each batch [nq + 1]
    long long *tev;                  // interactions of each tile [nq]
    int32_t *cnt;                    // [0] groups, [1] batches
    double *gmax;                    // largest t_end of the group starting at each position [nq]
    int32_t stride;                  // nq + 1
    int32_t levels;                  // doubling levels the jump buffer holds
};

// Launchers (tds_kernels.hip). All enqueue on `st`, return hipError_t.
hipError_t launch_ingest(const double *const *raw, int64_t n, const int32_t *perm_sorted,
                         const int64_t *traj_raw, double *t0, double *t1, double *x0, double *y0,
                         double *z0, double *vx, double *vy, double *vz, float4 *ecen,
                         float *erad, double ox, double oy, double oz, int32_t *orig,
                         int64_t *traj, hipStream_t st);
// ev_start (optional) records the start of the first kernel. With zero
// false the per-bucket counters and the batch counters are taken as already
// cleared (the previous batch's last kernel, k_emit, cleared them, see NextClear).
hipError_t launch_prepare(const double *const *q, const double *d, DevBatch b, DevIndex ix,
                          hipStream_t st, hipEvent_t ev_start = nullptr, bool zero = true);
// What the last kernel of a batch clears for the next batch of the same
// query handle (null ctr: nothing): the next batch's counters and the first
// nbuckets per-bucket counters (bcount = 0, bj2 = -1).
struct NextClear {
    Counters *ctr;
    int32_t *bcount;
    int32_t *bj2;
    int32_t nbuckets;
    int32_t pad;
};
// Workgroups of the pair launch: `grid` when > 0, else one per resident slot
// (persistent launch). Slabs.nwaves must be pair_grid(...) * block / 64.
int pair_grid(int mode, int block, int grid, int kernel_overlap);
// ev0 / ev1 (optional) record the start and the end of the pair kernel.
hipError_t launch_pair(DevBatch b, DevIndex ix, int mode, int block, int grid, int kernel_overlap,
                       Slabs sl, hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Refine the selected pairs into hit slabs, then scan the hit counts;
// ev_stop (optional) records the end of the scan.
// host_out (optional): pinned host copy of the final counters, written by the scan.
hipError_t launch_refine(DevBatch b, DevIndex ix, Slabs sl, hipStream_t st,
                         hipEvent_t ev_stop = nullptr);
// The batch's last kernel: hit offsets, the dense caller-index records of the
// first n hits (none when out_hits is null), the final counters (also to
// host_out when not null) and the clearing of the next batch's counters.
hipError_t launch_emit(Slabs sl, Counters *ctr, int64_t n, DevIndex ix, void *out_hits,
                       int count_ovl, Counters *host_out, NextClear next, hipStream_t st,
                       hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
hipError_t launch_reset_counters(Counters *c, int all, hipStream_t st);
// Trajectory merge (tds_traj.hip): temp bytes for n hits, and the launch
// (n > 0 hits; writes the merged records to `out` and their number to *total).
size_t traj_temp_bytes(long long n);
// Exact (t_start, caller index) order of the bucketed query segments (after
// launch_prepare with a Periodic or greedy tiling, b.skey / b.sidx set):
// perm, first_s and last_s in that order (tds_greedy.hip).
hipError_t launch_bucket_sort(DevBatch b, hipStream_t st);
// Periodic tiles over the sorted order and their unit and cost offsets.
hipError_t launch_periodic(DevBatch b, DevIndex ix, hipStream_t st);
// GreedySetSplit tiles (after launch_bucket_sort): builds the runs, the
// batch chain and the tiles, and scans the work units.
hipError_t launch_greedy(DevBatch b, GreedyBufs g, DevIndex ix, int bound, int is_max,
                         hipStream_t st);
hipError_t launch_traj_merge(Slabs sl, const Counters *ctr, long long n, const int64_t *qtraj,
                             DevIndex ix, TrajBufs t, void *temp,
                             size_t temp_bytes, tds_traj_hit *out, long long *total,
                             hipStream_t st);
int chunk_for(int mode, int block);
int nbuckets_for(int tiling, int nb, int m);
// Sets the calling thread's tds_last_error message; returns code.
int set_error(int code, const char *msg);

}  // namespace tds
