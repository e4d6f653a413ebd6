// Internal layouts shared by the host runtime (tds_api.cpp) and the HIP
// kernels (tds_kernels.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Conservative binary32 box of a query segment: span rounded outward and
// spatial bounding box widened by d + band and rounded outward (32 bytes).
struct alignas(32) QBox32 {
    float t0, t1;
    float xlo, xhi, ylo, yhi, zlo, zhi;
};

// A tile: sorted query segments [q0, q0 + nq) against entries [e0, e0 + ne).
struct Tile {
    int32_t q0, nq;
    int32_t e0, ne;
};

// Device result record: positions in sorted query / sorted entry order.
struct Hit24 {
    uint32_t q, e;
    double ta, tb;
};

// Device counters of one batch (zeroed before the pair kernel).
struct Counters {
    unsigned long long hits;
    unsigned long long refine;
    unsigned long long overlap;
    unsigned long long n_eval;
    unsigned long long n_overlap_exact;
    unsigned int err;           // bit 0: invalid query segment
    unsigned int n_tiles;
    unsigned int n_items;
    unsigned int pad;
};

// Index arrays in device memory (sorted by t_start).
struct DevIndex {
    int64_t n;
    int32_t nb;  // non-empty bins
    int32_t pad;
    const double *t0, *t1, *x0, *y0, *z0, *vx, *vy, *vz;
    const float4 *boxa;   // (t0 down, t1 up, xlo down, xhi up)
    const float4 *boxb;   // (ylo down, yhi up, zlo down, zhi up)
    const int32_t *orig;  // caller index of each sorted entry
    const int64_t *traj;  // trajectory id of each sorted entry
    const double *t0s;    // t_start, sorted (for overlap counts)
    const double *t1s;    // t_end, sorted independently
    const double *bstart, *bpend;  // per non-empty bin: min t_start, prefix max of t_end
    const int32_t *bfirst, *blast;
    double band_rel;      // box slack per unit of (d + query extent + ext_max)
    double band_abs;      // box slack per unit of coordinate magnitude
    double ext_max;       // largest |dx|+|dy|+|dz| of an entry segment
    double mag_max;       // largest |coordinate| of an entry end point
};

// Query-side buffers of one batch (device).
struct DevBatch {
    int32_t nq;
    int32_t s;            // tile size
    int32_t tiling;
    int32_t chunk;
    QRec64 *rec;          // caller order
    QBox32 *box;          // caller order
    QRec64 *rec_s;        // sorted order
    QBox32 *box_s;        // sorted order
    int32_t *first, *last;      // caller order candidate range (last < first: empty)
    int32_t *first_s, *last_s;  // sorted order
    unsigned long long *key_in, *key_out;
    int32_t *val_in, *perm;     // perm[sorted position] = caller index
    int32_t *head;              // tile-head flags, then their exclusive scan
    int32_t *tile_of_head;
    Tile *tiles;
    int32_t *items;             // work items per tile (zero past the last tile)
    int32_t *item_off;          // exclusive scan of items
    Counters *ctr;
};

enum : int { kModeFP64 = 0, kModeFP32Refine = 1 };
enum : int { kTilePeriodic = 0, kTileRange = 1 };

// Launchers (tds_kernels.hip). All enqueue on `st`, return hipError_t.
hipError_t launch_ingest(const double *const *raw, int64_t n, const int32_t *perm_sorted,
                         const int64_t *traj_raw, DevIndex ix, double *t0, double *t1, double *x0,
                         double *y0, double *z0, double *vx, double *vy, double *vz, float4 *boxa,
                         float4 *boxb, int32_t *orig, int64_t *traj, hipStream_t st);
hipError_t launch_qprep(const double *const *q, const double *d, DevBatch b, DevIndex ix,
                        double t_first, double t_span, hipStream_t st);
hipError_t sort_temp_bytes(int n, size_t *bytes);
hipError_t launch_sort(void *temp, size_t temp_bytes, DevBatch b, int end_bit, hipStream_t st);
hipError_t launch_gather(DevBatch b, DevIndex ix, hipStream_t st);
hipError_t scan_temp_bytes(int n, size_t *bytes);
hipError_t launch_scan(void *temp, size_t temp_bytes, const int32_t *in, int32_t *out, int n,
                       hipStream_t st);
hipError_t launch_tiles(DevBatch b, hipStream_t st);
hipError_t launch_pair(DevBatch b, DevIndex ix, int mode, int block, int grid, int count_overlap,
                       Hit24 *out, unsigned long long cap, hipStream_t st);
hipError_t launch_translate(const Hit24 *in, int64_t n, const int32_t *perm, DevIndex ix,
                            void *out_hits, hipStream_t st);
hipError_t launch_zero_counters(Counters *c, hipStream_t st);
int ept_for(int mode, int block);
int chunk_for(int mode, int block);

}  // namespace tds
