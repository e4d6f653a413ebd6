// HIP kernels of the distance-threshold search for CDNA4 (gfx950).
//
// Layout: entries sorted by t_start as a structure of arrays (one lane per
// entry, coalesced 64-lane loads); query segments of a batch grouped into
// tiles by a counting sort on their candidate bin range (or on their t_start
// bin for the paper's Periodic batches) and read wave-uniformly through the
// scalar cache; a persistent pair kernel splits the batch's work units
// (query segment x chunk of candidate entries) evenly over the resident
// waves, with no atomics and no workgroup barriers.
//
// The binary64 decision follows the paper's Alg. 1 (temporal intersection,
// then the time interval within d from the degree-two polynomial of the
// squared distance) in one fixed evaluation order:
//   tlo = max(q.t0, e.t0), thi = min(q.t1, e.t1), compared only if tlo < thi
//   T = thi - tlo, tq = tlo - q.t0, te = tlo - e.t0
//   D_k = fma(q.v_k, tq, q.p0_k) - fma(e.v_k, te, e.p0_k), V_k = q.v_k - e.v_k
//   a = fma(Vz,Vz, fma(Vy,Vy, Vx*Vx)), B = fma(Dz,Vz, fma(Dy,Vy, Dx*Vx)),
//   c = fma(Dz,Dz, fma(Dy,Dy, fma(Dx,Dx, -dd)))
//   hit = c <= 0 || fma(fma(a,T,B+B),T,c) <= 0
//         || (B < 0 && fma(a,T,B) > 0 && fma(B,B,-(a*c)) >= 0)
// Built with -ffp-contract=off: every fma is explicit, nothing is fused or
// reassociated behind the source's back.
#include <hip/hip_ext.h>

#include <type_traits>

#include "tds_internal.h"


// Launch with optional start / stop events attached to the dispatch itself
// (hipExtLaunchKernelGGL), which adds no packets to the stream; a separate
// hipEventRecord around each kernel measured about 5 us per event here.
#define TDS_LAUNCH_EV(start, stop, kernel, grid, block, shm, st, ...)                          \
    do {                                                                                     \
        if ((start) || (stop))                                                               \
            hipExtLaunchKernelGGL(kernel, grid, block, shm, st, start, stop, 0, __VA_ARGS__); \
        else                                                                                 \
            hipLaunchKernelGGL(kernel, grid, block, shm, st, __VA_ARGS__);                   \
    } while (0)

namespace tds {

#define TDS_LAUNCH_CHECK() return hipGetLastError()

// max / min of finite values (the result is one of the operands; the sign
// of a zero result may differ from a compare-and-select, which no decision
// below can observe).
__device__ __forceinline__ double dmx(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ double dmn(double a, double b) { return __builtin_fmin(a, b); }

// Smallest binary32 value >= a binary64 value.
__device__ __forceinline__ float f32_up(double x) {
    float f = (float)x;
    return ((double)f < x) ? nextafterf(f, INFINITY) : f;
}


__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// --------------------------------------------------------------- ingest
// Ball of a segment for the binary32 test, relative to the origin (ox, oy,
// oz): centre c = the midpoint rounded to binary32, and a radius that holds
// the whole segment around c (half its length plus the distance from the
// exact midpoint to c), widened by `widen` and by kCmpSlack of itself, rounded
// up. Returns false when the ball is beyond the binary32 test's range.
__device__ __forceinline__ bool segment_ball(double a0, double b0, double c0, double a1, double b1,
                                             double c1, double ox, double oy, double oz,
                                             double widen, float &cx, float &cy, float &cz,
                                             float &r) {
    const double mx = 0.5 * (a0 + a1) - ox, my = 0.5 * (b0 + b1) - oy, mz = 0.5 * (c0 + c1) - oz;
    const double dx = a1 - a0, dy = b1 - b0, dz = c1 - c0;
    const double half = 0.5 * sqrt(dx * dx + dy * dy + dz * dz);
    const double reach = dmx(dmx(fabs(mx), fabs(my)), fabs(mz)) + half + widen;
    if (!(reach <= kSphereLimit)) return false;
    cx = (float)mx;
    cy = (float)my;
    cz = (float)mz;
    // m - c is exact in binary64 (c is m rounded to 24 bits)
    const double ex = mx - (double)cx, ey = my - (double)cy, ez = mz - (double)cz;
    const double rr = half + sqrt(ex * ex + ey * ey + ez * ez) + widen;
    r = f32_up(rr + kCmpSlack * rr);
    return true;
}

// One thread per sorted position p: gather the caller's segment perm[p],
// compute its velocity and its conservative binary32 ball.
__global__ void k_ingest(const double *__restrict__ rx0, const double *__restrict__ ry0,
                         const double *__restrict__ rz0, const double *__restrict__ rt0,
                         const double *__restrict__ rx1, const double *__restrict__ ry1,
                         const double *__restrict__ rz1, const double *__restrict__ rt1,
                         int64_t n, const int32_t *__restrict__ perm,
                         const int64_t *__restrict__ traj_raw, double *t0, double *t1, double *x0,
                         double *y0, double *z0, double *vx, double *vy, double *vz, float4 *ecen,
                         float *erad, double ox, double oy, double oz, int32_t *orig,
                         int64_t *traj) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int32_t i = perm[p];
    double a0 = rx0[i], b0 = ry0[i], c0 = rz0[i], s0 = rt0[i];
    double a1 = rx1[i], b1 = ry1[i], c1 = rz1[i], s1 = rt1[i];
    double dt = s1 - s0;
    t0[p] = s0;
    t1[p] = s1;
    x0[p] = a0;
    y0[p] = b0;
    z0[p] = c0;
    vx[p] = (a1 - a0) / dt;
    vy[p] = (b1 - b0) / dt;
    vz[p] = (c1 - c0) / dt;
    // the entry's share of the error band (magnitude of its own coordinates)
    const double mag = dmx(dmx(dmx(fabs(a0), fabs(a1)), dmx(fabs(b0), fabs(b1))), dmx(fabs(c0), fabs(c1)));
    const double ext = fabs(a1 - a0) + fabs(b1 - b0) + fabs(c1 - c0);
    float cx, cy, cz, r;
    float4 e;
    if (segment_ball(a0, b0, c0, a1, b1, c1, ox, oy, oz, kBandRel * ext + kBandAbs * (mag + ext), cx,
                     cy, cz, r)) {
        const double e2 = (double)cx * cx + (double)cy * cy + (double)cz * cz;
        e = make_float4(cx, cy, cz, (float)e2);
    } else {  // beyond the binary32 test's range: s = -inf passes every query
        e = make_float4(0.0f, 0.0f, 0.0f, -INFINITY);
        r = 0.0f;
    }
    ecen[p] = e;
    erad[p] = r;
    orig[p] = i;
    traj[p] = traj_raw ? traj_raw[i] : (int64_t)i;
}

hipError_t launch_ingest(const double *const *raw, int64_t n, const int32_t *perm_sorted,
                         const int64_t *traj_raw, double *t0, double *t1, double *x0, double *y0,
                         double *z0, double *vx, double *vy, double *vz, float4 *ecen,
                         float *erad, double ox, double oy, double oz, int32_t *orig,
                         int64_t *traj, hipStream_t st) {
    if (n == 0) return hipSuccess;
    int blk = 256;
    int64_t grid = (n + blk - 1) / blk;
    hipLaunchKernelGGL(k_ingest, dim3((unsigned)grid), dim3(blk), 0, st, raw[0], raw[1], raw[2],
                       raw[3], raw[4], raw[5], raw[6], raw[7], n, perm_sorted, traj_raw, t0, t1, x0,
                       y0, z0, vx, vy, vz, ecen, erad, ox, oy, oz, orig, traj);
    TDS_LAUNCH_CHECK();
}

// --------------------------------------------------------------- prepare
int nbuckets_for(int tiling, int nb, int m) {
    return tiling == kTileRange ? (nb > 0 ? nb * kSpanClasses : 1) : (m > 0 ? m : 1);
}

// Clears the per-bucket counters and the batch counters.
__global__ void k_zero_batch(DevBatch b) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (int k = i; k < b.nbuckets; k += gridDim.x * blockDim.x) {
#pragma unroll
        for (int c = 0; c < kBucketSub; ++c) b.bcount[k * kBucketSub + c] = 0;
        b.bj2[k] = -1;
    }
    if (i == 0) {
        Counters z = {};
        *b.ctr = z;
    }
}

// Bin tables up to this size (16 bytes per bin) are staged in LDS by k_qprep.
constexpr int kQprepLdsBins = 2048;
// Groups of lanes with a common bucket that k_qprep ranks with one atomic each.
constexpr int kRankGroups = 4;

// Number of leading elements < x of a non-decreasing array.
__device__ __forceinline__ int64_t count_less(const double *a, int64_t n, double x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}
// Number of leading elements <= x of a non-decreasing array.
__device__ __forceinline__ int64_t count_leq(const double *a, int64_t n, double x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// One thread per query segment (caller order): validate it, build its
// binary64 record and binary32 box, find its candidate range (Sec. 4: the
// bins whose temporal extent overlaps its span) with two binary searches
// over the non-empty bins, and count it into its bucket.
__global__ void k_qprep(const double *__restrict__ qx0, const double *__restrict__ qy0,
                        const double *__restrict__ qz0, const double *__restrict__ qt0,
                        const double *__restrict__ qx1, const double *__restrict__ qy1,
                        const double *__restrict__ qz1, const double *__restrict__ qt1,
                        const double *__restrict__ qd, DevBatch b, DevIndex ix) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    // the segment's inputs are requested before the block waits for the bins
    double a0 = 0.0, b0 = 0.0, c0 = 0.0, s0 = 0.0, a1 = 0.0, b1 = 0.0, c1 = 0.0, s1 = 1.0;
    double d = 0.0;
    if (i < b.nq) {
        a0 = qx0[i], b0 = qy0[i], c0 = qz0[i], s0 = qt0[i];
        a1 = qx1[i], b1 = qy1[i], c1 = qz1[i], s1 = qt1[i];
        d = qd[i];
    }
    // Small bin tables are searched in LDS (one coalesced copy per block).
    extern __shared__ double s_bins[];  // running maximum ends, then starts
    const bool in_lds = ix.nb <= kQprepLdsBins;
    if (in_lds) {
        for (int k = threadIdx.x; k < ix.nb; k += blockDim.x) {
            s_bins[k] = ix.bpend[k];
            s_bins[ix.nb + k] = ix.bstart[k];
        }
        __syncthreads();
    }
    unsigned long long novl = 0;
    int key = -1, kj2 = -1;  // bucket, and the last bin for the open span class
    if (i < b.nq) {
        bool ok = isfinite(a0) && isfinite(b0) && isfinite(c0) && isfinite(s0) && isfinite(a1) &&
                  isfinite(b1) && isfinite(c1) && isfinite(s1) && isfinite(d) && d >= 0.0 &&
                  s1 > s0;
        if (!ok) {
            atomicOr(&b.ctr->err, 1u);
            s0 = 0.0;
            s1 = 1.0;
            a0 = b0 = c0 = a1 = b1 = c1 = 0.0;
            d = 0.0;
        }
        double dt = s1 - s0;
        QRec64 r;
        r.t0 = s0;
        r.t1 = s1;
        r.x0 = a0;
        r.y0 = b0;
        r.z0 = c0;
        r.vx = (a1 - a0) / dt;
        r.vy = (b1 - b0) / dt;
        r.vz = (c1 - c0) / dt;
        r.dd = d * d;
        r.pad = 0.0;
        b.rec[i] = r;

        // Ball of the segment widened by d plus the query's share of the
        // error band (the binary64 decision's own rounding and that of
        // computed positions): every point within d of the segment lies in
        // it. An entry ball of radius r_e that it does not meet holds no
        // point of the entry segment, so no hit.
        double ext = fabs(a1 - a0) + fabs(b1 - b0) + fabs(c1 - c0);
        double mag = dmx(dmx(fabs(a0), fabs(a1)), dmx(dmx(fabs(b0), fabs(b1)), dmx(fabs(c0), fabs(c1))));
        double w = d + kBandRel * (d + ext) + kBandAbs * (1.0 + d + mag + ext);
        QCube32 bx;
        if (!segment_ball(a0, b0, c0, a1, b1, c1, ix.ox, ix.oy, ix.oz, w, bx.cx, bx.cy, bx.cz, bx.r)) {
            // beyond the binary32 test's range: pass every entry
            bx.cx = bx.cy = bx.cz = 0.0f;
            bx.r = INFINITY;
        }
        b.box[i] = bx;

        // Candidate bins (Sec. 4): those whose extent overlaps (t0, t1) with
        // positive length, j1 .. j2 (searches in LDS when the bins fit).
        int j1 = 0, j2 = -1;
        const bool found =
            in_lds ? bins_of_interval(s_bins + ix.nb, s_bins, ix.btree, ix.bleaf, ix.nb, s0, s1, &j1, &j2)
                   : bins_of_interval(ix.bstart, ix.bpend, ix.btree, ix.bleaf, ix.nb, s0, s1, &j1, &j2);
        bool any = ok && found;
        b.first[i] = any ? ix.bfirst[j1] : 0;
        b.last[i] = any ? ix.blast[j2] : -1;

        if (b.count_overlap && ok)
            novl = (unsigned long long)(count_less(ix.t0, ix.n, s1) - count_leq(ix.t1s, ix.n, s0));

        if (b.tiling == kTileRange) {
            if (any) {
                int cls = min(j2 - j1, kSpanClasses - 1);
                key = j1 * kSpanClasses + cls;
                if (cls == kSpanClasses - 1) kj2 = j2;
            }
        } else if (any) {  // Periodic and greedy: segments with candidates, by t_start bin
            double u = floor((s0 - ix.t_first) / ix.width);
            key = u <= 0.0 ? 0 : (u >= (double)(b.nbuckets - 1) ? b.nbuckets - 1 : (int)u);
        }
        b.key[i] = key;
    }
    // Rank within the bucket. Returning atomics on one address serialize, so
    // lanes of a wave that share a bucket (up to kRankGroups groups, most
    // often all of them) take their ranks with one atomic per group; the rest
    // take one each. The open span class's last bin goes up the same way.
    static_assert(kBucketSub == 1, "grouped ranks assume one counter per bucket");
    {
        const int lane = (int)lane_id();
        bool done = key < 0;
        int rank = 0;
        for (int it = 0; it < kRankGroups; ++it) {
            const unsigned long long act = __ballot(!done);
            if (act == 0ull) break;
            const int leader = __ffsll((long long)act) - 1;
            const int kl = __shfl(key, leader);
            const bool mine = !done && key == kl;
            const unsigned long long m = __ballot(mine);
            // a lone lane: the keys of this wave differ, one atomic each is as cheap
            if (__popcll(m) == 1 && it == 0) break;
            int jm = mine ? kj2 : -1;  // the group's largest last bin
            for (int off = 32; off > 0; off >>= 1) jm = max(jm, __shfl_xor(jm, off));
            int base = 0;
            if (lane == leader) {
                base = atomicAdd(&b.bcount[kl], __popcll(m));
                if (jm >= 0) atomicMax(&b.bj2[kl], jm);
            }
            base = __shfl(base, leader);
            if (mine) {
                rank = base + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                done = true;
            }
        }
        if (!done) {
            rank = atomicAdd(&b.bcount[key], 1);
            if (kj2 >= 0) atomicMax(&b.bj2[key], kj2);
        }
        if (i < b.nq) b.qrank[i] = key >= 0 ? rank : 0;
    }
    novl = wave_sum_u64(novl);
    if (lane_id() == 0 && novl) atomicAdd(&b.ctr->n_overlap_exact, novl);
}

// Exclusive scan of one value per thread over a block of BLOCK threads;
// returns the prefix and writes the block total to *total.
template <int BLOCK>
__device__ __forceinline__ long long block_exclusive_scan(long long v, long long *total) {
    __shared__ long long warp_sums[BLOCK / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    long long incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        long long y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    if (lane == 63) warp_sums[w] = incl;
    __syncthreads();
    if (w == 0) {
        long long s = lane < BLOCK / 64 ? warp_sums[lane] : 0;
        for (int off = 1; off < 64; off <<= 1) {
            long long y = __shfl_up(s, off);
            if (lane >= off) s += y;
        }
        if (lane < BLOCK / 64) warp_sums[lane] = s;  // inclusive over warps
    }
    __syncthreads();
    long long before = w > 0 ? warp_sums[w - 1] : 0;
    *total = warp_sums[BLOCK / 64 - 1];
    __syncthreads();
    return before + incl - v;
}

// Four exclusive scans over the block at once (one value of each per
// thread): the wave-level steps of the four run side by side and the
// warp totals of value k are scanned by wave k, so the four cost about one.
template <int BLOCK>
__device__ __forceinline__ void block_exclusive_scan4(const long long (&v)[4], long long (&run)[4],
                                                      long long (&total)[4]) {
    static_assert(BLOCK / 64 >= 4 && BLOCK / 64 <= 64, "one wave per value, one lane per wave");
    __shared__ long long warp_sums[4][BLOCK / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    long long incl[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) incl[k] = v[k];
    for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const long long y = __shfl_up(incl[k], off);
            if (lane >= off) incl[k] += y;
        }
    }
    if (lane == 63) {
#pragma unroll
        for (int k = 0; k < 4; ++k) warp_sums[k][w] = incl[k];
    }
    __syncthreads();
    if (w < 4) {
        long long s = lane < BLOCK / 64 ? warp_sums[w][lane] : 0;
        for (int off = 1; off < 64; off <<= 1) {
            const long long y = __shfl_up(s, off);
            if (lane >= off) s += y;
        }
        if (lane < BLOCK / 64) warp_sums[w][lane] = s;  // inclusive over warps
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        total[k] = warp_sums[k][BLOCK / 64 - 1];
        run[k] = (w > 0 ? warp_sums[k][w - 1] : 0) + incl[k] - v[k];
    }
    __syncthreads();
}

// Candidate range of a range bucket (all its queries share it).
__device__ __forceinline__ void bucket_range(const DevBatch &b, const DevIndex &ix, int k,
                                             int *e0, int *ne) {
    int j1 = k / kSpanClasses, cls = k - j1 * kSpanClasses;
    int j2 = cls < kSpanClasses - 1 ? j1 + cls : b.bj2[k];
    *e0 = ix.bfirst[j1];
    *ne = ix.blast[j2] - ix.bfirst[j1] + 1;
}

// One block: exclusive scan of the bucket counts (sorted offsets). For range
// tiling each non-empty bucket is a tile of nchunk * nq work units, and the
// tiles' unit offsets are scanned here as well.
constexpr int kScanBlock = 1024;
// Each thread takes a contiguous run of buckets; runs of up to kBucketRun
// have their counts and ranges read with loads issued together and kept in
// registers for both passes (longer runs read them again).
constexpr int kBucketRun = 4;

// The scan of one workgroup of kScanBlock threads. publish: write the
// offsets (bq_off), the tiles, their unit and cost offsets and the counters;
// s_off (optional, LDS): the offset of every bucket, for the scatter of the
// same workgroup.
__device__ __forceinline__ void bucket_scan_body(const DevBatch &b, const DevIndex &ix, int *s_off,
                                                 bool publish) {
    const int n = b.nbuckets;
    const int per = (n + kScanBlock - 1) / kScanBlock;
    const int lo = min(n, (int)threadIdx.x * per), hi = min(n, lo + per);
    const bool range = publish && b.tiling == kTileRange;
    const bool held = per <= kBucketRun;
    int hc[kBucketRun], he0[kBucketRun], hne[kBucketRun];
    auto count_of = [&](int k) {
        int c = 0;
#pragma unroll
        for (int j = 0; j < kBucketSub; ++j) c += b.bcount[k * kBucketSub + j];
        return c;
    };
    if (held) {
        int j2r[kBucketRun];
#pragma unroll
        for (int r = 0; r < kBucketRun; ++r) {
            const int k = lo + r;
            hc[r] = k < hi ? count_of(k) : 0;
            he0[r] = hne[r] = 0;
            j2r[r] = -1;
            if (range && k < hi) {
                const int j1 = k / kSpanClasses, cls = k - j1 * kSpanClasses;
                j2r[r] = cls < kSpanClasses - 1 ? j1 + cls : b.bj2[k];
                he0[r] = ix.bfirst[j1];
            }
        }
#pragma unroll
        for (int r = 0; r < kBucketRun; ++r)
            if (range && lo + r < hi && hc[r] > 0) hne[r] = ix.blast[j2r[r]] - he0[r] + 1;
    }
    auto get = [&](int r, int *c, int *e0, int *ne) {  // bucket lo + r
        if (held) {
            *c = hc[r];
            *e0 = he0[r];
            *ne = hne[r];
        } else {
            *c = count_of(lo + r);
            *e0 = *ne = 0;
            if (range && *c > 0) bucket_range(b, ix, lo + r, e0, ne);
        }
    };
    long long c_sum = 0, t_sum = 0, u_sum = 0, k_sum = 0;
    unsigned long long ev = 0;
    auto tally = [&](int r) {
        int c, e0, ne;
        get(r, &c, &e0, &ne);
        c_sum += c;
        if (publish && b.tiling != kTileRange && c > kSortLds) atomicAdd(&b.ctr->big_bins, 1u);
        if (range && c > 0) {
            const int nch = (ne + b.chunk - 1) / b.chunk;
            t_sum += 1;
            u_sum += (long long)nch * c;
            k_sum += tile_cost(c, nch, b.pass_cost, b.stage_cost);
            ev += (unsigned long long)c * (unsigned long long)ne;
        }
    };
    if (held) {  // unrolled, so the held values stay in registers
#pragma unroll
        for (int r = 0; r < kBucketRun; ++r)
            if (lo + r < hi) tally(r);
    } else {
        for (int r = 0; r < hi - lo; ++r) tally(r);
    }
    const long long sums[4] = {c_sum, t_sum, u_sum, k_sum};
    long long runs[4], tots[4];
    block_exclusive_scan4<kScanBlock>(sums, runs, tots);
    long long c_run = runs[0], t_run = runs[1], u_run = runs[2], k_run = runs[3];
    const long long c_tot = tots[0], t_tot = tots[1], u_tot = tots[2];
    const long long k_tot = tots[3];
    auto place = [&](int r) {
        const int k = lo + r;
        int c, e0, ne;
        get(r, &c, &e0, &ne);
        int part = 0;
        if (s_off) s_off[k] = (int)c_run;
        if (publish) {
#pragma unroll
            for (int j = 0; j < kBucketSub; ++j) {
                b.bq_off[k * kBucketSub + j] = (int)c_run + part;
                if (kBucketSub > 1) part += b.bcount[k * kBucketSub + j];
            }
        }
        if (range && c > 0) {
            Tile tl;
            tl.q0 = (int)c_run;
            tl.nq = c;
            tl.e0 = e0;
            tl.ne = ne;
            tl.nchunk = (ne + b.chunk - 1) / b.chunk;
            tl.echunk = chunk_entries(ne, tl.nchunk);
            tl.pad0 = tl.pad1 = 0;
            b.tiles[t_run] = tl;
            b.unit_off[t_run] = u_run;
            b.cost_off[t_run] = k_run;
            t_run += 1;
            u_run += (long long)tl.nchunk * c;
            k_run += tile_cost(c, tl.nchunk, b.pass_cost, b.stage_cost);
        }
        c_run += c;
    };
    if (held) {
#pragma unroll
        for (int r = 0; r < kBucketRun; ++r)
            if (lo + r < hi) place(r);
    } else {
        for (int r = 0; r < hi - lo; ++r) place(r);
    }
    if (!publish) return;
    ev = wave_sum_u64(ev);
    if (lane_id() == 0 && ev) atomicAdd(&b.ctr->n_eval, ev);
    if (threadIdx.x == 0) {
        b.ctr->n_sorted = (unsigned)c_tot;
        if (range) {
            b.ctr->n_tiles = (unsigned)t_tot;
            b.ctr->n_units = (unsigned long long)u_tot;
            b.unit_off[t_tot] = u_tot;
            b.cost_off[t_tot] = k_tot;
        }
    }
}

__global__ __launch_bounds__(kScanBlock) void k_bucket_scan(DevBatch b, DevIndex ix) {
    bucket_scan_body(b, ix, nullptr, true);
}

// Query segment i with candidates goes to its bucket's offset (from bq_off,
// or from `off` when given) plus the rank the histogram gave it (the kernels
// after this read its record and ball through perm).
__device__ __forceinline__ void scatter_one(const DevBatch &b, int i, const int *off) {
    if (i >= b.nq) return;
    int k = b.key[i];
    if (k < 0) return;
    int pos = (off ? off[k] : b.bq_off[k * kBucketSub + (i % kBucketSub)]) + b.qrank[i];
    if (b.skey) {  // sorted tilings: the order key, for the bin sort
        b.skey[pos] = start_bits(b.rec[i].t0);
        b.sidx[pos] = i;
        return;
    }
    b.perm[pos] = i;
    b.first_s[pos] = b.first[i];
    b.last_s[pos] = b.last[i];
}

__global__ void k_scatter(DevBatch b) { scatter_one(b, blockIdx.x * blockDim.x + threadIdx.x, nullptr); }

// The bucket scan and the scatter in one launch, when the bucket offsets fit
// LDS: every workgroup scans the bucket counts itself into LDS (a few
// thousand counts, read from L2), workgroup 0 also publishes the offsets,
// tiles and counters, and then each workgroup places its own kScanBlock
// query segments.
constexpr int kScanScatterBuckets = 8192;
__global__ __launch_bounds__(kScanBlock) void k_scan_scatter(DevBatch b, DevIndex ix) {
    static_assert(kBucketSub == 1, "one offset per bucket in LDS");
    extern __shared__ int s_off[];
    bucket_scan_body(b, ix, s_off, blockIdx.x == 0);
    __syncthreads();
    scatter_one(b, blockIdx.x * kScanBlock + threadIdx.x, s_off);
}

// Periodic tiles (Sec. 6): one wave per tile of s consecutive query segments
// in (t_start, caller index) order. The tile's candidate range is that of its
// temporal extent (Sec. 4): from the first member's t_start (the smallest)
// to the largest t_end of its members; it holds every member's own range and
// may hold more (a bin between two members' spans that neither overlaps).
__global__ void k_periodic_tiles(DevBatch b, DevIndex ix) {
    const int t = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (t >= b.ntiles_cap) return;
    const int q0 = t * b.s;
    // tiles past the sorted segments (those without candidates are not
    // placed) stay empty
    const int nq = max(0, min(b.s, (int)b.ctr->n_sorted - q0));
    double hi_t = -INFINITY;
    for (int k = lane; k < nq; k += 64) hi_t = dmx(hi_t, b.rec[b.perm[q0 + k]].t1);
    for (int off = 32; off > 0; off >>= 1) hi_t = dmx(hi_t, __shfl_xor(hi_t, off));
    if (lane == 0) {
        int j1 = 0, j2 = -1;
        const bool any = nq > 0 && bins_of_interval(ix.bstart, ix.bpend, ix.btree, ix.bleaf, ix.nb,
                                                    b.rec[b.perm[q0]].t0, hi_t, &j1, &j2);
        Tile tl;
        tl.q0 = q0;
        tl.nq = nq;
        tl.e0 = any ? ix.bfirst[j1] : 0;
        tl.ne = any ? ix.blast[j2] - ix.bfirst[j1] + 1 : 0;
        tl.nchunk = (tl.ne + b.chunk - 1) / b.chunk;
        tl.echunk = chunk_entries(tl.ne, tl.nchunk);
        tl.pad0 = tl.pad1 = 0;
        b.tiles[t] = tl;
        b.units[t] = (long long)tl.nchunk * nq;
    }
}

// One block: exclusive scans of the periodic tiles' work units and costs,
// and their interactions (n_eval).
__global__ __launch_bounds__(kScanBlock) void k_unit_scan(DevBatch b) {
    const int n = b.ntiles_cap;
    const int per = (n + kScanBlock - 1) / kScanBlock;
    const int lo = min(n, (int)threadIdx.x * per), hi = min(n, lo + per);
    long long s = 0, k_sum = 0;
    unsigned long long ev = 0;
    for (int k = lo; k < hi; ++k) {
        s += b.units[k];
        k_sum += tile_cost(b.tiles[k].nq, b.tiles[k].nchunk, b.pass_cost, b.stage_cost);
        ev += (unsigned long long)b.tiles[k].nq * (unsigned long long)b.tiles[k].ne;
    }
    const long long vals[4] = {s, k_sum, (long long)ev, 0};
    long long runs[4], tots[4];
    block_exclusive_scan4<kScanBlock>(vals, runs, tots);
    long long run = runs[0], k_run = runs[1];
    const long long tot = tots[0], k_tot = tots[1];
    for (int k = lo; k < hi; ++k) {
        b.unit_off[k] = run;
        b.cost_off[k] = k_run;
        run += b.units[k];
        k_run += tile_cost(b.tiles[k].nq, b.tiles[k].nchunk, b.pass_cost, b.stage_cost);
    }
    if (threadIdx.x == 0) {
        // empty tiles come last and add no units or cost
        b.ctr->n_tiles = (b.ctr->n_sorted + (unsigned)b.s - 1) / (unsigned)b.s;
        b.ctr->n_units = (unsigned long long)tot;
        b.ctr->n_eval = (unsigned long long)tots[2];
        b.unit_off[n] = tot;
        b.cost_off[n] = k_tot;
    }
}

hipError_t launch_prepare(const double *const *q, const double *d, DevBatch b, DevIndex ix,
                          hipStream_t st, hipEvent_t ev_start, bool zero) {
    const int blk = 256;
    if (zero || b.nq == 0) {
        int zgrid = (b.nbuckets + blk - 1) / blk;
        zgrid = zgrid < 1 ? 1 : (zgrid > 1024 ? 1024 : zgrid);
        TDS_LAUNCH_EV(ev_start, nullptr, k_zero_batch, dim3(zgrid), dim3(blk), 0, st, b);
        ev_start = nullptr;
    }
    if (b.nq == 0) TDS_LAUNCH_CHECK();
    const int qgrid = (b.nq + blk - 1) / blk;
    const size_t lds = ix.nb <= kQprepLdsBins ? (size_t)ix.nb * 2 * sizeof(double) : 0;
    TDS_LAUNCH_EV(ev_start, nullptr, k_qprep, dim3(qgrid), dim3(blk), lds, st, q[0], q[1], q[2], q[3],
                  q[4], q[5], q[6], q[7], d, b, ix);
    if (b.nbuckets <= kScanScatterBuckets) {
        hipLaunchKernelGGL(k_scan_scatter, dim3((b.nq + kScanBlock - 1) / kScanBlock), dim3(kScanBlock),
                           (size_t)b.nbuckets * sizeof(int), st, b, ix);
    } else {
        hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(kScanBlock), 0, st, b, ix);
        hipLaunchKernelGGL(k_scatter, dim3(qgrid), dim3(blk), 0, st, b);
    }
    TDS_LAUNCH_CHECK();
}

hipError_t launch_periodic(DevBatch b, DevIndex ix, hipStream_t st) {
    const int blk = 256;
    const int waves = b.ntiles_cap;
    hipLaunchKernelGGL(k_periodic_tiles, dim3((waves * 64 + blk - 1) / blk), dim3(blk), 0, st, b, ix);
    hipLaunchKernelGGL(k_unit_scan, dim3(1), dim3(kScanBlock), 0, st, b);
    TDS_LAUNCH_CHECK();
}

// --------------------------------------------------------------- pair test
// The binary64 decision (Sec. 5, Alg. 1: temporal intersection, then the
// degree-two polynomial of the squared distance) in the pinned order.
struct Pair64 {
    double tlo, thi, T, a, B, c;
    bool in0, inT, hit;
};

__device__ __forceinline__ Pair64 decide64(const QRec64 &q, double et0, double et1, double ex0,
                                           double ey0, double ez0, double evx, double evy,
                                           double evz) {
    Pair64 p;
    p.tlo = dmx(q.t0, et0);
    p.thi = dmn(q.t1, et1);
    p.hit = p.in0 = p.inT = false;
    if (!(p.tlo < p.thi)) return p;
    p.T = p.thi - p.tlo;
    const double tq = p.tlo - q.t0;
    const double te = p.tlo - et0;
    const double Dx = __builtin_fma(q.vx, tq, q.x0) - __builtin_fma(evx, te, ex0);
    const double Dy = __builtin_fma(q.vy, tq, q.y0) - __builtin_fma(evy, te, ey0);
    const double Dz = __builtin_fma(q.vz, tq, q.z0) - __builtin_fma(evz, te, ez0);
    const double Vx = q.vx - evx;
    const double Vy = q.vy - evy;
    const double Vz = q.vz - evz;
    p.a = __builtin_fma(Vz, Vz, __builtin_fma(Vy, Vy, Vx * Vx));
    p.B = __builtin_fma(Dz, Vz, __builtin_fma(Dy, Vy, Dx * Vx));
    p.c = __builtin_fma(Dz, Dz, __builtin_fma(Dy, Dy, __builtin_fma(Dx, Dx, -q.dd)));
    p.in0 = p.c <= 0.0;
    p.inT = __builtin_fma(__builtin_fma(p.a, p.T, p.B + p.B), p.T, p.c) <= 0.0;
    const bool vtx = (p.B < 0.0) && (__builtin_fma(p.a, p.T, p.B) > 0.0) &&
                     (__builtin_fma(p.B, p.B, -(p.a * p.c)) >= 0.0);
    p.hit = p.in0 || p.inT || vtx;
    return p;
}

__device__ __forceinline__ bool overlaps64(const QRec64 &q, double et0, double et1) {
    return dmx(q.t0, et0) < dmn(q.t1, et1);
}

// Interval of a hit: [tlo, thi] when within d at both ends (convexity),
// else the stable roots of the quadratic clamped to the common span,
// collapsed to the clamped vertex if rounding crosses them.
__device__ __forceinline__ void interval64(const Pair64 &p, double *ta, double *tb) {
    if (p.in0 && p.inT) {
        *ta = p.tlo;
        *tb = p.thi;
        return;
    }
    double h = __builtin_fma(p.B, p.B, -(p.a * p.c));
    if (h < 0.0) h = 0.0;
    const double s = sqrt(h);
    const double qq = (p.B >= 0.0) ? -(p.B + s) : (s - p.B);
    const double r1 = qq / p.a;
    const double r2 = (qq != 0.0) ? p.c / qq : r1;
    const double lo = dmn(r1, r2);
    const double hi = dmx(r1, r2);
    double xa = p.in0 ? p.tlo : p.tlo + dmx(lo, 0.0);
    double xb = p.inT ? p.thi : p.tlo + dmn(hi, p.T);
    if (xa > xb) {
        const double tv = dmn(dmx(-p.B / p.a, 0.0), p.T);
        xa = p.tlo + tv;
        xb = xa;
    }
    *ta = xa;
    *tb = xb;
}

// Tile owning work unit u: the last t in [0, n) with off[t] <= u (tiles
// without units share their successor's offset; off[0] = 0 <= u). The same
// search finds the tile owning a cost position in the cost offsets. A 64-way
// search: each round the lanes probe 64 evenly spaced offsets of [lo, hi) and
// the last probe <= u becomes lo, so n tiles take ceil(log64 n) rounds.
__device__ __forceinline__ int tile_of_unit(const long long *__restrict__ off, int n, long long u) {
    const int lane = (int)lane_id();
    int lo = 0, hi = n;  // off[lo] <= u, and u < off[hi] when hi < n
    while (hi - lo > 1) {
        const int step = (hi - lo + 63) >> 6;
        const int p = lo + lane * step;
        const unsigned long long m = __ballot(p < hi && off[p] <= u);  // bit 0 always set
        const int l = 63 - __builtin_clzll(m);
        lo += l * step;
        hi = min(hi, lo + step);
    }
    return lo;
}

// Conservative binary32 test (the ball of every point within d + band of the
// query segment against the ball that holds an entry segment): with centres
// C and c relative to the index origin, |C - c|^2 = |c|^2 - 2C.c + |C|^2, so
// per pair the test costs three multiply-adds, s = e2 + (-2C).c, compared
// with a per-query threshold T that takes the chunk's largest entry radius
// H and the rounding bound (kDotSlack). Multiply-adds issue at twice the rate
// of the minimum, maximum and compare instructions on gfx950, which a
// box test (three differences and a three-way maximum per pair) needs.
// Query balls staged in LDS per wave: 64 at a time, one per lane.
constexpr int kStage = 64;
// Staged queries tested between two branches of the binary32 walk.
#ifndef TDS_GROUP
#define TDS_GROUP 2
#endif
constexpr int kGroup = TDS_GROUP;

// Wave priority for the SIMD's instruction arbiter (0 lowest .. 3 highest).
__device__ __forceinline__ void set_prio(int p) {
    switch (p) {
    case 0: __builtin_amdgcn_s_setprio(0); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    default: __builtin_amdgcn_s_setprio(3); break;
    }
}

// Entries per lane: each wave holds 64 * EPT candidate entries of a chunk.
#ifndef TDS_EPT32
#define TDS_EPT32 5
#endif
#ifndef TDS_EPT64
#define TDS_EPT64 2
#endif
constexpr int ept_for_mode(int mode) { return mode == kModeFP64 ? TDS_EPT64 : TDS_EPT32; }
int chunk_for(int mode, int) { return 64 * ept_for_mode(mode); }

// The binary64 walk reads a chunk's 64-byte entries once per work range
// and the tile's 80-byte query records once per chunk pass: its entry loads
// are marked non-temporal, so that the L2 keeps the query records rather
// than the entry stream (binary64 traffic 1.49x -> 1.18x of the unique bytes
// on the 5M-entry workload at unchanged time). The binary32 filter keeps
// ordinary loads: its 20-byte entries are re-read by neighbouring tiles
// from L2, and marking them non-temporal made it slower.
__device__ __forceinline__ double stream_load(const double *p) {
    return __builtin_nontemporal_load(p);
}

__device__ __forceinline__ long long rfl64(long long v) {
    unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(unsigned long long)v);
    unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// Persistent pair kernel. The batch's work units (one query segment against
// one chunk of <= 64*EPT candidate entries of its tile) are numbered tile by
// tile, query-fastest, and wave w of W resident waves takes the contiguous
// range [w*U/W, (w+1)*U/W): every wave gets the same amount of work and
// consecutive units share their chunk, so a wave loads each chunk once. Lane l
// holds entries c0 + 64*j + l (slot j < EPT); the query segment is
// wave-uniform: binary64 records come through the scalar cache, binary32
// boxes are staged in LDS.
//
// The kernel only selects pairs: in binary64 mode the pairs the pinned
// decision calls hits, in binary32 mode the pairs that survive the box
// filter. Selected pairs go to a compact list that k_refine turns into hits
// with their intervals, so neither the interval arithmetic nor the refine's
// registers weigh on this loop.
template <int MODE, int BLOCK, int EPT, bool COUNT_OVL>
__global__ __launch_bounds__(BLOCK) void k_pair(const QRec64 *__restrict__ rec,
                                                const QCube32 *__restrict__ box,
                                                const int32_t *__restrict__ perm, int nq,
                                                const Tile *__restrict__ tiles,
                                                const long long *__restrict__ unit_off,
                                                const long long *__restrict__ cost_off,
                                                int pass_cost, int stage_cost, DevIndex ix,
                                                Slabs sl, Counters *__restrict__ ctr) {
    const int lane = threadIdx.x & 63;
    const long long nwaves = (long long)gridDim.x * (BLOCK / 64);
    // Workgroups are dealt to the 8 XCDs in turn (block b on XCD b % 8), each
    // XCD with its own L2. Numbering the waves XCD by XCD gives every XCD one
    // contiguous eighth of the work units, so the tiles' query records and
    // entry chunks are fetched into one L2 rather than into all eight.
    const int g_all = (int)gridDim.x, g_x = (int)blockIdx.x % 8;
    const int lblock = g_x * (g_all / 8) + min(g_x, g_all % 8) + (int)blockIdx.x / 8;
    const long long w =
        (long long)lblock * (BLOCK / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long total = rfl64((long long)ctr->n_units);
    const int ntiles = __builtin_amdgcn_readfirstlane((int)ctr->n_tiles);
    unsigned long long ovl_acc = 0;
    // Selections go to the wave's current slab (its own one first); when a
    // ballot does not fit, the wave closes that slab with its count and takes
    // a fresh spill slab with one atomic. A slab number past nslabs is
    // counted but not stored, so the host can size the re-run exactly: the
    // number of slabs a wave takes depends only on its own selections.
    long long cs = w < sl.nwaves ? w : -1;  // waves beyond the slabs (not launched so) spill
    int cn = w < sl.nwaves ? 0 : kSlab;
    auto select = [&](bool flag, const Cand &rec) {
        const unsigned long long m = __ballot(flag);
        if (m == 0ull) return;
        const int cnt = __popcll(m);
        const unsigned rank = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (cn + cnt > kSlab) {
            const int leader = __ffsll((long long)m) - 1;
            unsigned long long k = 0;
            if (lane == leader) {
                if (cs >= 0 && cs < sl.nslabs) sl.slab_n[cs] = cn;
                k = atomicAdd(&ctr->spill, 1ull);
            }
            cs = (long long)sl.nwaves + (long long)__shfl(k, leader);
            cn = 0;
        }
        if (flag && cs < sl.nslabs) sl.cand[cs * kSlab + cn + rank] = rec;
        cn += cnt;
    };
    // progress-based wave priority (see below): one step down per pr_step units
    int prio = 3, pr_step = 1, pr_next = 1;
    auto progress = [&](int units) {
        pr_next -= units;
        if (pr_next <= 0) {
            pr_next += pr_step;
            if (prio > 0) set_prio(--prio);
        }
    };
    // Units [u, uend) of consecutive tiles.
    auto run_range = [&](long long u, const long long uend) {
    int t = tile_of_unit(unit_off, ntiles, u);
    while (u < uend) {
        const Tile tl = tiles[t];
        const long long base = unit_off[t];
        const long long tend = min(uend, base + (long long)tl.nchunk * tl.nq);
        while (u < tend) {
            const long long local = u - base;
            const int ch = (int)(local / tl.nq);
            const int qf = (int)(local - (long long)ch * tl.nq);
            const int ql = (int)min((long long)tl.nq, qf + (tend - u));
            const int qb = tl.q0 + qf, qe = tl.q0 + ql;
            const int wb = tl.e0 + ch * tl.echunk;
            const int we = min(tl.e0 + tl.ne, wb + tl.echunk);
            const int nv = min(EPT, (we - wb + 63) >> 6);  // slots holding entries (>= 1)
            u += ql - qf;

            if constexpr (MODE == kModeFP64) {
                double et0[EPT], et1[EPT], ex0[EPT], ey0[EPT], ez0[EPT], evx[EPT], evy[EPT],
                    evz[EPT];
#pragma unroll
                for (int j = 0; j < EPT; ++j) {
                    const int e = wb + j * 64 + lane;
                    if (e < we) {  // streamed: read once per tile (see stream_load)
                        et0[j] = stream_load(&ix.t0[e]);
                        et1[j] = stream_load(&ix.t1[e]);
                        ex0[j] = stream_load(&ix.x0[e]);
                        ey0[j] = stream_load(&ix.y0[e]);
                        ez0[j] = stream_load(&ix.z0[e]);
                        evx[j] = stream_load(&ix.vx[e]);
                        evy[j] = stream_load(&ix.vy[e]);
                        evz[j] = stream_load(&ix.vz[e]);
                    } else {  // an empty span never overlaps
                        et0[j] = INFINITY;
                        et1[j] = -INFINITY;
                        ex0[j] = ey0[j] = ez0[j] = evx[j] = evy[j] = evz[j] = 0.0;
                    }
                }
                auto walk = [&](auto full) {
                    constexpr bool FULL = decltype(full)::value;  // all EPT slots hold entries
                    // Records in caller order through perm, read one query
                    // ahead (and perm two ahead). perm carries two spare slots;
                    // positions past the placed segments hold no index, so
                    // the read-ahead clamps it.
                    auto clampq = [&](int i) { return min(max(i, 0), nq - 1); };
                    int pcur = perm[qb];  // caller index of query qs
                    QRec64 qn = rec[clampq(pcur)];
                    int pnext = perm[qb + 1];
                    for (int qs = qb; qs < qe; ++qs) {
                        const QRec64 q = qn;
                        const int pq = pcur;
                        const int pn = pnext;
                        pnext = perm[qs + 2];
                        qn = rec[clampq(pn)];
                        pcur = pn;
                        progress(1);
#pragma unroll
                        for (int j = 0; j < EPT; ++j) {
                            if (!FULL && j >= nv) break;  // wave-uniform
                            const Pair64 p = decide64(q, et0[j], et1[j], ex0[j], ey0[j], ez0[j],
                                                      evx[j], evy[j], evz[j]);
                            if (COUNT_OVL) ovl_acc += __popcll(__ballot(p.tlo < p.thi));
                            select(p.hit, Cand{(uint32_t)pq, (uint32_t)(wb + j * 64 + lane)});
                        }
                    }
                };
                if (nv == EPT)
                    walk(std::true_type{});
                else
                    walk(std::false_type{});
            } else {
                // Conservative binary32 filter: the entry's ball against the
                // query's ball; time is left to the refine. Each slot holds
                // (c, e2) of an entry, or NaN for no entry (NaN never passes).
                float4 ec[EPT];
                float hmax = 0.0f, e2max = 0.0f;
#pragma unroll
                for (int j = 0; j < EPT; ++j) {
                    const int e = wb + j * 64 + lane;
                    if (e < we) {
                        ec[j] = ix.ecen[e];
                        e2max = fmaxf(e2max, ec[j].w);
                        hmax = fmaxf(hmax, ix.erad[e]);
                    } else {
                        ec[j] = make_float4(0.0f, 0.0f, 0.0f, NAN);
                    }
                }
                // H: the largest entry radius of the chunk, E2: its largest
                // |c|^2 (wave-uniform)
                for (int off = 32; off > 0; off >>= 1) {
                    hmax = fmaxf(hmax, __shfl_xor(hmax, off));
                    e2max = fmaxf(e2max, __shfl_xor(e2max, off));
                }
                const float H = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(hmax)));
                const float E2 = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(e2max)));
                // s = e2 + (-2C).c with one multiply-add per axis; a staged
                // query is (T, -2C): component k of the query then sits one
                // register after component k of the entry, in another
                // register bank of the four (a multiply-add whose sources
                // share a bank issues slower)
                auto dot_of = [&](const float4 &c, const float4 &q) {
                    return __builtin_fmaf(c.z, q.w, __builtin_fmaf(c.y, q.z, __builtin_fmaf(c.x, q.y, c.w)));
                };
                // Smallest s of a staged query over the lane's slots.
                auto gmin_of = [&](const float4 &qv, auto full) {
                    constexpr bool FULL = decltype(full)::value;
                    float g = dot_of(ec[0], qv);  // slot 0 always holds entries
#pragma unroll
                    for (int j = 1; j < EPT; ++j)
                        if (FULL || j < nv) g = fminf(g, dot_of(ec[j], qv));
                    return g;
                };
                // The selections of one query: its s are computed again
                // (this path is rare, and keeping every s of the common path
                // in registers would cost occupancy).
                auto emit = [&](const float4 &qv, const int qs, auto full) {
                    constexpr bool FULL = decltype(full)::value;
                    const uint32_t qc = (uint32_t)perm[qs];  // caller index
#pragma unroll
                    for (int j = 0; j < EPT; ++j) {
                        const bool has = FULL || j < nv;  // wave-uniform
                        const float g = has ? dot_of(ec[j], qv) : NAN;
                        select(g <= qv.x, Cand{qc, (uint32_t)(wb + j * 64 + lane)});
                    }
                };
                auto count_ovl = [&](const int qs) {
                    if (COUNT_OVL) {
                        const QRec64 q = rec[perm[qs]];
#pragma unroll
                        for (int j = 0; j < EPT; ++j) {
                            const int e = wb + j * 64 + lane;
                            const bool ov = e < we && overlaps64(q, ix.t0[e], ix.t1[e]);
                            ovl_acc += __popcll(__ballot(ov));
                        }
                    }
                };
                // The wave stages up to 64 query balls in its LDS slice (one
                // coalesced load, lane i takes ball s0 + i) as (T, -2C), T the
                // ball's threshold against this chunk, evaluated in binary64
                // with margins for its own rounding and rounded up:
                //   T = (r + H)^2 - |C|^2 + kDotSlack (E2 + |C|^2);
                // then it walks them kGroup at a time with broadcast LDS
                // reads at fixed offsets: the kGroup smallest s (each the
                // minimum over the lane's EPT entries) are computed before the
                // one (rarely taken) branch, which gives the scheduler
                // kGroup x EPT independent chains. LDS requests of one wave
                // complete in order, so the slice is rewritten only after the
                // previous walk has read it.
                __shared__ float4 s_q[BLOCK / 64][kStage];
                const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
                auto walk = [&](auto full) {
                    for (int s0 = qb; s0 < qe; s0 += kStage) {
                        const int ns = __builtin_amdgcn_readfirstlane(min(kStage, qe - s0));
                        if (lane < ns) {
                            const QCube32 c = box[perm[s0 + lane]];
                            float4 v = make_float4(INFINITY, 0.0f, 0.0f, 0.0f);  // passes all
                            if (c.r != INFINITY) {
                                const double C2 = (double)c.cx * c.cx + (double)c.cy * c.cy +
                                                  (double)c.cz * c.cz;
                                const double R = (double)c.r + (double)H;
                                const double T = R * R * (1.0 + 0x1p-40) - C2 * (1.0 - 0x1p-40) +
                                                 kDotSlack * ((double)E2 + C2);
                                v = make_float4(f32_up(T), -2.0f * c.cx, -2.0f * c.cy, -2.0f * c.cz);
                            }
                            s_q[wv][lane] = v;
                        }
                        const float4 *sq = s_q[wv];
                        // kGroup queries per branch (compile-time)
                        auto group = [&](const int j) {
                            bool p = false;
#pragma unroll
                            for (int k = 0; k < kGroup; ++k) {
                                const float4 qk = sq[j + k];
                                p |= gmin_of(qk, full) <= qk.x;
                            }
                            if (__builtin_expect(__ballot(p) != 0ull, 0)) {
                                for (int k = 0; k < kGroup; ++k) emit(sq[j + k], s0 + j + k, full);
                            }
                        };
                        int j = 0;
                        for (; j + kGroup <= ns; j += kGroup) group(j);
                        for (; j < ns; ++j) {
                            const float4 qa = sq[j];
                            if (__builtin_expect(__ballot(gmin_of(qa, full) <= qa.x) != 0ull, 0))
                                emit(qa, s0 + j, full);
                        }
                        if (COUNT_OVL)
                            for (int k = 0; k < ns; ++k) count_ovl(s0 + k);
                        progress(ns);
                    }
                };
                if (nv == EPT)
                    walk(std::true_type{});
                else
                    walk(std::false_type{});
            }
        }
        ++t;
    }
    };
    // Even static split of the batch's cost over the launched waves (every
    // wave is resident from the start, see resident_blocks). A cost position
    // maps to the first work unit at or after it; the overhead of a chunk
    // pass counts before its first segment. The SIMD issues the oldest ready
    // wave first, so without correction the first waves finish early and the
    // last ones run nearly alone; each wave therefore lowers its priority by
    // one step per quarter of its share done, keeping the waves of a SIMD at
    // similar progress so they finish together.
    const long long ctot = rfl64(cost_off[ntiles]);
    auto unit_at = [&](const long long c) -> long long {
        if (c >= ctot) return total;
        const int t = tile_of_unit(cost_off, ntiles, c);
        const Tile tl = tiles[t];
        const long long ov = pass_overhead(tl.nq, pass_cost, stage_cost);
        const long long lc = c - cost_off[t];
        const long long ch = lc / (tl.nq + ov);
        const long long r = lc - ch * (tl.nq + ov) - ov;
        return unit_off[t] + ch * tl.nq + (r > 0 ? r : 0);
    };
    const long long u0 = unit_at((w * ctot) / nwaves), u1 = unit_at(((w + 1) * ctot) / nwaves);
    pr_step = (int)max(1LL, min((u1 - u0) / 4, (long long)INT_MAX));
    pr_next = pr_step;
    set_prio(3);
    if (u0 < u1) run_range(u0, u1);
    if (lane == 0 && cs >= 0 && cs < sl.nslabs) sl.slab_n[cs] = cn;
    if (COUNT_OVL && lane == 0 && w < sl.nwaves) sl.wave_ovl[w] = ovl_acc;
}

// Selected pairs -> hits: the pinned binary64 decision again (a selected
// pair of the binary32 filter may be a miss) and, for hits, the interval.
// One wave per slab (grid-stride); the hits of slab s are compacted to the
// front of hit slab s with a ballot, so no atomics are needed.
__global__ __launch_bounds__(256) void k_refine(const QRec64 *__restrict__ rec, Slabs sl,
                                                DevIndex ix, const Counters *__restrict__ ctr) {
    const int lane = threadIdx.x & 63;
    const long long nsl = sl.nwaves + min((long long)ctr->spill, sl.nslabs - sl.nwaves);
    const long long nw = (long long)gridDim.x * 4;
    for (long long s = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); s < nsl; s += nw) {
        // the count and the records are read together (a slab's memory
        // exists whatever its count; records past it are not used)
        const int cnt = sl.slab_n[s];
        const Cand c = sl.cand[s * kSlab + lane];
        bool hit = false;
        Hit24 h;
        if (lane < cnt) {
            const QRec64 q = rec[c.q];
            const int e = (int)c.e;
            const Pair64 p = decide64(q, ix.t0[e], ix.t1[e], ix.x0[e], ix.y0[e], ix.z0[e], ix.vx[e],
                                      ix.vy[e], ix.vz[e]);
            hit = p.hit;
            h.q = c.q;
            h.e = c.e;
            h.ta = h.tb = 0.0;
            if (hit) interval64(p, &h.ta, &h.tb);
        }
        const unsigned long long m = __ballot(hit);
        if (hit) {
            const unsigned rank = __builtin_amdgcn_mbcnt_hi(
                (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            sl.hits[s * kSlab + rank] = h;
        }
        if (lane == 0) sl.slab_h[s] = __popcll(m);
    }
}

// Grid of a persistent launch: the blocks that are resident at once. On
// MI355X a launch sized by the occupancy query leaves one wave per SIMD (per
// CU: 4 waves) without a slot, measured with per-wave start stamps: that many
// blocks start only when others end and then run their share alone. So one
// wave per SIMD less is launched than the query reports.
template <class K>
static int resident_blocks(K kernel, int block) {
    int dev = 0, cus = 256, per_cu = 0;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int wpb = block / 64;                 // waves per block
    const int per_simd = per_cu * wpb / 4;      // waves per SIMD the query allows
    const int fit = ((per_simd - 1) * 4) / wpb;  // blocks per CU with one wave per SIMD less
    return cus * (fit < 1 ? 1 : fit);
}

template <int MODE, int BLOCK>
static int pair_grid_b(int grid, int kernel_overlap) {
    constexpr int EPT = ept_for_mode(MODE);
    if (grid > 0) return grid;
    if (kernel_overlap) {
        static const int resident = resident_blocks(k_pair<MODE, BLOCK, EPT, true>, BLOCK);
        return resident;
    }
    static const int resident = resident_blocks(k_pair<MODE, BLOCK, EPT, false>, BLOCK);
    return resident;
}

int pair_grid(int mode, int block, int grid, int kernel_overlap) {
#define TDS_GRID_CASE(M, BS) \
    case BS: return pair_grid_b<M, BS>(grid, kernel_overlap);
    if (mode == kModeFP64) {
        switch (block) {
            TDS_GRID_CASE(kModeFP64, 64)
            TDS_GRID_CASE(kModeFP64, 128)
            TDS_GRID_CASE(kModeFP64, 256)
            TDS_GRID_CASE(kModeFP64, 512)
            TDS_GRID_CASE(kModeFP64, 1024)
        }
    } else {
        switch (block) {
            TDS_GRID_CASE(kModeFP32Refine, 64)
            TDS_GRID_CASE(kModeFP32Refine, 128)
            TDS_GRID_CASE(kModeFP32Refine, 256)
            TDS_GRID_CASE(kModeFP32Refine, 512)
            TDS_GRID_CASE(kModeFP32Refine, 1024)
        }
    }
#undef TDS_GRID_CASE
    return 0;
}

template <int MODE, int BLOCK>
static hipError_t launch_pair_b(DevBatch b, DevIndex ix, int grid, int kernel_overlap, Slabs sl,
                                hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    constexpr int EPT = ept_for_mode(MODE);
    const int g = pair_grid_b<MODE, BLOCK>(grid, kernel_overlap);
    if ((long long)g * (BLOCK / 64) != sl.nwaves || sl.nslabs <= sl.nwaves)
        return hipErrorInvalidValue;  // slabs sized for another launch
    if (kernel_overlap)
        TDS_LAUNCH_EV(ev0, ev1, (k_pair<MODE, BLOCK, EPT, true>), dim3(g), dim3(BLOCK), 0, st,
                      b.rec, b.box, b.perm, b.nq, b.tiles, b.unit_off, b.cost_off,
                      b.pass_cost, b.stage_cost, ix, sl, b.ctr);
    else
        TDS_LAUNCH_EV(ev0, ev1, (k_pair<MODE, BLOCK, EPT, false>), dim3(g), dim3(BLOCK), 0, st,
                      b.rec, b.box, b.perm, b.nq, b.tiles, b.unit_off, b.cost_off,
                      b.pass_cost, b.stage_cost, ix, sl, b.ctr);
    TDS_LAUNCH_CHECK();
}

hipError_t launch_pair(DevBatch b, DevIndex ix, int mode, int block, int grid, int kernel_overlap,
                       Slabs sl, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    if (b.nq == 0) {  // nothing to launch: the events still mark the point
        if (ev0) (void)hipEventRecord(ev0, st);
        if (ev1) (void)hipEventRecord(ev1, st);
        return hipGetLastError();
    }
#define TDS_PAIR_CASE(M, BS) \
    case BS: return launch_pair_b<M, BS>(b, ix, grid, kernel_overlap, sl, st, ev0, ev1);
    if (mode == kModeFP64) {
        switch (block) {
            TDS_PAIR_CASE(kModeFP64, 64)
            TDS_PAIR_CASE(kModeFP64, 128)
            TDS_PAIR_CASE(kModeFP64, 256)
            TDS_PAIR_CASE(kModeFP64, 512)
            TDS_PAIR_CASE(kModeFP64, 1024)
        }
    } else {
        switch (block) {
            TDS_PAIR_CASE(kModeFP32Refine, 64)
            TDS_PAIR_CASE(kModeFP32Refine, 128)
            TDS_PAIR_CASE(kModeFP32Refine, 256)
            TDS_PAIR_CASE(kModeFP32Refine, 512)
            TDS_PAIR_CASE(kModeFP32Refine, 1024)
        }
    }
#undef TDS_PAIR_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_refine(DevBatch b, DevIndex ix, Slabs sl, hipStream_t st, hipEvent_t ev_stop) {
    if (b.nq == 0) {
        if (ev_stop) (void)hipEventRecord(ev_stop, st);
        return hipGetLastError();
    }
    static const int grid = resident_blocks(k_refine, 256);
    TDS_LAUNCH_EV(nullptr, ev_stop, k_refine, dim3(grid), dim3(256), 0, st, b.rec, sl, ix, b.ctr);
    TDS_LAUNCH_CHECK();
}

// Clears the counters that the pair kernel (all = 1) or only the refine
// kernel (all = 0) accumulates, so they can run again (overflow retry).
__global__ void k_reset_counters(Counters *c, int all) {
    c->hits = 0;
    if (all) {
        c->cand = 0;
        c->overlap = 0;
        c->spill = 0;
        c->n_slabs = 0;
    }
}

hipError_t launch_reset_counters(Counters *c, int all, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(1), 0, st, c, all);
    TDS_LAUNCH_CHECK();
}

// The batch's last kernel, enqueued when the caller fetches: the position of
// each hit slab's hits in the dense output (hit_off), the records of the
// first n hits in caller indices, and the final counters. Workgroup g takes
// a contiguous run of slabs; its hits follow those of every earlier slab,
// which it sums itself (each workgroup reads the hit counts before its run,
// a few thousand counts from L2 with independent loads), so no second pass
// or inter-workgroup wait is needed. The run goes in rounds
// of kEmitBlock slabs: a workgroup scan gives the slabs' offsets, then each
// thread takes hits of the round (a search over the round's offsets in LDS
// finds a hit's slab), so the loads of all hits are in flight together.
// Workgroup 0 also sums hits, selections and (when the pair kernel counted
// them) overlapping pairs over the whole batch, publishes the counters (also
// to `host_out`, pinned host memory that the host reads after the stream is
// synchronized, which saves a copy on the stream) and clears the counters of
// the handle's next batch (its own Counters slot, and bucket counters no
// kernel of this batch reads). Running it again (another output buffer)
// gives the same offsets and counters.
constexpr int kEmitBlock = 256;
constexpr int kEmitMinGroups = 64;
constexpr int kEmitSpillPerGroup = 8;
constexpr int kEmitIlp = 4;  // independent loads per thread in the sums

// Sum of v[k] over k in [lo, hi) by the workgroup (every thread gets it).
template <class T>
__device__ __forceinline__ long long emit_sum(const T *__restrict__ v, long long lo, long long hi,
                                              long long *s_red) {
    long long acc[kEmitIlp] = {};
    long long k = lo + threadIdx.x;
    for (; k + (kEmitIlp - 1) * kEmitBlock < hi; k += kEmitIlp * kEmitBlock) {
#pragma unroll
        for (int j = 0; j < kEmitIlp; ++j) acc[j] += (long long)v[k + j * kEmitBlock];
    }
    for (; k < hi; k += kEmitBlock) acc[0] += (long long)v[k];
    long long t = 0;
#pragma unroll
    for (int j = 0; j < kEmitIlp; ++j) t += acc[j];
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
    __syncthreads();  // s_red is free again
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = t;
    __syncthreads();
    long long r = 0;
#pragma unroll
    for (int w = 0; w < kEmitBlock / 64; ++w) r += s_red[w];
    return r;
}

__global__ __launch_bounds__(kEmitBlock) void k_emit(Slabs sl, Counters *__restrict__ ctr, int64_t n,
                                                     DevIndex ix, int64_t *out, int count_ovl,
                                                     Counters *host_out, NextClear next) {
    __shared__ long long s_red[kEmitBlock / 64];
    __shared__ int s_loc[kEmitBlock + 1];  // round-local exclusive offsets, then the total
    const int tid = threadIdx.x;
    const long long spill = min((long long)ctr->spill, sl.nslabs - sl.nwaves);
    const long long nsl = sl.nwaves + spill;
    // workgroups in use: kEmitMinGroups, and more as the selections spill
    // beyond the wave slabs (batches with many hits); the rest return
    const long long groups = min((long long)gridDim.x, kEmitMinGroups + spill / kEmitSpillPerGroup);
    if ((long long)blockIdx.x >= groups) return;
    const long long per = (nsl + groups - 1) / groups;
    const long long lo = min(nsl, (long long)blockIdx.x * per), hi = min(nsl, lo + per);
    long long pre = emit_sum(sl.slab_h, 0, lo, s_red);
    for (long long base = lo; base < hi; base += kEmitBlock) {
        const long long k = base + tid;
        const int h = k < hi ? sl.slab_h[k] : 0;
        const long long vals[4] = {h, 0, 0, 0};
        long long runs[4], tots[4];
        block_exclusive_scan4<kEmitBlock>(vals, runs, tots);
        s_loc[tid] = (int)runs[0];
        if (tid == 0) s_loc[kEmitBlock] = (int)tots[0];
        if (k < hi) sl.hit_off[k] = pre + runs[0];
        __syncthreads();
        const int cnt = (int)min((long long)kEmitBlock, hi - base);
        const int rh = s_loc[kEmitBlock];
        // hits of the round in output order; hit r lies in the last slab j
        // of the round with s_loc[j] <= r
        for (int r = tid; r < rh && pre + r < n; r += kEmitBlock) {
            int a = 0, z = cnt - 1;
            while (a < z) {
                const int m = (a + z + 1) >> 1;
                if (s_loc[m] <= r) a = m; else z = m - 1;
            }
            const Hit24 hh = sl.hits[(base + a) * kSlab + (r - s_loc[a])];
            int64_t *o = out + 5 * (pre + r);
            o[0] = hh.q;
            o[1] = ix.orig[hh.e];
            o[2] = ix.traj[hh.e];
            o[3] = __double_as_longlong(hh.ta);
            o[4] = __double_as_longlong(hh.tb);
        }
        pre += tots[0];
        __syncthreads();  // s_loc is rewritten by the next round
    }
    if (blockIdx.x != 0) return;
    if (next.ctr) {
        for (int k = tid; k < next.nbuckets; k += kEmitBlock) {
            next.bcount[k] = 0;
            next.bj2[k] = -1;
        }
        if (tid == 0) *next.ctr = Counters{};
    }
    const long long sh = emit_sum(sl.slab_h, 0, nsl, s_red);
    const long long sn = emit_sum(sl.slab_n, 0, nsl, s_red);
    const long long so = count_ovl ? emit_sum(sl.wave_ovl, 0, sl.nwaves, s_red) : 0;
    if (tid == 0) {
        ctr->hits = (unsigned long long)sh;
        ctr->cand = (unsigned long long)sn;
        ctr->n_slabs = (unsigned long long)nsl;
        if (count_ovl) ctr->overlap = (unsigned long long)so;
        if (host_out) *host_out = *ctr;
    }
}

hipError_t launch_emit(Slabs sl, Counters *ctr, int64_t n, DevIndex ix, void *out_hits,
                       int count_ovl, Counters *host_out, NextClear next, hipStream_t st,
                       hipEvent_t ev_start, hipEvent_t ev_stop) {
    // up to as many workgroups as are resident at once: batches with many
    // hits write them in parallel (the kernel uses 64 of them, plus one per
    // 8 spill slabs)
    static const int grid = resident_blocks(k_emit, kEmitBlock);
    TDS_LAUNCH_EV(ev_start, ev_stop, k_emit, dim3(grid), dim3(kEmitBlock), 0, st, sl, ctr,
                  out_hits ? n : (int64_t)0, ix, (int64_t *)out_hits, count_ovl, host_out, next);
    TDS_LAUNCH_CHECK();
}

}  // namespace tds
