// HIP kernels of the distance-threshold search for CDNA4 (gfx950).
//
// Data layout: entries are sorted by t_start and stored as a structure of
// arrays (coalesced 64-lane loads); query segments of a batch are sorted,
// grouped into tiles and read wave-uniformly (scalar loads); one lane holds
// EPT entries of a work item and walks the tile's query segments.
//
// The binary64 decision below follows the paper's Alg. 1 (temporal
// intersection, then the time interval within d from the degree-two
// polynomial of the squared distance) in one fixed evaluation order:
//   tlo = max(q.t0, e.t0), thi = min(q.t1, e.t1), compared only if tlo < thi
//   T = thi - tlo, tq = tlo - q.t0, te = tlo - e.t0
//   D_k = fma(q.v_k, tq, q.p0_k) - fma(e.v_k, te, e.p0_k), V_k = q.v_k - e.v_k
//   a = fma(Vz,Vz, fma(Vy,Vy, Vx*Vx)), B = fma(Dz,Vz, fma(Dy,Vy, Dx*Vx)),
//   c = fma(Dz,Dz, fma(Dy,Dy, fma(Dx,Dx, -dd)))
//   hit = c <= 0 || fma(fma(a,T,B+B),T,c) <= 0
//         || (B < 0 && fma(a,T,B) > 0 && fma(B,B,-(a*c)) >= 0)
// Built with -ffp-contract=off: every fma is explicit, nothing is fused or
// reassociated behind the source's back.
#include <hipcub/hipcub.hpp>

#include "tds_internal.h"

namespace tds {

#define TDS_LAUNCH_CHECK() return hipGetLastError()

__device__ __forceinline__ double dmx(double a, double b) { return a > b ? a : b; }
__device__ __forceinline__ double dmn(double a, double b) { return a < b ? a : b; }

// binary32 neighbours of a binary64 value: largest float <= x, smallest >= x.
__device__ __forceinline__ float f32_down(double x) {
    float f = (float)x;
    return ((double)f > x) ? nextafterf(f, -INFINITY) : f;
}
__device__ __forceinline__ float f32_up(double x) {
    float f = (float)x;
    return ((double)f < x) ? nextafterf(f, INFINITY) : f;
}

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// --------------------------------------------------------------- ingest
// One thread per sorted position p: gather the caller's segment perm[p],
// compute its velocity and its conservative binary32 box.
__global__ void k_ingest(const double *__restrict__ rx0, const double *__restrict__ ry0,
                         const double *__restrict__ rz0, const double *__restrict__ rt0,
                         const double *__restrict__ rx1, const double *__restrict__ ry1,
                         const double *__restrict__ rz1, const double *__restrict__ rt1,
                         int64_t n, const int32_t *__restrict__ perm,
                         const int64_t *__restrict__ traj_raw, double *t0, double *t1, double *x0,
                         double *y0, double *z0, double *vx, double *vy, double *vz, float4 *boxa,
                         float4 *boxb, int32_t *orig, int64_t *traj) {
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
    boxa[p] = make_float4(f32_down(s0), f32_up(s1), f32_down(dmn(a0, a1)), f32_up(dmx(a0, a1)));
    boxb[p] = make_float4(f32_down(dmn(b0, b1)), f32_up(dmx(b0, b1)), f32_down(dmn(c0, c1)),
                          f32_up(dmx(c0, c1)));
    orig[p] = i;
    traj[p] = traj_raw ? traj_raw[i] : (int64_t)i;
}

hipError_t launch_ingest(const double *const *raw, int64_t n, const int32_t *perm_sorted,
                         const int64_t *traj_raw, DevIndex, double *t0, double *t1, double *x0,
                         double *y0, double *z0, double *vx, double *vy, double *vz, float4 *boxa,
                         float4 *boxb, int32_t *orig, int64_t *traj, hipStream_t st) {
    if (n == 0) return hipSuccess;
    int blk = 256;
    int64_t grid = (n + blk - 1) / blk;
    hipLaunchKernelGGL(k_ingest, dim3((unsigned)grid), dim3(blk), 0, st, raw[0], raw[1], raw[2],
                       raw[3], raw[4], raw[5], raw[6], raw[7], n, perm_sorted, traj_raw, t0, t1, x0,
                       y0, z0, vx, vy, vz, boxa, boxb, orig, traj);
    TDS_LAUNCH_CHECK();
}

// --------------------------------------------------------------- query prep
// First index k in [0, nb) with a[k] > x (a non-decreasing), nb if none.
__device__ __forceinline__ int first_greater(const double *a, int nb, double x) {
    int lo = 0, hi = nb;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] > x) hi = mid; else lo = mid + 1;
    }
    return lo;
}
// Number of elements < x in a sorted array.
__device__ __forceinline__ int64_t count_less(const double *a, int64_t n, double x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}
// Number of elements <= x in a sorted array.
__device__ __forceinline__ int64_t count_leq(const double *a, int64_t n, double x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// One thread per query segment (caller order): validate, build its binary64
// record and binary32 box, find its candidate range with two binary
// searches over the non-empty bins (Sec. 4: bins whose temporal extent
// overlaps the segment's), count its overlapping entries, and make its
// sort key.
__global__ void k_qprep(const double *__restrict__ qx0, const double *__restrict__ qy0,
                        const double *__restrict__ qz0, const double *__restrict__ qt0,
                        const double *__restrict__ qx1, const double *__restrict__ qy1,
                        const double *__restrict__ qz1, const double *__restrict__ qt1,
                        const double *__restrict__ qd, DevBatch b, DevIndex ix, double t_first,
                        double t_span) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long novl = 0;
    if (i < b.nq) {
        double a0 = qx0[i], b0 = qy0[i], c0 = qz0[i], s0 = qt0[i];
        double a1 = qx1[i], b1 = qy1[i], c1 = qz1[i], s1 = qt1[i];
        double d = qd[i];
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

        // Box widened by d plus a band that covers the binary64 decision's
        // own rounding (a hit in binary64 implies the exact distance is
        // below d + band at some common time) and the rounding of positions.
        double ext = fabs(a1 - a0) + fabs(b1 - b0) + fabs(c1 - c0);
        double mag = dmx(dmx(fabs(a0), fabs(a1)), dmx(dmx(fabs(b0), fabs(b1)), dmx(fabs(c0), fabs(c1))));
        double w = d + ix.band_rel * (d + ext + ix.ext_max) +
                   ix.band_abs * (1.0 + d + mag + ext + ix.mag_max + ix.ext_max);
        QBox32 bx;
        bx.t0 = f32_down(s0);
        bx.t1 = f32_up(s1);
        bx.xlo = f32_down(dmn(a0, a1) - w);
        bx.xhi = f32_up(dmx(a0, a1) + w);
        bx.ylo = f32_down(dmn(b0, b1) - w);
        bx.yhi = f32_up(dmx(b0, b1) + w);
        bx.zlo = f32_down(dmn(c0, c1) - w);
        bx.zhi = f32_up(dmx(c0, c1) + w);
        b.box[i] = bx;

        // Candidate bins: j1 = first bin whose prefix-max end exceeds t0,
        // j2 = last bin whose start is below t1 (strict: spans must overlap
        // with positive length).
        int j1 = first_greater(ix.bpend, ix.nb, s0);
        int j2;
        {
            int lo = 0, hi = ix.nb;  // number of bins with start < t1
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (ix.bstart[mid] < s1) lo = mid + 1; else hi = mid;
            }
            j2 = lo - 1;
        }
        int first = 0, last = -1;
        if (ok && j1 <= j2) {
            first = ix.bfirst[j1];
            last = ix.blast[j2];
        }
        b.first[i] = first;
        b.last[i] = last;

        if (ok) novl = (unsigned long long)(count_less(ix.t0s, ix.n, s1) - count_leq(ix.t1s, ix.n, s0));

        unsigned long long key;
        if (b.tiling == kTilePeriodic) {
            double u = (s0 - t_first) / t_span;
            u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
            double k = u * 4294967295.0;
            key = (unsigned long long)k;
        } else {
            unsigned long long K = (unsigned long long)ix.nb + 1ull;
            if (j1 <= j2 && ok)
                key = (unsigned long long)j1 * K + (unsigned long long)(j2 - j1);
            else
                key = (unsigned long long)ix.nb * K;
        }
        b.key_in[i] = key;
        b.val_in[i] = i;
    }
    novl = wave_sum_u64(novl);
    if (lane_id() == 0 && novl) atomicAdd(&b.ctr->n_overlap_exact, novl);
}

hipError_t launch_qprep(const double *const *q, const double *d, DevBatch b, DevIndex ix,
                        double t_first, double t_span, hipStream_t st) {
    if (b.nq == 0) return hipSuccess;
    int blk = 256;
    int grid = (b.nq + blk - 1) / blk;
    hipLaunchKernelGGL(k_qprep, dim3(grid), dim3(blk), 0, st, q[0], q[1], q[2], q[3], q[4], q[5],
                       q[6], q[7], d, b, ix, t_first, t_span);
    TDS_LAUNCH_CHECK();
}

// --------------------------------------------------------------- sort
hipError_t sort_temp_bytes(int n, size_t *bytes) {
    *bytes = 0;
    return hipcub::DeviceRadixSort::SortPairs(nullptr, *bytes, (const unsigned long long *)nullptr,
                                              (unsigned long long *)nullptr,
                                              (const int32_t *)nullptr, (int32_t *)nullptr, n, 0,
                                              64, (hipStream_t)0);
}

hipError_t launch_sort(void *temp, size_t temp_bytes, DevBatch b, int end_bit, hipStream_t st) {
    if (b.nq == 0) return hipSuccess;
    size_t tb = temp_bytes;
    return hipcub::DeviceRadixSort::SortPairs(temp, tb, b.key_in, b.key_out, b.val_in, b.perm, b.nq,
                                              0, end_bit, st);
}

hipError_t scan_temp_bytes(int n, size_t *bytes) {
    *bytes = 0;
    return hipcub::DeviceScan::ExclusiveSum(nullptr, *bytes, (const int32_t *)nullptr,
                                            (int32_t *)nullptr, n, (hipStream_t)0);
}

hipError_t launch_scan(void *temp, size_t temp_bytes, const int32_t *in, int32_t *out, int n,
                       hipStream_t st) {
    if (n == 0) return hipSuccess;
    size_t tb = temp_bytes;
    return hipcub::DeviceScan::ExclusiveSum(temp, tb, in, out, n, st);
}

// --------------------------------------------------------------- gather
// One thread per sorted position: move the query's record, box and range
// into sorted order and flag tile heads (every s-th position, and for range
// tiling also wherever the candidate bin range changes).
__global__ void k_gather(DevBatch b) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= b.nq) return;
    int i = b.perm[p];
    b.rec_s[p] = b.rec[i];
    b.box_s[p] = b.box[i];
    b.first_s[p] = b.first[i];
    b.last_s[p] = b.last[i];
    int h = (p % b.s) == 0;
    if (b.tiling == kTileRange && p > 0 && b.key_out[p] != b.key_out[p - 1]) h = 1;
    b.head[p] = h;
}

hipError_t launch_gather(DevBatch b, DevIndex, hipStream_t st) {
    if (b.nq == 0) return hipSuccess;
    int blk = 256;
    hipLaunchKernelGGL(k_gather, dim3((b.nq + blk - 1) / blk), dim3(blk), 0, st, b);
    TDS_LAUNCH_CHECK();
}

// --------------------------------------------------------------- tiles
// One thread per sorted position. A head position writes its tile: the
// queries up to the next head and the union of their candidate ranges; the
// number of work items is ceil(range / chunk). Positions past the last tile
// write zero items so that the item scan can run over nq slots.
__global__ void k_tiles(DevBatch b) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long ev = 0;
    if (p < b.nq) {
        int n_tiles;
        int t;
        if (b.tiling == kTilePeriodic) {
            n_tiles = (b.nq + b.s - 1) / b.s;
            t = (p % b.s == 0) ? p / b.s : -1;
        } else {
            n_tiles = b.tile_of_head[b.nq - 1] + b.head[b.nq - 1];
            t = b.head[p] ? b.tile_of_head[p] : -1;
        }
        if (p >= n_tiles) b.items[p] = 0;
        if (p == 0) b.ctr->n_tiles = (unsigned)n_tiles;
        if (t >= 0) {
            int end = p + 1;
            while (end < b.nq && end - p < b.s && !b.head[end]) ++end;
            int lo = 0x7fffffff, hi = -1;
            for (int k = p; k < end; ++k) {
                int f = b.first_s[k], l = b.last_s[k];
                if (l >= f) {
                    lo = min(lo, f);
                    hi = max(hi, l);
                }
            }
            Tile tl;
            tl.q0 = p;
            tl.nq = end - p;
            tl.e0 = hi >= lo ? lo : 0;
            tl.ne = hi >= lo ? hi - lo + 1 : 0;
            b.tiles[t] = tl;
            b.items[t] = (tl.ne + b.chunk - 1) / b.chunk;
            ev = (unsigned long long)tl.nq * (unsigned long long)tl.ne;
        }
    }
    ev = wave_sum_u64(ev);
    if (lane_id() == 0 && ev) atomicAdd(&b.ctr->n_eval, ev);
}

hipError_t launch_tiles(DevBatch b, hipStream_t st) {
    if (b.nq == 0) return hipSuccess;
    int blk = 256;
    hipLaunchKernelGGL(k_tiles, dim3((b.nq + blk - 1) / blk), dim3(blk), 0, st, b);
    TDS_LAUNCH_CHECK();
}

// --------------------------------------------------------------- pair test
// Kernel arguments of the pair kernel. Uniform tables (query records,
// tiles, item offsets) are separate restrict-qualified pointers so that
// their wave-uniform loads can go through the scalar cache.
struct PairArgs {
    Hit24 *out;
    unsigned long long cap;
    Counters *ctr;
};

// The binary64 decision and, for hits, the interval (stable roots of the
// quadratic, clamped to the common span).
__device__ __forceinline__ bool pair64(const QRec64 &q, double et0, double et1, double ex0,
                                       double ey0, double ez0, double evx, double evy, double evz,
                                       bool *ovl, double *ta, double *tb, bool want_interval) {
    double tlo = dmx(q.t0, et0);
    double thi = dmn(q.t1, et1);
    *ovl = tlo < thi;
    if (!*ovl) return false;
    double T = thi - tlo;
    double tq = tlo - q.t0;
    double te = tlo - et0;
    double Dx = __builtin_fma(q.vx, tq, q.x0) - __builtin_fma(evx, te, ex0);
    double Dy = __builtin_fma(q.vy, tq, q.y0) - __builtin_fma(evy, te, ey0);
    double Dz = __builtin_fma(q.vz, tq, q.z0) - __builtin_fma(evz, te, ez0);
    double Vx = q.vx - evx;
    double Vy = q.vy - evy;
    double Vz = q.vz - evz;
    double a = __builtin_fma(Vz, Vz, __builtin_fma(Vy, Vy, Vx * Vx));
    double B = __builtin_fma(Dz, Vz, __builtin_fma(Dy, Vy, Dx * Vx));
    double c = __builtin_fma(Dz, Dz, __builtin_fma(Dy, Dy, __builtin_fma(Dx, Dx, -q.dd)));
    bool in0 = c <= 0.0;
    bool inT = __builtin_fma(__builtin_fma(a, T, B + B), T, c) <= 0.0;
    bool vtx = (B < 0.0) && (__builtin_fma(a, T, B) > 0.0) && (__builtin_fma(B, B, -(a * c)) >= 0.0);
    bool hit = in0 || inT || vtx;
    if (want_interval && hit) {
        if (in0 && inT) {
            *ta = tlo;
            *tb = thi;
        } else {
            double h = __builtin_fma(B, B, -(a * c));
            if (h < 0.0) h = 0.0;
            double s = sqrt(h);
            double qq = (B >= 0.0) ? -(B + s) : (s - B);
            double r1 = qq / a;
            double r2 = (qq != 0.0) ? c / qq : r1;
            double lo = dmn(r1, r2);
            double hi = dmx(r1, r2);
            double xa = in0 ? tlo : tlo + dmx(lo, 0.0);
            double xb = inT ? thi : tlo + dmn(hi, T);
            if (xa > xb) {
                double tv = dmn(dmx(-B / a, 0.0), T);
                xa = tlo + tv;
                xb = xa;
            }
            *ta = xa;
            *tb = xb;
        }
    }
    return hit;
}

// Wave-aggregated append: one atomic per wave, lanes place their records by
// their rank among the wave's hit lanes. Records past `cap` are counted but
// not stored (the host re-runs with a larger buffer).
__device__ __forceinline__ void emit(bool hit, uint32_t q, uint32_t e, double ta, double tb,
                                     Hit24 *__restrict__ out, unsigned long long cap,
                                     Counters *__restrict__ ctr) {
    unsigned long long m = __ballot(hit);
    if (m == 0ull) return;
    unsigned lane = lane_id();
    int leader = __ffsll((long long)m) - 1;
    unsigned long long base = 0;
    if ((int)lane == leader) base = atomicAdd(&ctr->hits, (unsigned long long)__popcll(m));
    base = __shfl(base, leader);
    if (hit) {
        unsigned rank = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        unsigned long long pos = base + rank;
        if (pos < cap) {
            Hit24 r;
            r.q = q;
            r.e = e;
            r.ta = ta;
            r.tb = tb;
            out[pos] = r;
        }
    }
}

// Tile of work item `it`: last t with item_off[t] <= it (tiles with zero
// items share their successor's offset, so this is the tile that owns it).
__device__ __forceinline__ int tile_of_item(const int32_t *off, int n, int it) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= it) lo = mid + 1; else hi = mid;
    }
    return lo - 1;
}

template <int MODE, int BLOCK, int EPT, bool COUNT_OVL>
__global__ __launch_bounds__(BLOCK) void k_pair(const QRec64 *__restrict__ rec,
                                                const QBox32 *__restrict__ box,
                                                const Tile *__restrict__ tiles,
                                                const int32_t *__restrict__ items,
                                                const int32_t *__restrict__ item_off, int nslots,
                                                DevIndex ix, Hit24 *__restrict__ out,
                                                unsigned long long cap, Counters *__restrict__ ctr) {
    const int tid = threadIdx.x;
    const int total = item_off[nslots - 1] + items[nslots - 1];
    if (blockIdx.x == 0 && tid == 0) ctr->n_items = (unsigned)total;
    unsigned long long ovl_acc = 0, ref_acc = 0;
    constexpr int CHUNK = BLOCK * EPT;
    for (int it = blockIdx.x; it < total; it += gridDim.x) {
        const int t = tile_of_item(item_off, nslots, it);
        const Tile tl = tiles[t];
        const int c = it - item_off[t];
        const int eb = tl.e0 + c * CHUNK;
        const int ee = min(tl.e0 + tl.ne, eb + CHUNK);

        if constexpr (MODE == kModeFP64) {
            double et0[EPT], et1[EPT], ex0[EPT], ey0[EPT], ez0[EPT], evx[EPT], evy[EPT], evz[EPT];
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                int e = eb + j * BLOCK + tid;
                if (e < ee) {
                    et0[j] = ix.t0[e];
                    et1[j] = ix.t1[e];
                    ex0[j] = ix.x0[e];
                    ey0[j] = ix.y0[e];
                    ez0[j] = ix.z0[e];
                    evx[j] = ix.vx[e];
                    evy[j] = ix.vy[e];
                    evz[j] = ix.vz[e];
                } else {  // an empty span never overlaps
                    et0[j] = INFINITY;
                    et1[j] = -INFINITY;
                    ex0[j] = ey0[j] = ez0[j] = evx[j] = evy[j] = evz[j] = 0.0;
                }
            }
            for (int qi = 0; qi < tl.nq; ++qi) {
                const int qs = tl.q0 + qi;
                const QRec64 q = rec[qs];
#pragma unroll
                for (int j = 0; j < EPT; ++j) {
                    bool ovl;
                    double ta = 0.0, tb = 0.0;
                    bool hit = pair64(q, et0[j], et1[j], ex0[j], ey0[j], ez0[j], evx[j], evy[j],
                                      evz[j], &ovl, &ta, &tb, true);
                    if (COUNT_OVL) ovl_acc += __popcll(__ballot(ovl));
                    emit(hit, (uint32_t)qs, (uint32_t)(eb + j * BLOCK + tid), ta, tb, out, cap, ctr);
                }
            }
        } else {
            float4 ba[EPT], bb[EPT];
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                int e = eb + j * BLOCK + tid;
                if (e < ee) {
                    ba[j] = ix.boxa[e];
                    bb[j] = ix.boxb[e];
                } else {  // an empty span never overlaps
                    ba[j] = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
                    bb[j] = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
                }
            }
            for (int qi = 0; qi < tl.nq; ++qi) {
                const int qs = tl.q0 + qi;
                const QBox32 qb = box[qs];
#pragma unroll
                for (int j = 0; j < EPT; ++j) {
                    bool tov = (qb.t0 < ba[j].y) & (ba[j].x < qb.t1);
                    if (COUNT_OVL) ovl_acc += __popcll(__ballot(tov));
                    bool pass = tov & (ba[j].z <= qb.xhi) & (qb.xlo <= ba[j].w) &
                                (bb[j].x <= qb.yhi) & (qb.ylo <= bb[j].y) & (bb[j].z <= qb.zhi) &
                                (qb.zlo <= bb[j].w);
                    unsigned long long pm = __ballot(pass);
                    if (pm) {
                        ref_acc += __popcll(pm);
                        const QRec64 q = rec[qs];
                        const int e = eb + j * BLOCK + tid;
                        bool hit = false;
                        double ta = 0.0, tb = 0.0;
                        if (pass) {
                            bool ovl;
                            hit = pair64(q, ix.t0[e], ix.t1[e], ix.x0[e], ix.y0[e], ix.z0[e],
                                         ix.vx[e], ix.vy[e], ix.vz[e], &ovl, &ta, &tb, true);
                        }
                        emit(hit, (uint32_t)qs, (uint32_t)e, ta, tb, out, cap, ctr);
                    }
                }
            }
        }
    }
    if (lane_id() == 0) {
        if (COUNT_OVL && ovl_acc) atomicAdd(&ctr->overlap, ovl_acc);
        if (MODE == kModeFP32Refine && ref_acc) atomicAdd(&ctr->refine, ref_acc);
    }
}

// Entries per lane and work item for a mode and block size.
int ept_for(int mode, int block) { return (block >= 512) ? 1 : (mode == kModeFP64 ? 2 : 4); }
int chunk_for(int mode, int block) { return block * ept_for(mode, block); }

template <int MODE, int BLOCK>
static hipError_t launch_pair_b(DevBatch b, DevIndex ix, int grid, int count_overlap, Hit24 *out,
                                unsigned long long cap, hipStream_t st) {
    constexpr int EPT = (BLOCK >= 512) ? 1 : (MODE == kModeFP64 ? 2 : 4);
    if (count_overlap)
        hipLaunchKernelGGL((k_pair<MODE, BLOCK, EPT, true>), dim3(grid), dim3(BLOCK), 0, st,
                           b.rec_s, b.box_s, b.tiles, b.items, b.item_off, b.nq, ix, out, cap, b.ctr);
    else
        hipLaunchKernelGGL((k_pair<MODE, BLOCK, EPT, false>), dim3(grid), dim3(BLOCK), 0, st,
                           b.rec_s, b.box_s, b.tiles, b.items, b.item_off, b.nq, ix, out, cap, b.ctr);
    TDS_LAUNCH_CHECK();
}

hipError_t launch_pair(DevBatch b, DevIndex ix, int mode, int block, int grid, int count_overlap,
                       Hit24 *out, unsigned long long cap, hipStream_t st) {
    if (b.nq == 0) return hipSuccess;
#define TDS_PAIR_CASE(M, BS) \
    case BS: return launch_pair_b<M, BS>(b, ix, grid, count_overlap, out, cap, st);
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

// --------------------------------------------------------------- translate
__global__ void k_translate(const Hit24 *__restrict__ in, int64_t n, const int32_t *__restrict__ perm,
                            DevIndex ix, int64_t *out) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    Hit24 h = in[k];
    int64_t *o = out + 5 * k;
    o[0] = perm[h.q];
    o[1] = ix.orig[h.e];
    o[2] = ix.traj[h.e];
    o[3] = __double_as_longlong(h.ta);
    o[4] = __double_as_longlong(h.tb);
}

hipError_t launch_translate(const Hit24 *in, int64_t n, const int32_t *perm, DevIndex ix,
                            void *out_hits, hipStream_t st) {
    if (n == 0) return hipSuccess;
    int blk = 256;
    int64_t grid = (n + blk - 1) / blk;
    hipLaunchKernelGGL(k_translate, dim3((unsigned)grid), dim3(blk), 0, st, in, n, perm, ix,
                       (int64_t *)out_hits);
    TDS_LAUNCH_CHECK();
}

__global__ void k_zero(unsigned *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t launch_zero_counters(Counters *c, hipStream_t st) {
    int n = (int)(sizeof(Counters) / sizeof(unsigned));
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, (unsigned *)c, n);
    TDS_LAUNCH_CHECK();
}

}  // namespace tds
