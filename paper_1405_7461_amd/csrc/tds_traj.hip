// Trajectory-level answers on the device: the segment-level hits of a batch
// merged into maximal intervals per (query trajectory, entry trajectory).
//
// The paper's query asks, per query trajectory, for the entry trajectories
// within d and when (Sec. 3); the segment-pair intervals of one trajectory
// pair are pieces of that answer, and their union is it. Steps: gather the
// hits with their two trajectory ids, sort by (query trajectory, entry
// trajectory, t_a), then one segmented running maximum of t_b (a single scan
// whose operator carries the pair-start flag) marks where a new maximal
// interval starts (its t_a lies after every earlier t_b of the pair; closed
// intervals that touch merge), and a scan of those marks numbers the output
// records. The sort: up to kTrajRankMax hits, each key's rank is the number
// of keys before it (counted by every workgroup of a grid over tiles of
// keys), a scatter puts them in order and one workgroup does the scans and
// the records (four launches); up to kTrajOneSortMax hits, one comparison
// merge sort of whole 32-byte keys; above that, three stable radix sorts
// (least significant key first).
#include <hip/hip_runtime.h>

#include <cstring>  // rocprim's headers use memset
#include <rocprim/rocprim.hpp>

#include "tds.h"
#include "tds_internal.h"

namespace tds {

namespace {

__device__ __forceinline__ unsigned long long order_bits(double x) {
    // ascending unsigned order of binary64 values (no NaN here)
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ unsigned long long order_bits(long long x) {
    return (unsigned long long)x ^ 0x8000000000000000ull;
}

// One wave per hit slab: dense hit k gets its trajectories and interval.
__global__ __launch_bounds__(256) void k_traj_gather(Slabs sl, const Counters *__restrict__ ctr,
                                                     const int64_t *__restrict__ qtraj_in,
                                                     DevIndex ix, TrajBufs t) {
    const int lane = threadIdx.x & 63;
    const long long nsl = (long long)ctr->n_slabs;
    const long long nw = (long long)gridDim.x * 4;
    for (long long s = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); s < nsl; s += nw) {
        if (lane < sl.slab_h[s]) {
            const long long k = sl.hit_off[s] + lane;
            const Hit24 h = sl.hits[s * kSlab + lane];
            t.qt[k] = qtraj_in[h.q];
            t.et[k] = ix.traj[h.e];
            t.ta[k] = h.ta;
            t.tb[k] = h.tb;
            t.key_a[k] = order_bits(h.ta);
            t.idx_a[k] = (int32_t)k;
            t.start[k] = 0;  // the rank accumulator of small merges
            if (t.kin) t.kin[k] = TrajKey{t.qt[k], t.et[k], h.ta, h.tb};
        }
    }
}

// key_out[i] = order bits of src[idx[i]] (the next, more significant key).
__global__ void k_traj_key(const int64_t *__restrict__ src, const int32_t *__restrict__ idx,
                           unsigned long long *__restrict__ key_out, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) key_out[i] = order_bits((long long)src[idx[i]]);
}

// Sorted order o = idx: pair-start flags and the sorted intervals.
__global__ void k_traj_flags(TrajBufs t, const int32_t *__restrict__ idx, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t o = idx[i];
    bool start = i == 0;
    if (!start) {
        const int32_t p = idx[i - 1];
        start = t.qt[o] != t.qt[p] || t.et[o] != t.et[p];
    }
    t.flag[i] = start ? 1 : 0;
    t.sta[i] = t.ta[o];
    t.seg_in[i] = SegMax{t.tb[o], start ? 1 : 0, 0};
}

// The same from the sorted whole keys of a small merge.
__global__ void k_traj_flags_one(TrajBufs t, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const TrajKey k = t.kout[i];
    bool start = i == 0;
    if (!start) {
        const TrajKey p = t.kout[i - 1];
        start = k.qt != p.qt || k.et != p.et;
    }
    t.flag[i] = start ? 1 : 0;
    t.sta[i] = k.ta;
    t.seg_in[i] = SegMax{k.tb, start ? 1 : 0, 0};
}

// A maximal interval starts where the pair starts or t_a exceeds the running
// maximum of the pair's earlier t_b.
__global__ void k_traj_starts(TrajBufs t, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool start = t.flag[i] || t.sta[i] > t.seg_out[i - 1].v;
    t.start[i] = start ? 1 : 0;
}

// Records: the first member gives the pair and t_a, the last member's
// running maximum is t_b.
__global__ void k_traj_emit(TrajBufs t, const int32_t *__restrict__ idx, long long n,
                            tds_traj_hit *__restrict__ out, long long *__restrict__ total) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long m = (long long)t.mid[i] - 1;
    if (t.start[i]) {
        if (idx) {
            const int32_t o = idx[i];
            out[m].query_traj = t.qt[o];
            out[m].entry_traj = t.et[o];
        } else {  // small merge: the sorted keys carry the ids
            out[m].query_traj = t.kout[i].qt;
            out[m].entry_traj = t.kout[i].et;
        }
        out[m].t_a = t.sta[i];
    }
    if (i == n - 1 || t.start[i + 1]) out[m].t_b = t.seg_out[i].v;
    if (i == n - 1) *total = m + 1;
}

// Segmented running maximum as one scan: a pair start resets the maximum
// (the usual flag-carrying operator, associative).
struct SegMaxOp {
    __device__ SegMax operator()(const SegMax &a, const SegMax &b) const {
        return SegMax{b.f ? b.v : (a.v > b.v ? a.v : b.v), a.f | b.f, 0};
    }
};
// (query trajectory, entry trajectory, t_a); equal keys may come in any
// order, as the merge takes the running maximum of their t_b
struct TrajLess {
    __device__ bool operator()(const TrajKey &a, const TrajKey &b) const {
        if (a.qt != b.qt) return a.qt < b.qt;
        if (a.et != b.et) return a.et < b.et;
        return a.ta < b.ta;
    }
};

// ------------------------------------------------ small merges by ranking
constexpr int kRankBlock = 256;   // keys i per workgroup (one per thread)
constexpr int kRankTile = 256;    // keys j per workgroup, staged in LDS

// Grid (i tiles, j tiles): each thread counts the keys of one j tile that
// precede its key i in the (query trajectory, entry trajectory, t_a) order,
// ties broken by position so that the ranks are a permutation, and adds the
// count to rank[i] (t.start, zeroed by the gather). The comparison is
// evaluated without branches (lane masks combined), the j keys are
// broadcast from LDS as three arrays and the loop is unrolled so that their
// reads overlap: n^2 / 64 comparisons per wave spread over the whole GPU.
__global__ __launch_bounds__(kRankBlock) void k_traj_rank(TrajBufs t, long long n) {
    __shared__ long long s_q[kRankTile], s_e[kRankTile];
    __shared__ double s_t[kRankTile];
    const long long i = (long long)blockIdx.x * kRankBlock + threadIdx.x;
    const long long j0 = (long long)blockIdx.y * kRankTile;
    const int nj = (int)min((long long)kRankTile, n - j0);
    for (int k = threadIdx.x; k < nj; k += kRankBlock) {
        const TrajKey kk = t.kin[j0 + k];
        s_q[k] = kk.qt;
        s_e[k] = kk.et;
        s_t[k] = kk.ta;
    }
    __syncthreads();
    if (i >= n) return;
    const TrajKey ki = t.kin[i];
    const long long lim = i - j0;  // tile slots k < lim hold keys at earlier positions
    int c = 0;
#pragma unroll 8
    for (int k = 0; k < nj; ++k) {
        const long long q = s_q[k], e = s_e[k];
        const double ta = s_t[k];
        const bool before =
            (q < ki.qt) |
            ((q == ki.qt) & ((e < ki.et) | ((e == ki.et) & ((ta < ki.ta) | ((ta == ki.ta) & (k < lim))))));
        c += before ? 1 : 0;
    }
    if (c) atomicAdd(&t.start[i], c);
}

// Sorted order: kout[rank[i]] = kin[i].
__global__ void k_traj_scatter(TrajBufs t, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) t.kout[t.start[i]] = t.kin[i];
}

constexpr int kMergeBlock = 1024;
constexpr int kMergeItems = (int)(kTrajRankMax / kMergeBlock);  // items per thread

// Inclusive scan of one value per thread over the workgroup (Hillis-Steele in
// LDS, s holds kMergeBlock values); afterwards s[k] is thread k's inclusive
// value.
template <class T, class Op>
__device__ __forceinline__ T block_scan_incl(T v, Op op, T *s) {
    const int tid = threadIdx.x;
    s[tid] = v;
    __syncthreads();
    for (int off = 1; off < kMergeBlock; off <<= 1) {
        const T o = tid >= off ? s[tid - off] : v;
        __syncthreads();
        if (tid >= off) v = op(o, v);
        s[tid] = v;
        __syncthreads();
    }
    return v;
}

struct IntPlus {
    __device__ int operator()(int a, int b) const { return a + b; }
};

// One workgroup over the sorted keys (n <= kTrajRankMax, consecutive items
// per thread): pair-start flags, the running maximum of t_b within each pair
// (segmented scan), the starts of maximal intervals (t_a beyond every earlier
// t_b of the pair), their record numbers (scan), and the records.
__global__ __launch_bounds__(kMergeBlock) void k_traj_merge_one(TrajBufs t, long long n,
                                                                tds_traj_hit *__restrict__ out,
                                                                long long *__restrict__ total) {
    __shared__ SegMax s_seg[kMergeBlock];
    __shared__ int s_cnt[kMergeBlock];
    const int tid = threadIdx.x;
    const long long b0 = (long long)tid * kMergeItems;
    TrajKey k[kMergeItems];
    bool f[kMergeItems];
    // pair-start flags and the thread's own segmented maximum
    SegMax agg{-INFINITY, 0, 0};
#pragma unroll
    for (int j = 0; j < kMergeItems; ++j) {
        const long long i = b0 + j;
        f[j] = false;
        if (i < n) {
            k[j] = t.kout[i];
            bool st = i == 0;
            if (!st) {
                const TrajKey p = j ? k[j - 1] : t.kout[i - 1];
                st = k[j].qt != p.qt || k[j].et != p.et;
            }
            f[j] = st;
            agg = SegMaxOp()(agg, SegMax{k[j].tb, st ? 1 : 0, 0});
        }
    }
    block_scan_incl(agg, SegMaxOp(), s_seg);
    // the segmented maximum over the earlier threads' items
    SegMax run = tid ? s_seg[tid - 1] : SegMax{-INFINITY, 0, 0};
    // starts of maximal intervals and the running maxima
    int cnt = 0;
    bool st[kMergeItems];
    double runmax[kMergeItems];
#pragma unroll
    for (int j = 0; j < kMergeItems; ++j) {
        const long long i = b0 + j;
        st[j] = false;
        runmax[j] = 0.0;
        if (i < n) {
            st[j] = f[j] || k[j].ta > run.v;
            run = SegMaxOp()(run, SegMax{k[j].tb, f[j] ? 1 : 0, 0});
            runmax[j] = run.v;
            cnt += st[j] ? 1 : 0;
        }
    }
    const int cinc = block_scan_incl(cnt, IntPlus(), s_cnt);
    long long m = (long long)(cinc - cnt) - 1;  // record of the last start before these items
#pragma unroll
    for (int j = 0; j < kMergeItems; ++j) {
        const long long i = b0 + j;
        if (i < n) {
            if (st[j]) {
                ++m;
                out[m].query_traj = k[j].qt;
                out[m].entry_traj = k[j].et;
                out[m].t_a = k[j].ta;
            }
            // the last item of a run gives its t_b: the next item starts a run
            bool last = i == n - 1;
            if (!last) {
                if (j + 1 < kMergeItems) {
                    last = st[j + 1];
                } else {
                    const TrajKey nx = t.kout[i + 1];
                    last = nx.qt != k[j].qt || nx.et != k[j].et || nx.ta > runmax[j];
                }
            }
            if (last) out[m].t_b = runmax[j];
            if (i == n - 1) *total = m + 1;
        }
    }
}

// Merge sort of the small merges: block sort of SortBlock x SortItems keys,
// then merge passes. Measured on 7,940 hits: 512 keys per block 0.149-0.155
// ms per merge, 1,024 0.17-0.18, rocprim's default for 32-byte keys 0.195
// (its block sort alone took 54 us); smaller configurations do not build.
#ifndef TDS_TRAJ_SORT_BLOCK
#define TDS_TRAJ_SORT_BLOCK 256
#endif
#ifndef TDS_TRAJ_SORT_ITEMS
#define TDS_TRAJ_SORT_ITEMS 2
#endif
using OneSortConfig = rocprim::merge_sort_config<TDS_TRAJ_SORT_BLOCK, TDS_TRAJ_SORT_BLOCK,
                                                 TDS_TRAJ_SORT_ITEMS>;

// All rocprim calls of one merge of n items; temp == nullptr only sizes.
hipError_t traj_rocprim(TrajBufs t, long long n, void *temp, size_t *temp_bytes, int step,
                        hipStream_t st) {
    size_t bytes = *temp_bytes;
    hipError_t e = hipSuccess;
    switch (step) {
    case 0:  // by t_a
        e = rocprim::radix_sort_pairs(temp, bytes, t.key_a, t.key_b, t.idx_a, t.idx_b, (size_t)n,
                                      0, 64, st);
        break;
    case 1:  // stable by entry trajectory (keys in key_a, values idx_b -> idx_a)
        e = rocprim::radix_sort_pairs(temp, bytes, t.key_a, t.key_b, t.idx_b, t.idx_a, (size_t)n,
                                      0, 64, st);
        break;
    case 2:  // stable by query trajectory (values idx_a -> idx_b)
        e = rocprim::radix_sort_pairs(temp, bytes, t.key_a, t.key_b, t.idx_a, t.idx_b, (size_t)n,
                                      0, 64, st);
        break;
    case 3:  // running maximum of t_b within a pair
        e = rocprim::inclusive_scan(temp, bytes, t.seg_in, t.seg_out, (size_t)n, SegMaxOp(), st);
        break;
    case 4:  // (no longer a separate step)
        bytes = 0;
        break;
    case 5:  // output record numbers
        e = rocprim::inclusive_scan(temp, bytes, t.start, t.mid, (size_t)n,
                                    rocprim::plus<int32_t>(), st);
        break;
    case 6:  // small merges: one sort of the whole keys
        e = rocprim::merge_sort<OneSortConfig>(temp, bytes, t.kin, t.kout, (size_t)n, TrajLess(), st);
        break;
    }
    *temp_bytes = bytes;
    return e;
}

}  // namespace

size_t traj_temp_bytes(long long n) {
    size_t most = 0;
    TrajBufs t{};
    for (int step = 0; step < 7; ++step) {
        if (step == 6 && n > kTrajOneSortMax) break;
        size_t b = 0;
        if (traj_rocprim(t, n, nullptr, &b, step, 0) != hipSuccess) return 0;
        most = b > most ? b : most;
    }
    return most;
}

hipError_t launch_traj_merge(Slabs sl, const Counters *ctr, long long n, const int64_t *qtraj,
                             DevIndex ix, TrajBufs t, void *temp,
                             size_t temp_bytes, tds_traj_hit *out, long long *total,
                             hipStream_t st) {
    if (n <= 0) return hipErrorInvalidValue;  // the caller handles a batch without hits
    const int blk = 256;
    const unsigned g = (unsigned)((n + blk - 1) / blk);
    const bool one = n <= kTrajOneSortMax;
    if (one && (!t.kin || !t.kout)) return hipErrorInvalidValue;
    if (!one) t.kin = t.kout = nullptr;
    hipLaunchKernelGGL(k_traj_gather, dim3(1024), dim3(256), 0, st, sl, ctr, qtraj, ix, t);
    if (n <= kTrajRankMax) {
        const dim3 rg((unsigned)((n + kRankBlock - 1) / kRankBlock), (unsigned)((n + kRankTile - 1) / kRankTile));
        hipLaunchKernelGGL(k_traj_rank, rg, dim3(kRankBlock), 0, st, t, n);
        hipLaunchKernelGGL(k_traj_scatter, dim3(g), dim3(blk), 0, st, t, n);
        hipLaunchKernelGGL(k_traj_merge_one, dim3(1), dim3(kMergeBlock), 0, st, t, n, out, total);
        return hipGetLastError();
    }
    hipError_t e;
    size_t b = temp_bytes;
    if (one) {
        if ((e = traj_rocprim(t, n, temp, &b, 6, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_traj_flags_one, dim3(g), dim3(blk), 0, st, t, n);
        b = temp_bytes;
        if ((e = traj_rocprim(t, n, temp, &b, 3, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_traj_starts, dim3(g), dim3(blk), 0, st, t, n);
        b = temp_bytes;
        if ((e = traj_rocprim(t, n, temp, &b, 5, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_traj_emit, dim3(g), dim3(blk), 0, st, t, (const int32_t *)nullptr, n,
                           out, total);
        return hipGetLastError();
    }
    if ((e = traj_rocprim(t, n, temp, &b, 0, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_traj_key, dim3(g), dim3(blk), 0, st, t.et, t.idx_b, t.key_a, n);
    b = temp_bytes;
    if ((e = traj_rocprim(t, n, temp, &b, 1, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_traj_key, dim3(g), dim3(blk), 0, st, t.qt, t.idx_a, t.key_a, n);
    b = temp_bytes;
    if ((e = traj_rocprim(t, n, temp, &b, 2, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_traj_flags, dim3(g), dim3(blk), 0, st, t, t.idx_b, n);
    b = temp_bytes;
    if ((e = traj_rocprim(t, n, temp, &b, 3, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_traj_starts, dim3(g), dim3(blk), 0, st, t, n);
    b = temp_bytes;
    if ((e = traj_rocprim(t, n, temp, &b, 5, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_traj_emit, dim3(g), dim3(blk), 0, st, t, t.idx_b, n, out, total);
    return hipGetLastError();
}

}  // namespace tds
