// GreedySetSplit tiles (Sec. 6, Alg. 4) built on the device.
//
// The algorithm walks the query segments in t_start order twice. Its first
// pass merges neighbours while the merge adds no interactions. A batch costs
// (its segments) x (entries of the candidate range of its temporal extent,
// Sec. 4), and a merged batch's range holds both ranges, so a merge is free
// exactly when the two ranges and the range of the merged extent are one and
// the same. Two conditions mark where a new group ("free-merge group")
// starts: the segment's range differs from its predecessor's (one flag per
// position), or, inside a run of identical ranges, the extent of the group
// so far grows into a bin that none of its members overlaps (a bin lying in
// a gap between their spans). The second is rare; one wave walks each run of
// identical ranges to find it.
//
// The second pass is sequential in the paper: a batch takes the following
// groups while it holds fewer than `bound` segments (Min), or while the
// merged batch stays within `bound` (Max). Which group starts the batch
// after a batch starting at group g depends only on g (next(g), a binary
// search over the group start positions), so the batch starts are the chain
// 0, next(0), next(next(0)), ... It is marked in parallel by pointer
// doubling: jump_k(g) = next^(2^k)(g) for k < L, then top down the chain
// nodes at multiples of 2^k are the ones at multiples of 2^(k+1) and their
// jump_k images. L levels cover chains of fewer than 2^L batches.
//
// Launches: the exact (t_start, caller index) order within each t_start bin
// (the query preparation's counting sort already orders the bins; this
// launch also orders Periodic tiling); the run flags; the walk of the runs of
// identical ranges; one workgroup for groups, chain and batch starts (in LDS
// when there are fewer than kChainLds groups); the tiles; one workgroup for
// the unit offsets.
#include <hip/hip_runtime.h>

#include "tds_internal.h"

namespace tds {

namespace {

// Exact (t_start, caller index) order within each t_start bin (the bins
// are already in order: the counting sort of the query preparation put the
// segments of bin k at positions bq_off[k] .. bq_off[k] + bcount[k] - 1, in
// no particular order, with their keys in skey / sidx). The key (order bits
// of t_start, caller index) is unique, so a segment's place is its bin
// offset plus the number of bin members with a smaller key. Blocks below
// nbuckets take one bin of at most kSortLds segments each and rank it in
// LDS: by counting (broadcast reads) up to kCountMax segments, by a bitonic
// network above (counting is quadratic: at 512 segments it took 65 us on a
// batch where the network takes 23 us). The blocks after them, one per
// window of kSortLds positions, sort the pieces of larger bins into tkey /
// tidx for k_gs_merge_big (such bins are rare; k_bucket_scan counts them,
// and with none these blocks return at once). Reads go to skey / sidx only
// and writes to perm, first_s, last_s, tkey, tidx only, so no block sees
// another's writes.
constexpr int kSortBlock = 256;
#ifndef TDS_COUNT_MAX
#define TDS_COUNT_MAX 64
#endif
constexpr int kCountMax = TDS_COUNT_MAX;

// Bitonic network over P = E * kSortBlock keys (padding sorts last) held in
// registers: element p = k * kSortBlock + thread is slot k of that thread.
// A compare-exchange at distance d pairs slots of one thread (d >=
// kSortBlock), lanes of one wave through shuffles (d < 64), or lanes of
// different waves through LDS (64 <= d < kSortBlock), so only the LDS steps
// need the workgroup barrier.
__device__ __forceinline__ bool key_gt(unsigned long long ka, int ia, unsigned long long kb, int ib) {
    return ka > kb || (ka == kb && ia > ib);
}

template <int E, class Put>
__device__ void bitonic_block(const DevBatch &b, int off, int cnt, unsigned long long *s_key,
                              int32_t *s_idx, Put put) {
    const int tid = threadIdx.x;
    constexpr int P = E * kSortBlock;
    unsigned long long key[E];
    int idx[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const int p = k * kSortBlock + tid;
        key[k] = p < cnt ? b.skey[off + p] : ~0ull;
        idx[k] = p < cnt ? b.sidx[off + p] : 0x7fffffff;
    }
    for (int size = 2; size <= P; size <<= 1) {
        for (int d = size >> 1; d > 0; d >>= 1) {
            if (d >= kSortBlock) {
                const int ks = d / kSortBlock;
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    if (k & ks) continue;
                    const int k2 = k | ks;
                    const bool up = ((k * kSortBlock + tid) & size) == 0;
                    if (key_gt(key[k], idx[k], key[k2], idx[k2]) == up) {
                        const unsigned long long tk = key[k];
                        const int ti = idx[k];
                        key[k] = key[k2];
                        idx[k] = idx[k2];
                        key[k2] = tk;
                        idx[k2] = ti;
                    }
                }
                continue;
            }
            const bool lower = (tid & d) == 0;  // this element precedes its partner
            if (d >= 64) {
                __syncthreads();  // the previous LDS step has been read
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    s_key[k * kSortBlock + tid] = key[k];
                    s_idx[k * kSortBlock + tid] = idx[k];
                }
                __syncthreads();
            }
#pragma unroll
            for (int k = 0; k < E; ++k) {
                unsigned long long pk;
                int pi;
                if (d >= 64) {
                    pk = s_key[(k * kSortBlock + tid) ^ d];
                    pi = s_idx[(k * kSortBlock + tid) ^ d];
                } else {
                    const unsigned lo = __shfl_xor((unsigned)key[k], d);
                    const unsigned hi = __shfl_xor((unsigned)(key[k] >> 32), d);
                    pk = ((unsigned long long)hi << 32) | lo;
                    pi = __shfl_xor(idx[k], d);
                }
                const bool up = ((k * kSortBlock + tid) & size) == 0;
                // the lower element keeps the smaller key when ascending
                const bool gt = key_gt(key[k], idx[k], pk, pi);
                if (lower == up ? gt : !gt) {
                    key[k] = pk;
                    idx[k] = pi;
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const int p = k * kSortBlock + tid;
        if (p < cnt) put(off + p, key[k], idx[k]);
    }
}

__global__ __launch_bounds__(kSortBlock) void k_gs_bin_sort(DevBatch b) {
    __shared__ unsigned long long s_key[kSortLds];
    __shared__ int32_t s_idx[kSortLds];
    const int tid = threadIdx.x;
    auto put = [&](int p, int i) {
        b.perm[p] = i;
        b.first_s[p] = b.first[i];
        b.last_s[p] = b.last[i];
    };
    auto put3 = [&](int p, unsigned long long, int i) { put(p, i); };
    if ((int)blockIdx.x >= b.nbuckets) {
        // Bins too large for LDS: window w of kSortLds positions sorts its
        // piece of each such bin it meets (at most two) into tkey / tidx at
        // the same positions; k_gs_merge_big then ranks across pieces.
        if (b.ctr->big_bins == 0) return;
        const int ns = (int)b.ctr->n_sorted;
        const int w0 = ((int)blockIdx.x - b.nbuckets) * kSortLds;
        const int wend = min(ns, w0 + kSortLds);
        auto keep = [&](int p, unsigned long long kk, int i) {
            b.tkey[p] = kk;
            b.tidx[p] = i;
        };
        for (int p0 = w0; p0 < wend;) {
            const int k = b.key[b.sidx[p0]];
            const int cnt = b.bcount[k], off = b.bq_off[k];
            const int pend = min(wend, off + cnt);
            if (cnt > kSortLds) {
                const int len = pend - p0;
                int P = kSortBlock;
                while (P < len) P <<= 1;
                switch (P / kSortBlock) {
                case 1: bitonic_block<1>(b, p0, len, s_key, s_idx, keep); break;
                case 2: bitonic_block<2>(b, p0, len, s_key, s_idx, keep); break;
                case 4: bitonic_block<4>(b, p0, len, s_key, s_idx, keep); break;
                default: bitonic_block<8>(b, p0, len, s_key, s_idx, keep); break;
                }
            }
            p0 = pend;
        }
        return;
    }
    const int k = blockIdx.x;
    const int cnt = b.bcount[k];
    if (cnt <= 0 || cnt > kSortLds) return;
    const int off = b.bq_off[k];
    if (cnt <= kCountMax) {
        for (int p = tid; p < cnt; p += kSortBlock) {
            s_key[p] = b.skey[off + p];
            s_idx[p] = b.sidx[off + p];
        }
        __syncthreads();
        for (int p = tid; p < cnt; p += kSortBlock) {
            const unsigned long long mine = s_key[p];
            const int i = s_idx[p];
            int rank = 0;
#pragma unroll 8
            for (int q = 0; q < cnt; ++q) {
                const unsigned long long o = s_key[q];
                rank += (o < mine || (o == mine && s_idx[q] < i)) ? 1 : 0;
            }
            put(off + rank, i);
        }
        return;
    }
    int P = kSortBlock;
    while (P < cnt) P <<= 1;
    switch (P / kSortBlock) {
    case 1: bitonic_block<1>(b, off, cnt, s_key, s_idx, put3); break;
    case 2: bitonic_block<2>(b, off, cnt, s_key, s_idx, put3); break;
    case 4: bitonic_block<4>(b, off, cnt, s_key, s_idx, put3); break;
    default: bitonic_block<8>(b, off, cnt, s_key, s_idx, put3); break;
    }
}

// Ranks of the members of bins too large for LDS (after k_gs_bin_sort sorted
// their pieces, one per window of kSortLds positions): a member's place in
// its bin is its index in its own sorted piece plus, for every other piece of
// the bin, the number of that piece's keys below it (a binary search), so a
// bin of n segments costs n (n / kSortLds) log2(kSortLds) reads rather than
// n^2. Returns at once when there are no such bins.
__global__ void k_gs_merge_big(DevBatch b) {
    if (b.ctr->big_bins == 0) return;
    const int ns = (int)b.ctr->n_sorted;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < ns; p += gridDim.x * blockDim.x) {
        const int k = b.key[b.sidx[p]];  // positions keep their bin in both orders
        const int cnt = b.bcount[k];
        if (cnt <= kSortLds) continue;
        const int off = b.bq_off[k], end = off + cnt;
        const unsigned long long mine = b.tkey[p];
        const int i = b.tidx[p];
        const int wp = p / kSortLds;
        int rank = p - max(off, wp * kSortLds);
        for (int w = off / kSortLds; w * kSortLds < end; ++w) {
            if (w == wp) continue;
            int lo = max(off, w * kSortLds), hi = min(end, (w + 1) * kSortLds);
            const int base = lo;
            while (lo < hi) {  // first key of the piece above mine
                const int mid = (lo + hi) >> 1;
                const unsigned long long o = b.tkey[mid];
                if (o < mine || (o == mine && b.tidx[mid] < i)) lo = mid + 1; else hi = mid;
            }
            rank += lo - base;
        }
        const int q = off + rank;
        b.perm[q] = i;
        b.first_s[q] = b.first[i];
        b.last_s[q] = b.last[i];
    }
}

// Run-start flags of the sorted order (one byte per position: 1 where the
// candidate range differs from the previous position's; positions past the
// segments with candidates, up to the next multiple of 16, get 0). k_gs_hull
// adds 2 where a run of identical ranges splits; every group start is a
// nonzero byte with one bit set.
__global__ void k_gs_flags(DevBatch b, GreedyBufs g, int n16) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n16) return;
    const int nv = (int)b.ctr->n_sorted;
    uint8_t flag = 0;
    if (p < nv)
        flag = (p == 0 || b.first_s[p] != b.first_s[p - 1] || b.last_s[p] != b.last_s[p - 1]) ? 1 : 0;
    g.flag[p] = flag;
}

// Splits of the runs of identical ranges (the second condition above). Wave w
// takes positions 64 w .. 64 w + 63 and walks every run that starts among
// them (flag 1). A run with range R = bins J1..J2 groups segments from its
// current group start s while every member's t_end stays at or below lim(s),
// the start of the first bin after J2 that ends after t_start(s): the
// group's extent (t_start(s), largest t_end) then overlaps no bin beyond J2,
// and none before J1 either (those end at or before every member's start).
// The first member past lim(s) starts the next group (flag 2). The walk also
// records each group's largest t_end (gmax at its start) for the tiles. Only
// positions inside the wave's own runs are written, and a run's end is found
// from the ranges, not from flags, so walks of different waves do not meet.
__device__ __forceinline__ double gs_limit(const DevIndex &ix, int j2, double a) {
    const int J = bins_first_end_above(ix.btree, ix.bleaf, ix.nb, j2 + 1, a);
    return J < ix.nb ? ix.bstart[J] : INFINITY;
}

__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

__global__ void k_gs_hull(DevBatch b, GreedyBufs g, DevIndex ix) {
    const int lane = threadIdx.x & 63;
    const int nv = (int)b.ctr->n_sorted;
    const int nwaves = (int)(gridDim.x * (blockDim.x >> 6));
    for (int c0 = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64; c0 < nv; c0 += nwaves * 64) {
        unsigned long long starts = __ballot(c0 + lane < nv && g.flag[c0 + lane] == 1);
        while (starts) {
            const int r0 = c0 + __ffsll((long long)starts) - 1;
            starts &= starts - 1;
            const int f = b.first_s[r0], l = b.last_s[r0];
            const QRec64 q0 = b.rec[b.perm[r0]];
            int j1 = 0, j2 = -1;
            (void)bins_of_interval(ix.bstart, ix.bpend, ix.btree, ix.bleaf, ix.nb, q0.t0, q0.t1, &j1, &j2);
            int s = r0;
            double lim = gs_limit(ix, j2, q0.t0), mx = q0.t1;
            for (int p0 = r0 + 1;; p0 += 64) {
                const int p = p0 + lane;
                const bool in = p < nv && b.first_s[p] == f && b.last_s[p] == l;
                const unsigned long long out = __ballot(!in);
                const int nin = out ? __ffsll((long long)out) - 1 : 64;  // run members p0 .. p0 + nin - 1
                const bool act = lane < nin;
                const double t1 = act ? b.rec[b.perm[p]].t1 : -INFINITY;
                int from = 0;  // lanes below `from` belong to earlier groups
                for (;;) {
                    const unsigned long long bad = __ballot(act && lane >= from && t1 > lim);
                    if (bad == 0ull) break;
                    const int k = __ffsll((long long)bad) - 1;
                    mx = fmax(mx, wave_max(lane >= from && lane < k ? t1 : -INFINITY));
                    if (lane == 0) g.gmax[s] = mx;
                    s = p0 + k;
                    if (lane == 0) g.flag[s] = 2;
                    lim = gs_limit(ix, j2, b.rec[b.perm[s]].t0);
                    mx = __shfl(t1, k);
                    from = k + 1;
                }
                mx = fmax(mx, wave_max(act && lane >= from ? t1 : -INFINITY));
                if (nin < 64) break;
            }
            if (lane == 0) g.gmax[s] = mx;
        }
    }
}

constexpr int kChainBlock = 1024;
constexpr int kChainLds = 1024;     // groups + 1 held in LDS
constexpr int kChainLdsLevels = 10; // 2^10 > any chain of fewer than kChainLds groups

// Exclusive scan of one value per thread over the block; the block total
// goes to *total.
__device__ long long gs_block_scan(long long v, long long *total) {
    __shared__ long long sums[kChainBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    long long incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        const long long y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    if (lane == 63) sums[w] = incl;
    __syncthreads();
    if (w == 0) {
        long long s = lane < kChainBlock / 64 ? sums[lane] : 0;
        for (int off = 1; off < 64; off <<= 1) {
            const long long y = __shfl_up(s, off);
            if (lane >= off) s += y;
        }
        if (lane < kChainBlock / 64) sums[lane] = s;
    }
    __syncthreads();
    const long long before = w > 0 ? sums[w - 1] : 0;
    *total = sums[kChainBlock / 64 - 1];
    __syncthreads();
    return before + incl - v;
}

__device__ __forceinline__ int flag_count(const uint4 v) {
    return __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w);  // bytes are 0, 1 or 2
}

// One workgroup: groups (run starts), next(), the doubling levels, the
// chain marks and the batch starts. Writes gpos, gb and cnt to global memory.
__global__ __launch_bounds__(kChainBlock) void k_gs_chain(DevBatch b, GreedyBufs g, int bound,
                                                          int is_max) {
    __shared__ int32_t s_gpos[kChainLds];
    __shared__ int32_t s_mark[kChainLds];
    __shared__ int32_t s_jump[kChainLdsLevels * kChainLds];
    const int tid = threadIdx.x;
    const int nv = (int)b.ctr->n_sorted;

    // groups: each thread counts the flags of a run of 16-byte words
    const int nw = (nv + 15) >> 4;
    const int per = (nw + kChainBlock - 1) / kChainBlock;
    const int w0 = min(nw, tid * per), w1 = min(nw, w0 + per);
    const uint4 *fw = reinterpret_cast<const uint4 *>(g.flag);
    long long c = 0;
    for (int k = w0; k < w1; ++k) c += flag_count(fw[k]);
    long long gtot;
    long long base = gs_block_scan(c, &gtot);
    const int G = (int)gtot;
    const bool lds = G + 1 <= kChainLds;
    int32_t *gp = lds ? s_gpos : g.gpos;
    int32_t *jp = lds ? s_jump : g.jump;
    int32_t *mk = lds ? s_mark : g.mark;
    const size_t stride = lds ? (size_t)kChainLds : (size_t)g.stride;
    for (int k = w0; k < w1; ++k) {
        const uint4 v = fw[k];
        const uint32_t words[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if ((words[q] >> (8 * j)) & 0xffu) gp[base++] = k * 16 + q * 4 + j;
    }
    if (tid == 0) gp[G] = nv;
    __syncthreads();

    // levels: 2^L > G >= chain length (the global buffer holds g.levels)
    int L = 1;
    while ((1 << L) <= G) ++L;
    if (!lds) L = min(L, g.levels);

    for (int x = tid; x <= G; x += kChainBlock) {
        int h = G;
        if (x < G) {
            const long long target = (long long)gp[x] + bound;
            if (!is_max) {  // smallest h > x with gpos[h] >= gpos[x] + bound, else G
                int lo = x + 1, hi = G;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if ((long long)gp[mid] >= target) hi = mid; else lo = mid + 1;
                }
                h = lo;
            } else {  // largest h with gpos[h] <= gpos[x] + bound, at least x + 1
                int lo = x + 1, hi = G + 1;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if ((long long)gp[mid] > target) hi = mid; else lo = mid + 1;
                }
                h = max(x + 1, lo - 1);
            }
        }
        jp[x] = h;
        mk[x] = (x == 0 && G > 0) ? L : -1;
    }
    __syncthreads();
    for (int k = 1; k < L; ++k) {  // jump_k = jump_{k-1} o jump_{k-1}
        const int32_t *prev = jp + (size_t)(k - 1) * stride;
        int32_t *cur = jp + (size_t)k * stride;
        for (int x = tid; x <= G; x += kChainBlock) cur[x] = prev[prev[x]];
        __syncthreads();
    }
    // Chain nodes found above level k map to the nodes 2^k further on; a
    // node marked at level k is not a source at level k, so no thread of a
    // level reads a mark another thread of the same level writes.
    for (int k = L - 1; k >= 0; --k) {
        const int32_t *jk = jp + (size_t)k * stride;
        for (int x = tid; x < G; x += kChainBlock) {
            if (mk[x] > k) {
                const int y = jk[x];
                if (y < G) mk[y] = k;
            }
        }
        __syncthreads();
    }

    // batch starts: the marked groups, numbered in order
    const int perg = (G + kChainBlock - 1) / kChainBlock;
    const int x0 = min(G, tid * perg), x1 = min(G, x0 + perg);
    long long nb_loc = 0;
    for (int x = x0; x < x1; ++x) nb_loc += mk[x] >= 0 ? 1 : 0;
    long long nbt;
    long long bpos = gs_block_scan(nb_loc, &nbt);
    for (int x = x0; x < x1; ++x)
        if (mk[x] >= 0) g.gb[bpos++] = x;
    if (lds)
        for (int x = tid; x <= G; x += kChainBlock) g.gpos[x] = s_gpos[x];
    if (tid == 0) {
        g.gb[nbt] = G;
        g.cnt[0] = G;
        g.cnt[1] = (int)nbt;
    }
}

// Tiles, one wave at a time (grid-stride over the batches): the members are
// the groups gb[t] .. gb[t+1]-1, the range is that of the batch's temporal
// extent (Sec. 4): from the first member's t_start to the largest t_end of
// its groups.
constexpr int kTileGrid = 1024;

__global__ void k_gs_tiles(DevBatch b, GreedyBufs g, DevIndex ix) {
    const int lane = threadIdx.x & 63;
    const int nwaves = (int)(gridDim.x * (blockDim.x >> 6));
    const int nb = g.cnt[1];
    for (int t = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6); t < nb; t += nwaves) {
        const int g0 = g.gb[t], g1 = g.gb[t + 1];
        double hi_t = -INFINITY;
        for (int k = g0 + lane; k < g1; k += 64) hi_t = fmax(hi_t, g.gmax[g.gpos[k]]);
        hi_t = wave_max(hi_t);
        if (lane == 0) {
            const int q0 = g.gpos[g0], nq = g.gpos[g1] - q0;
            int j1 = 0, j2 = -1;
            const bool any = bins_of_interval(ix.bstart, ix.bpend, ix.btree, ix.bleaf, ix.nb,
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
            g.tev[t] = (long long)nq * tl.ne;
        }
    }
}

// One block: unit and cost offsets of the tiles, the tile count, the work
// units and the interactions (n_eval).
__global__ __launch_bounds__(kChainBlock) void k_gs_unit_scan(DevBatch b, GreedyBufs g) {
    const int n = g.cnt[1];
    const int per = (n + kChainBlock - 1) / kChainBlock;
    const int lo = min(n, (int)threadIdx.x * per), hi = min(n, lo + per);
    long long s = 0, ev = 0, k_sum = 0;
    for (int k = lo; k < hi; ++k) {
        s += b.units[k];
        ev += g.tev[k];
        k_sum += tile_cost(b.tiles[k].nq, b.tiles[k].nchunk, b.pass_cost, b.stage_cost);
    }
    long long tot, ev_tot, k_tot;
    long long run = gs_block_scan(s, &tot);
    (void)gs_block_scan(ev, &ev_tot);
    long long k_run = gs_block_scan(k_sum, &k_tot);
    for (int k = lo; k < hi; ++k) {
        b.unit_off[k] = run;
        b.cost_off[k] = k_run;
        run += b.units[k];
        k_run += tile_cost(b.tiles[k].nq, b.tiles[k].nchunk, b.pass_cost, b.stage_cost);
    }
    if (threadIdx.x == 0) {
        b.unit_off[n] = tot;
        b.cost_off[n] = k_tot;
        b.ctr->n_tiles = (unsigned)n;
        b.ctr->n_units = (unsigned long long)tot;
        b.ctr->n_eval = (unsigned long long)ev_tot;
    }
}

}  // namespace

hipError_t launch_bucket_sort(DevBatch b, hipStream_t st) {
    const int nq = b.nq;
    if (nq <= 0 || !b.skey || !b.sidx) return hipErrorInvalidValue;
    // big-bin blocks only where a bin can exceed the LDS sort
    // one workgroup per window of kSortLds positions for bins larger than that
    const int wins = nq > kSortLds ? (nq + kSortLds - 1) / kSortLds : 0;
    hipLaunchKernelGGL(k_gs_bin_sort, dim3(b.nbuckets + wins), dim3(kSortBlock), 0, st, b);
    if (wins > 0) {
        const int need = (nq + kSortBlock - 1) / kSortBlock;
        hipLaunchKernelGGL(k_gs_merge_big, dim3(need < 1024 ? need : 1024), dim3(kSortBlock), 0, st, b);
    }
    return hipGetLastError();
}

hipError_t launch_greedy(DevBatch b, GreedyBufs g, DevIndex ix, int bound, int is_max,
                         hipStream_t st) {
    const int nq = b.nq;
    if (nq <= 0) return hipErrorInvalidValue;  // the caller skips an empty batch
    const int blk = 256;
    const int n16 = (nq + 15) & ~15;
    hipLaunchKernelGGL(k_gs_flags, dim3((n16 + blk - 1) / blk), dim3(blk), 0, st, b, g, n16);
    const int hgrid = (nq + blk - 1) / blk;  // one wave per 64 positions
    hipLaunchKernelGGL(k_gs_hull, dim3(hgrid < 4096 ? hgrid : 4096), dim3(blk), 0, st, b, g, ix);
    hipLaunchKernelGGL(k_gs_chain, dim3(1), dim3(kChainBlock), 0, st, b, g, bound, is_max);
    hipLaunchKernelGGL(k_gs_tiles, dim3(kTileGrid), dim3(blk), 0, st, b, g, ix);
    hipLaunchKernelGGL(k_gs_unit_scan, dim3(1), dim3(kChainBlock), 0, st, b, g);
    return hipGetLastError();
}

}  // namespace tds
