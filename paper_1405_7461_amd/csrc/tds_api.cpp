// Host runtime of the C ABI declared in include/tds.h: argument checks,
// index construction (sort by t_start, temporal bins, upload), query-batch
// orchestration on a HIP stream, overflow retry and result translation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "tds.h"
#include "tds_internal.h"

using namespace tds;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(e_ == hipErrorOutOfMemory ? TDS_ENOMEM : TDS_EDEVICE, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                \
    } while (0)

// A device allocation that only grows.
// Device allocator in force (tds_set_allocator); null functions = HIP.
struct DevAlloc {
    tds_alloc_fn alloc = nullptr;
    tds_free_fn free = nullptr;
    void *ctx = nullptr;
};
DevAlloc g_alloc;
// Stream of the library call in progress on this thread (passed to the hook).
thread_local void *g_call_stream = nullptr;

struct CallStream {  // sets g_call_stream for the duration of a library call
    void *prev;
    explicit CallStream(void *s) : prev(g_call_stream) { g_call_stream = s; }
    ~CallStream() { g_call_stream = prev; }
};

struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevAlloc by;          // allocator that made p
    void *stream = nullptr;
    hipError_t ensure(size_t need) {
        if (need <= bytes && p) return hipSuccess;
        if (p) {
            hipError_t e = free_now();
            if (e != hipSuccess) return e;
        }
        size_t nb = std::max<size_t>(need, 256);
        by = g_alloc;
        stream = g_call_stream;
        if (by.alloc) {
            p = by.alloc(nb, stream, by.ctx);
            if (!p) return hipErrorOutOfMemory;
        } else {
            hipError_t e = hipMalloc(&p, nb);
            if (e != hipSuccess) {
                p = nullptr;
                return e;
            }
        }
        bytes = nb;
        return hipSuccess;
    }
    hipError_t free_now() {
        hipError_t e = hipSuccess;
        if (p) {
            if (by.free)
                by.free(p, stream, by.ctx);
            else
                e = hipFree(p);
        }
        p = nullptr;
        bytes = 0;
        return e;
    }
    void release() { (void)free_now(); }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

bool seg_ok(const double *const *a, int64_t i) {
    for (int k = 0; k < 8; ++k)
        if (!std::isfinite(a[k][i])) return false;
    return a[7][i] > a[3][i];
}

// Bins of entries sorted by t_start (Sec. 4): width (t_last - t_first)/m,
// entry p in bin clamp(floor((t0[p] - t_first)/width), 0, m-1); only
// non-empty bins are returned, in time order.
void plan_bins(const double *t0, const double *t1, int64_t n, int32_t m, std::vector<tds_bin> *out,
               double *t_first, double *t_last, double *width) {
    out->clear();
    if (n == 0) {
        *t_first = *t_last = 0.0;
        *width = 1.0;
        return;
    }
    double tf = t0[0];
    double tl = t1[0];
    for (int64_t i = 1; i < n; ++i) tl = std::max(tl, t1[i]);
    double w = (tl - tf) / (double)m;
    *t_first = tf;
    *t_last = tl;
    *width = w;
    int64_t cur = -1;
    for (int64_t p = 0; p < n; ++p) {
        double u = std::floor((t0[p] - tf) / w);
        int64_t j = u <= 0.0 ? 0 : (u >= (double)(m - 1) ? (int64_t)(m - 1) : (int64_t)u);
        if (j != cur) {
            tds_bin b;
            b.start = t0[p];
            b.end = t1[p];
            b.first = p;
            b.last = p;
            b.bin = j;
            out->push_back(b);
            cur = j;
        } else {
            tds_bin &b = out->back();
            b.end = std::max(b.end, t1[p]);
            b.last = p;
        }
    }
}

// Max-tree of bin ends for the candidate-range search (bins_of_interval):
// P leaves (the smallest power of two >= nb), node k < P the larger of
// nodes 2k and 2k+1; tree[0] is unused.
int tree_leaves(int64_t nb) {
    int P = 1;
    while (P < nb) P <<= 1;
    return P;
}

std::vector<double> bin_end_tree(const std::vector<double> &ends) {
    const int P = tree_leaves((int64_t)ends.size());
    std::vector<double> t(2 * (size_t)P, -INFINITY);
    for (size_t j = 0; j < ends.size(); ++j) t[P + j] = ends[j];
    for (int k = P - 1; k >= 1; --k) t[k] = std::max(t[2 * k], t[2 * k + 1]);
    return t;
}

}  // namespace

struct tds_index {
    int device = 0;
    int64_t n = 0;
    int32_t m = 0;
    double t_first = 0, t_last = 0, width = 1;
    std::vector<tds_bin> bins;
    DBuf t0, t1, x0, y0, z0, vx, vy, vz, ecen, erad, orig, traj, t1s;
    double ox = 0, oy = 0, oz = 0;  // origin of the binary32 coordinates
    DBuf bstart, bpend, bfirst, blast, btree;
    DevIndex dev{};
    int64_t device_bytes = 0;
    int live_queries = 0;
};

struct tds_query {
    tds_index *ix = nullptr;
    int32_t cap_q = 0;        // query slots allocated
    int32_t cap_buckets = 0;  // bucket slots allocated
    DBuf rec, box, first, last, first_s, last_s, key, perm;
    DBuf qrank, bcount, bj2, bq_off, tiles, units, unit_off, cost_off, ctr;
    DBuf qstage, cand, hits, slab_n, slab_h, hit_off, wave_ovl, out_stage;
    DBuf tr_qtraj, tr_work, tr_temp, tr_out;  // trajectory merge
    DBuf gs_work, gs_jump;                     // GreedySetSplit tiling
    Slabs sl{};                    // slab view of the buffers above
    long long nslabs_alloc = 0;    // slabs the cand / hits buffers hold
    int32_t nwaves_alloc = 0;      // wave slabs slab_n / wave_ovl hold
    Counters *host_ctr = nullptr;  // pinned
    // The batch counters live in two slots used in turn: the last kernel of
    // a batch (k_emit, enqueued at fetch) clears the other slot and the
    // bucket counters, so the next batch starts without a clearing kernel.
    // clear_needed: they were not cleared (new buffers, a batch without
    // segments, an error).
    int ctr_slot = 0;
    bool clear_needed = true;
    NextClear next{};
    hipStream_t stream = nullptr;
    DevBatch b{};
    tds_query_opts opts{};
    int block = 256, grid = 0;
    bool pending = false, fetched = false;
    bool emitted = false;     // k_emit is enqueued after the last search run
    int64_t n_sorted = 0;     // query segments placed in tiles (last fetched batch)
    bool fetch_timed = false; // ev[4], ev[5] bracket the last fetch's translation
    bool traj_valid = false;  // tr_out holds the merged records of this batch
    long long traj_total = 0;
    tds_stats stats{};
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // recorded after the handle's own work for the host's waits, so that a
    // wait does not also cover what other callers enqueue later on the same
    // stream
    hipEvent_t ev_wait = nullptr;
};

// Device scratch of tds_search_noalloc: every per-batch buffer of that entry
// point (query records, ranges, buckets, tiles, counters, result slabs) is
// carved from this array, so the call allocates nothing. Each device holds
// its own copy for the life of the process; its device address is taken once
// per device with hipGetSymbolAddress (host code must not use the array's
// name as an address).
static __device__ __align__(256) unsigned char scratch[TDS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's scratch (looked up on first use).
int scratch_ptr(void **out, const char *who) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(TDS_EDEVICE, "%s: hipGetDevice: %s", who, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(TDS_EDEVICE, "%s: device %d out of range", who, dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(TDS_EDEVICE, "%s: hipGetSymbolAddress(scratch): %s", who, hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return TDS_OK;
}

// Regions laid out one after another from a base address, each aligned to
// 256 bytes; with a null base it only adds up the size.
struct Carver {
    char *base;
    size_t used = 0;
    template <class T>
    T *take(size_t bytes) {
        used = (used + 255) & ~(size_t)255;
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += bytes;
        return p;
    }
};

}  // namespace

namespace tds {
int set_error(int code, const char *msg) { return fail(code, "%s", msg); }
}  // namespace tds

extern "C" {

const char *tds_last_error(void) { return g_err.c_str(); }

int tds_set_allocator(tds_alloc_fn alloc, tds_free_fn free_fn, void *ctx) {
    if ((alloc == nullptr) != (free_fn == nullptr))
        return fail(TDS_EINVAL, "tds_set_allocator: give both functions or neither");
    g_alloc.alloc = alloc;
    g_alloc.free = free_fn;
    g_alloc.ctx = alloc ? ctx : nullptr;
    return TDS_OK;
}
int tds_abi_version(void) { return TDS_ABI_VERSION; }

int tds_plan_bins(const double *t0_sorted, const double *t1_sorted, int64_t n, int32_t num_bins,
                  tds_bin *out, int64_t cap, int64_t *n_out) {
    if (!n_out || n < 0 || num_bins < 1 || (n > 0 && (!t0_sorted || !t1_sorted)) ||
        (cap > 0 && !out))
        return fail(TDS_EINVAL, "tds_plan_bins: invalid argument");
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(t0_sorted[i]) || !std::isfinite(t1_sorted[i]) ||
            !(t1_sorted[i] > t0_sorted[i]))
            return fail(TDS_EINVAL, "tds_plan_bins: segment %lld has an invalid span", (long long)i);
        if (i > 0 && t0_sorted[i] < t0_sorted[i - 1])
            return fail(TDS_EINVAL, "tds_plan_bins: t_start not sorted at %lld", (long long)i);
    }
    std::vector<tds_bin> bins;
    double tf, tl, w;
    plan_bins(t0_sorted, t1_sorted, n, num_bins, &bins, &tf, &tl, &w);
    *n_out = (int64_t)bins.size();
    for (int64_t k = 0; k < (int64_t)bins.size() && k < cap; ++k) out[k] = bins[k];
    return TDS_OK;
}

int tds_plan_ranges(const tds_bin *bins, int64_t nb, const double *t0, const double *t1,
                    int64_t nq, int64_t *first, int64_t *last) {
    if (nb < 0 || nq < 0 || (nb > 0 && !bins) || (nq > 0 && (!t0 || !t1 || !first || !last)))
        return fail(TDS_EINVAL, "tds_plan_ranges: invalid argument");
    if (nb >= (int64_t)INT32_MAX / 2) return fail(TDS_EINVAL, "tds_plan_ranges: too many bins");
    std::vector<double> start(nb), pend(nb), end(nb);
    for (int64_t k = 0; k < nb; ++k) {
        start[k] = bins[k].start;
        end[k] = bins[k].end;
        pend[k] = k ? std::max(pend[k - 1], bins[k].end) : bins[k].end;
    }
    const std::vector<double> tree = bin_end_tree(end);
    const int P = tree_leaves(nb);
    for (int64_t i = 0; i < nq; ++i) {
        int j1 = 0, j2 = -1;
        if (nb > 0 && bins_of_interval(start.data(), pend.data(), tree.data(), P, (int)nb, t0[i], t1[i],
                                       &j1, &j2)) {
            first[i] = bins[j1].first;
            last[i] = bins[j2].last;
        } else {
            first[i] = 0;
            last[i] = -1;
        }
    }
    return TDS_OK;
}

int tds_build_index(const tds_segments *db, const tds_index_opts *opts, void *stream,
                    tds_index **out) {
    CallStream call_stream_scope(stream);
    if (!db || !opts || !out) return fail(TDS_EINVAL, "tds_build_index: null argument");
    *out = nullptr;
    if (db->n < 0 || db->n >= (int64_t)INT32_MAX)
        return fail(TDS_EINVAL, "tds_build_index: n = %lld out of range", (long long)db->n);
    if (opts->num_bins < 1 || opts->num_bins > (1 << 24))
        return fail(TDS_EINVAL, "tds_build_index: num_bins must be in 1..2^24");
    if (db->mem != TDS_MEM_HOST && db->mem != TDS_MEM_DEVICE)
        return fail(TDS_EINVAL, "tds_build_index: bad mem");
    const int64_t n = db->n;
    const double *src[8] = {db->x0, db->y0, db->z0, db->t0, db->x1, db->y1, db->z1, db->t1};
    if (n > 0)
        for (int k = 0; k < 8; ++k)
            if (!src[k]) return fail(TDS_EINVAL, "tds_build_index: null coordinate array");
    hipStream_t st = (hipStream_t)stream;

    // Host copies (the sort and the bin table are built on the host once).
    std::vector<double> host[8];
    const double *h[8];
    for (int k = 0; k < 8; ++k) {
        if (db->mem == TDS_MEM_DEVICE && n > 0) {
            host[k].resize(n);
            HIP_TRY(hipMemcpy(host[k].data(), src[k], n * sizeof(double), hipMemcpyDeviceToHost));
            h[k] = host[k].data();
        } else {
            h[k] = src[k];
        }
    }
    for (int64_t i = 0; i < n; ++i)
        if (!seg_ok(h, i))
            return fail(TDS_EINVAL, "tds_build_index: segment %lld is invalid", (long long)i);

    // Stable order by t_start; ties keep the input order.
    std::vector<int32_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(),
                     [&](int32_t a, int32_t b) { return h[3][a] < h[3][b]; });
    std::vector<double> t0s(n), t1p(n), t1s(n);
    for (int64_t p = 0; p < n; ++p) {
        int32_t i = perm[p];
        t0s[p] = h[3][i];
        t1p[p] = h[7][i];
    }
    t1s = t1p;
    std::sort(t1s.begin(), t1s.end());

    tds_index *ix = new tds_index();
    ix->n = n;
    ix->m = opts->num_bins;
    (void)hipGetDevice(&ix->device);
    plan_bins(t0s.data(), t1p.data(), n, opts->num_bins, &ix->bins, &ix->t_first, &ix->t_last,
              &ix->width);
    const int64_t nb = (int64_t)ix->bins.size();
    // Origin of the binary32 coordinates: the per-axis median of the end
    // points (robust to a few far outliers), so that |c| stays near the data's
    // own extent and the binary32 test's rounding bound with it.
    if (n > 0) {
        std::vector<double> v((size_t)2 * n);
        double *org[3] = {&ix->ox, &ix->oy, &ix->oz};
        for (int k = 0; k < 3; ++k) {
            for (int64_t i = 0; i < n; ++i) {
                v[(size_t)2 * i] = h[k][i];
                v[(size_t)2 * i + 1] = h[k + 4][i];
            }
            std::nth_element(v.begin(), v.begin() + n, v.end());
            *org[k] = v[(size_t)n];
        }
    }

    auto cleanup = [&](int code) {
        tds_index_destroy(ix);
        return code;
    };
#define IX_TRY(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return cleanup(fail(e_ == hipErrorOutOfMemory ? TDS_ENOMEM : TDS_EDEVICE, "%s: %s", \
                                #expr, hipGetErrorString(e_)));                            \
    } while (0)

    const size_t n1 = (size_t)std::max<int64_t>(n, 1);
    for (DBuf *b : {&ix->t0, &ix->t1, &ix->x0, &ix->y0, &ix->z0, &ix->vx, &ix->vy, &ix->vz,
                    &ix->traj, &ix->t1s})
        IX_TRY(b->ensure(n1 * 8));
    IX_TRY(ix->ecen.ensure(n1 * 16));
    IX_TRY(ix->erad.ensure(n1 * 4));
    IX_TRY(ix->orig.ensure(n1 * 4));
    const size_t nb1 = (size_t)std::max<int64_t>(nb, 1);
    IX_TRY(ix->bstart.ensure(nb1 * 8));
    IX_TRY(ix->bpend.ensure(nb1 * 8));
    IX_TRY(ix->bfirst.ensure(nb1 * 4));
    IX_TRY(ix->blast.ensure(nb1 * 4));

    std::vector<double> bs(nb), bp(nb), be(nb);
    std::vector<int32_t> bf(nb), bl(nb);
    for (int64_t k = 0; k < nb; ++k) {
        bs[k] = ix->bins[k].start;
        be[k] = ix->bins[k].end;
        bp[k] = k ? std::max(bp[k - 1], ix->bins[k].end) : ix->bins[k].end;
        bf[k] = (int32_t)ix->bins[k].first;
        bl[k] = (int32_t)ix->bins[k].last;
    }
    const std::vector<double> bt = bin_end_tree(be);
    IX_TRY(ix->btree.ensure(bt.size() * 8));

    if (n > 0) {
        // Raw arrays to the device (caller order), then gather + derive.
        DBuf raw, dperm, dtraj;
        IX_TRY(raw.ensure((size_t)n * 8 * 8));
        IX_TRY(dperm.ensure((size_t)n * 4));
        const double *rawp[8];
        for (int k = 0; k < 8; ++k) {
            double *dst = raw.as<double>() + (size_t)k * n;
            IX_TRY(hipMemcpyAsync(dst, src[k], n * sizeof(double),
                                  db->mem == TDS_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                            : hipMemcpyHostToDevice,
                                  st));
            rawp[k] = dst;
        }
        IX_TRY(hipMemcpyAsync(dperm.p, perm.data(), n * 4, hipMemcpyHostToDevice, st));
        const int64_t *traj_dev = nullptr;
        if (db->traj_id) {
            IX_TRY(dtraj.ensure((size_t)n * 8));
            IX_TRY(hipMemcpyAsync(dtraj.p, db->traj_id, n * 8,
                                  db->mem == TDS_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                            : hipMemcpyHostToDevice,
                                  st));
            traj_dev = dtraj.as<int64_t>();
        }
        IX_TRY(launch_ingest(rawp, n, dperm.as<int32_t>(), traj_dev, ix->t0.as<double>(),
                             ix->t1.as<double>(), ix->x0.as<double>(), ix->y0.as<double>(),
                             ix->z0.as<double>(), ix->vx.as<double>(), ix->vy.as<double>(),
                             ix->vz.as<double>(), ix->ecen.as<float4>(), ix->erad.as<float>(),
                             ix->ox, ix->oy, ix->oz, ix->orig.as<int32_t>(),
                             ix->traj.as<int64_t>(), st));
        IX_TRY(hipMemcpyAsync(ix->t1s.p, t1s.data(), n * 8, hipMemcpyHostToDevice, st));
        IX_TRY(hipMemcpyAsync(ix->bstart.p, bs.data(), nb * 8, hipMemcpyHostToDevice, st));
        IX_TRY(hipMemcpyAsync(ix->bpend.p, bp.data(), nb * 8, hipMemcpyHostToDevice, st));
        IX_TRY(hipMemcpyAsync(ix->bfirst.p, bf.data(), nb * 4, hipMemcpyHostToDevice, st));
        IX_TRY(hipMemcpyAsync(ix->blast.p, bl.data(), nb * 4, hipMemcpyHostToDevice, st));
        IX_TRY(hipMemcpyAsync(ix->btree.p, bt.data(), bt.size() * 8, hipMemcpyHostToDevice, st));
        IX_TRY(hipStreamSynchronize(st));
        raw.release();
        dperm.release();
        dtraj.release();
    }
#undef IX_TRY

    DevIndex &d = ix->dev;
    d.n = n;
    d.nb = (int32_t)nb;
    d.m = ix->m;
    d.t_first = ix->t_first;
    d.width = ix->width > 0.0 ? ix->width : 1.0;
    d.t0 = ix->t0.as<double>();
    d.t1 = ix->t1.as<double>();
    d.x0 = ix->x0.as<double>();
    d.y0 = ix->y0.as<double>();
    d.z0 = ix->z0.as<double>();
    d.vx = ix->vx.as<double>();
    d.vy = ix->vy.as<double>();
    d.vz = ix->vz.as<double>();
    d.ecen = ix->ecen.as<float4>();
    d.erad = ix->erad.as<float>();
    d.ox = ix->ox;
    d.oy = ix->oy;
    d.oz = ix->oz;
    d.orig = ix->orig.as<int32_t>();
    d.traj = ix->traj.as<int64_t>();
    d.t1s = ix->t1s.as<double>();
    d.bstart = ix->bstart.as<double>();
    d.bpend = ix->bpend.as<double>();
    d.bfirst = ix->bfirst.as<int32_t>();
    d.blast = ix->blast.as<int32_t>();
    d.btree = ix->btree.as<double>();
    d.bleaf = tree_leaves(nb);
    d.pad_b = 0;
    ix->device_bytes = (int64_t)(n * (8 * 8 + 16 + 4 + 4 + 8 + 8) + nb * 24 + (int64_t)bt.size() * 8);
    *out = ix;
    return TDS_OK;
}

int tds_index_info_get(const tds_index *ix, tds_index_info *out) {
    if (!ix || !out) return fail(TDS_EINVAL, "tds_index_info_get: null argument");
    out->n = ix->n;
    out->num_bins = ix->m;
    out->nonempty_bins = (int32_t)ix->bins.size();
    out->t_first = ix->t_first;
    out->t_last = ix->t_last;
    out->bin_width = ix->n > 0 ? ix->width : 0.0;
    out->device_bytes = ix->device_bytes;
    return TDS_OK;
}

int tds_index_bins(const tds_index *ix, tds_bin *out, int64_t cap, int64_t *n_out) {
    if (!ix || !n_out || (cap > 0 && !out)) return fail(TDS_EINVAL, "tds_index_bins: null argument");
    *n_out = (int64_t)ix->bins.size();
    for (int64_t k = 0; k < *n_out && k < cap; ++k) out[k] = ix->bins[k];
    return TDS_OK;
}

int tds_index_times(const tds_index *ix, double *t_start_sorted, double *t_end_sorted, int64_t n) {
    if (!ix || (n > 0 && (!t_start_sorted || !t_end_sorted)))
        return fail(TDS_EINVAL, "tds_index_times: null argument");
    if (n != ix->n) return fail(TDS_EINVAL, "tds_index_times: n must equal the entry count");
    if (n == 0) return TDS_OK;
    HIP_TRY(hipMemcpy(t_start_sorted, ix->t0.p, (size_t)n * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(t_end_sorted, ix->t1s.p, (size_t)n * 8, hipMemcpyDeviceToHost));
    return TDS_OK;
}

void tds_index_destroy(tds_index *ix) {
    if (!ix) return;
    for (DBuf *b : {&ix->t0, &ix->t1, &ix->x0, &ix->y0, &ix->z0, &ix->vx, &ix->vy, &ix->vz,
                    &ix->ecen, &ix->erad, &ix->orig, &ix->traj, &ix->t1s, &ix->bstart, &ix->bpend,
                    &ix->bfirst, &ix->blast, &ix->btree})
        b->release();
    delete ix;
}

int tds_query_create(tds_index *ix, tds_query **out) {
    if (!ix || !out) return fail(TDS_EINVAL, "tds_query_create: null argument");
    tds_query *q = new tds_query();
    q->ix = ix;
    // pinned: the final counters, then the trajectory merge's record count
    hipError_t e = hipHostMalloc((void **)&q->host_ctr, sizeof(Counters) + 64, hipHostMallocDefault);
    if (e != hipSuccess) {
        delete q;
        return fail(TDS_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    std::memset(q->host_ctr, 0, sizeof(Counters) + 64);
    for (auto &ev : q->ev) {
        e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            tds_query_destroy(q);
            return fail(TDS_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
        }
    }
    e = hipEventCreateWithFlags(&q->ev_wait, hipEventDisableTiming);
    if (e != hipSuccess) {
        tds_query_destroy(q);
        return fail(TDS_EDEVICE, "hipEventCreateWithFlags: %s", hipGetErrorString(e));
    }
    ix->live_queries++;
    *out = q;
    return TDS_OK;
}

void tds_query_destroy(tds_query *q) {
    if (!q) return;
    if (q->pending) (void)hipStreamSynchronize(q->stream);
    for (DBuf *b : {&q->rec, &q->box, &q->first, &q->last, &q->first_s,
                    &q->last_s, &q->key, &q->perm, &q->qrank, &q->bcount, &q->bj2, &q->bq_off,
                    &q->tiles, &q->units, &q->unit_off, &q->cost_off, &q->ctr, &q->qstage, &q->cand,
                    &q->hits, &q->slab_n, &q->slab_h, &q->hit_off, &q->wave_ovl, &q->out_stage,
                    &q->tr_qtraj, &q->tr_work, &q->tr_temp, &q->tr_out, &q->gs_work,
                    &q->gs_jump})
        b->release();
    if (q->host_ctr) (void)hipHostFree(q->host_ctr);
    for (auto &ev : q->ev)
        if (ev) (void)hipEventDestroy(ev);
    if (q->ev_wait) (void)hipEventDestroy(q->ev_wait);
    if (q->ix) q->ix->live_queries--;
    delete q;
}

// Query-side buffers for nq segments and nbuckets buckets (grown, never shrunk).
static int ensure_capacity(tds_query *q, int32_t nq, int32_t nbuckets) {
    if (nq > q->cap_q || !q->ctr.p) {
        int32_t c = std::max<int32_t>(nq, std::max<int32_t>(1024, q->cap_q + q->cap_q / 2));
        size_t n = (size_t)c, n1 = n + 1;
        HIP_TRY(q->rec.ensure(n * sizeof(QRec64)));
        HIP_TRY(q->box.ensure(n * sizeof(QCube32)));
        for (DBuf *b : {&q->first, &q->last, &q->first_s, &q->last_s, &q->key, &q->qrank})
            HIP_TRY(b->ensure(n * 4));
        HIP_TRY(q->perm.ensure((n + 2) * 4));  // read-ahead slots
        HIP_TRY(q->tiles.ensure(n1 * sizeof(Tile)));
        HIP_TRY(q->units.ensure(n1 * 8));
        HIP_TRY(q->unit_off.ensure(n1 * 8));
        HIP_TRY(q->cost_off.ensure(n1 * 8));
        HIP_TRY(q->ctr.ensure(2 * sizeof(Counters)));
        q->cap_q = c;
        q->clear_needed = true;
    }
    if (nbuckets > q->cap_buckets) {
        size_t n = (size_t)nbuckets;
        for (DBuf *b : {&q->bcount, &q->bq_off}) HIP_TRY(b->ensure(n * kBucketSub * 4));
        HIP_TRY(q->bj2.ensure(n * 4));
        q->cap_buckets = nbuckets;
        q->clear_needed = true;
    }
    return TDS_OK;
}

// Work arrays of the GreedySetSplit tiling of nq query segments. The batch
// chain is marked with `levels` doubling passes, enough for 2^levels - 1
// batches: with Min every batch but the last holds at least `bound`
// segments, with Max two neighbouring batches hold more than `bound`.
struct GreedySize {
    int levels;
    size_t work, jump;  // bytes
};

static GreedySize greedy_size(int32_t nq, int32_t bound, bool is_max, bool chain) {
    const long long most = is_max ? 2LL * nq / ((long long)bound + 1) + 2 : (long long)nq / bound + 2;
    int levels = 1;
    while (chain && (1LL << levels) <= most) ++levels;
    const size_t n = (size_t)nq, n1 = n + 1;
    // 8-byte arrays first: kin, tkey, tev, gmax; then the 4-byte ones, then the flags
    const size_t n16 = (n + 15) & ~(size_t)15;
    GreedySize z;
    z.levels = levels;
    z.work = n * 8 * 4 + n * 4 * 2 + n1 * 4 * 3 + 2 * 4 + n16 + 64;
    z.jump = chain ? (size_t)levels * n1 * 4 : 0;
    return z;
}

// Lays the greedy work arrays out in `work` (z.work bytes) and `jump`.
static void carve_greedy(char *w, int32_t *jump, int32_t nq, const GreedySize &z, GreedyBufs *g) {
    const size_t n = (size_t)nq, n1 = n + 1;
    const size_t n16 = (n + 15) & ~(size_t)15;
    auto take = [&](size_t b) { char *p = w; w += b; return p; };
    g->kin = (unsigned long long *)take(n * 8);
    g->tkey = (unsigned long long *)take(n * 8);
    g->tev = (long long *)take(n * 8);
    g->gmax = (double *)take(n * 8);
    g->vout = (int32_t *)take(n * 4);
    g->tidx = (int32_t *)take(n * 4);
    g->gpos = (int32_t *)take(n1 * 4);
    g->mark = (int32_t *)take(n1 * 4);
    g->gb = (int32_t *)take(n1 * 4);
    g->cnt = (int32_t *)take(2 * 4);
    w = (char *)(((uintptr_t)w + 15) & ~(uintptr_t)15);
    g->flag = (uint8_t *)take(n16);
    g->jump = jump;
    g->stride = (int32_t)n1;
    g->levels = z.levels;
}

static int greedy_buffers(tds_query *q, int32_t nq, int32_t bound, bool is_max, bool chain,
                          GreedyBufs *g) {
    const GreedySize z = greedy_size(nq, bound, is_max, chain);
    HIP_TRY(q->gs_work.ensure(z.work));
    if (chain) HIP_TRY(q->gs_jump.ensure(z.jump));
    carve_greedy(q->gs_work.as<char>(), chain ? q->gs_jump.as<int32_t>() : nullptr, nq, z, g);
    return TDS_OK;
}

// Slab buffers for a pair launch of `nwaves` waves with `spill` spill slabs
// after the wave slabs (grown, never shrunk).
static int ensure_slabs(tds_query *q, int32_t nwaves, unsigned long long spill) {
    const long long want = (long long)nwaves + 1 + (long long)spill;
    if (want > q->nslabs_alloc) {
        const long long n = std::max<long long>(want, q->nslabs_alloc + q->nslabs_alloc / 2);
        HIP_TRY(q->cand.ensure((size_t)n * kSlab * sizeof(Cand)));
        HIP_TRY(q->hits.ensure((size_t)n * kSlab * sizeof(Hit24)));
        HIP_TRY(q->slab_n.ensure((size_t)n * sizeof(int32_t)));
        HIP_TRY(q->slab_h.ensure((size_t)n * sizeof(int32_t)));
        HIP_TRY(q->hit_off.ensure((size_t)(n + 1) * sizeof(long long)));
        q->nslabs_alloc = n;
    }
    if (nwaves > q->nwaves_alloc) {
        HIP_TRY(q->wave_ovl.ensure((size_t)nwaves * sizeof(unsigned long long)));
        q->nwaves_alloc = nwaves;
    }
    Slabs &sl = q->sl;
    sl.cand = q->cand.as<Cand>();
    sl.hits = q->hits.as<Hit24>();
    sl.slab_n = q->slab_n.as<int32_t>();
    sl.slab_h = q->slab_h.as<int32_t>();
    sl.hit_off = q->hit_off.as<long long>();
    sl.wave_ovl = q->wave_ovl.as<unsigned long long>();
    sl.nwaves = nwaves;
    sl.pad = 0;
    sl.nslabs = q->nslabs_alloc;
    return TDS_OK;
}

// Spill slabs available after the wave slabs.
static unsigned long long spill_capacity(const Slabs &sl) {
    return (unsigned long long)(sl.nslabs - sl.nwaves);
}

// Pair kernel (selects pairs), then refine (turns them into hits), with HIP
// events around the pair kernel and the refine when timing is on. The
// batch's last kernel (k_emit: offsets, records, final counters) follows at
// fetch; a batch without query segments has none, so its counters are
// copied here.
static int launch_search(tds_query *q) {
    const bool timing = (q->opts.flags & TDS_QF_TIMING) != 0;
    const int kovl = (q->opts.flags & TDS_QF_KERNEL_OVERLAP) ? 1 : 0;
    // timing: events attached to the pair kernel's dispatch (start, end) and
    // to the end of the refine
    const bool tpair = timing || (q->opts.flags & TDS_QF_TIMING_PAIR) != 0;
    HIP_TRY(launch_pair(q->b, q->ix->dev, q->opts.mode, q->block, q->opts.grid, kovl, q->sl,
                        q->stream, tpair ? q->ev[1] : nullptr, tpair ? q->ev[2] : nullptr));
    HIP_TRY(launch_refine(q->b, q->ix->dev, q->sl, q->stream, timing ? q->ev[3] : nullptr));
    if (q->b.nq == 0)
        HIP_TRY(hipMemcpyAsync(q->host_ctr, q->b.ctr, sizeof(Counters), hipMemcpyDeviceToHost,
                               q->stream));
    q->emitted = false;
    return TDS_OK;
}

// The batch's last kernel with `n` records to `out` (null: offsets and
// counters only); it writes the final counters to host_ctr and clears the
// next batch's counters. The fetch's timing events bracket it when it writes
// records.
static int enqueue_emit(tds_query *q, void *out, int64_t n) {
    if (q->b.nq > 0) {
        const bool timing = (q->opts.flags & TDS_QF_TIMING) != 0 && out;
        const int kovl = (q->opts.flags & TDS_QF_KERNEL_OVERLAP) ? 1 : 0;
        HIP_TRY(launch_emit(q->sl, q->b.ctr, n, q->ix->dev, out, kovl, q->host_ctr, q->next,
                            q->stream, timing ? q->ev[4] : nullptr, timing ? q->ev[5] : nullptr));
    }
    q->emitted = true;
    return TDS_OK;
}

// Checks a batch's arguments and fills in the option defaults (shared by
// tds_query_batch and tds_search_noalloc; `who` names the caller).
static int check_batch(const tds_segments *qs, const double *d, const tds_query_opts *opts,
                       tds_query_opts *o_out, const char *who) {
    if (!qs || !opts || (qs->n > 0 && !d)) return fail(TDS_EINVAL, "%s: null argument", who);
    if (qs->n < 0 || qs->n >= (int64_t)INT32_MAX / 2)
        return fail(TDS_EINVAL, "%s: n = %lld out of range", who, (long long)qs->n);
    if (qs->mem != TDS_MEM_HOST && qs->mem != TDS_MEM_DEVICE) return fail(TDS_EINVAL, "%s: bad mem", who);
    tds_query_opts o = *opts;
    if (o.mode != TDS_MODE_FP64 && o.mode != TDS_MODE_FP32_REFINE)
        return fail(TDS_EINVAL, "%s: unknown mode %d", who, o.mode);
    if (o.tiling != TDS_TILE_PERIODIC && o.tiling != TDS_TILE_RANGE &&
        o.tiling != TDS_TILE_GREEDY_MIN && o.tiling != TDS_TILE_GREEDY_MAX)
        return fail(TDS_EINVAL, "%s: unknown tiling %d", who, o.tiling);
    if (o.batch_size == 0) o.batch_size = 128;
    if (o.batch_size < 1 || o.batch_size > 65536)
        return fail(TDS_EINVAL, "%s: batch_size %d out of 1..65536", who, o.batch_size);
    if (o.reserved0 != 0) return fail(TDS_EINVAL, "%s: reserved0 must be 0", who);
    if (o.block_size == 0) o.block_size = 256;
    if (o.block_size != 64 && o.block_size != 128 && o.block_size != 256 && o.block_size != 512 &&
        o.block_size != 1024)
        return fail(TDS_EINVAL, "%s: block_size %d not supported", who, o.block_size);
    if (o.max_retries < 0) o.max_retries = 4;
    if (o.capacity < 0 || o.grid < 0) return fail(TDS_EINVAL, "%s: negative option", who);
    const double *src[8] = {qs->x0, qs->y0, qs->z0, qs->t0, qs->x1, qs->y1, qs->z1, qs->t1};
    const int32_t nq = (int32_t)qs->n;
    if (nq > 0)
        for (int k = 0; k < 8; ++k)
            if (!src[k]) return fail(TDS_EINVAL, "%s: null coordinate array", who);
    // The segments' values are checked by the preparation kernel, in host and
    // device memory alike (a check here would read every input on the CPU:
    // about 1 ms for 200,000 segments, most of a host-memory batch); the
    // fetch reports them.
    *o_out = o;
    return TDS_OK;
}

// The scalar fields of a batch (its buffers are set by the caller).
static void batch_scalars(DevBatch &b, const tds_query_opts &o, int32_t nq, int nbuckets) {
    b.nq = nq;
    b.s = o.batch_size;
    b.chunk = chunk_for(o.mode, o.block_size);
    b.tiling = o.tiling;
    b.nbuckets = nbuckets;
    b.ntiles_cap = o.tiling == TDS_TILE_PERIODIC ? (nq + o.batch_size - 1) / o.batch_size : nq;
    b.count_overlap = (o.flags & TDS_QF_COUNT_OVERLAP) ? 1 : 0;
    b.pass_cost = o.mode == TDS_MODE_FP64 ? TDS_PASS_COST64 : TDS_PASS_COST32;
    b.stage_cost = o.mode == TDS_MODE_FP64 ? TDS_STAGE_COST64 : TDS_STAGE_COST32;
    b.pad = 0;
}

// Query preparation and tiling of a batch whose buffers are set (shared by
// tds_query_batch and tds_search_noalloc).
static int enqueue_tiles(DevBatch &b, const GreedyBufs &gb, const tds_index *ix,
                         const double *const *qin, const double *din, const tds_query_opts &o,
                         hipStream_t st, hipEvent_t ev_start, bool zero = true) {
    const bool greedy = o.tiling == TDS_TILE_GREEDY_MIN || o.tiling == TDS_TILE_GREEDY_MAX;
    const bool sorted = greedy || o.tiling == TDS_TILE_PERIODIC;
    HIP_TRY(launch_prepare(qin, din, b, ix->dev, st, ev_start, zero));
    if (sorted && b.nq > 0) HIP_TRY(launch_bucket_sort(b, st));
    if (o.tiling == TDS_TILE_PERIODIC && b.nq > 0) HIP_TRY(launch_periodic(b, ix->dev, st));
    if (greedy && b.nq > 0)
        HIP_TRY(launch_greedy(b, gb, ix->dev, o.batch_size, o.tiling == TDS_TILE_GREEDY_MAX, st));
    return TDS_OK;
}

int tds_query_batch(tds_query *q, const tds_segments *qs, const double *d,
                    const tds_query_opts *opts, void *stream) {
    CallStream call_stream_scope(stream);
    if (!q) return fail(TDS_EINVAL, "tds_query_batch: null argument");
    if (q->pending) return fail(TDS_ESTATE, "tds_query_batch: previous batch not fetched");
    tds_query_opts o;
    int rc = check_batch(qs, d, opts, &o, "tds_query_batch");
    if (rc) return rc;
    const double *src[8] = {qs->x0, qs->y0, qs->z0, qs->t0, qs->x1, qs->y1, qs->z1, qs->t1};
    const int32_t nq = (int32_t)qs->n;

    hipStream_t st = (hipStream_t)stream;
    const tds_index *ix = q->ix;
    const int nbuckets = nbuckets_for(o.tiling, ix->dev.nb, ix->dev.m);
    q->stream = st;
    q->opts = o;
    q->block = o.block_size;
    rc = ensure_capacity(q, std::max<int32_t>(nq, 1), nbuckets);
    if (rc) return rc;
    const int kovl = (o.flags & TDS_QF_KERNEL_OVERLAP) ? 1 : 0;
    const int grid = pair_grid(o.mode, o.block_size, o.grid, kovl);
    if (grid < 1 || (long long)grid * (o.block_size / 64) > INT32_MAX / kSlab)
        return fail(TDS_EINVAL, "tds_query_batch: grid %d not supported", grid);
    q->grid = grid;
    // capacity: selections beyond the per-wave slabs to make room for, in
    // spill slabs of kSlab
    const unsigned long long sel = o.capacity > 0 ? (unsigned long long)o.capacity : (1ull << 20);
    rc = ensure_slabs(q, grid * (o.block_size / 64), (sel + kSlab - 1) / kSlab);
    if (rc) return rc;

    const double *qin[8];
    const double *din = d;
    if (qs->mem == TDS_MEM_HOST && nq > 0) {
        HIP_TRY(q->qstage.ensure((size_t)nq * 9 * 8));
        for (int k = 0; k < 8; ++k) {
            double *dst = q->qstage.as<double>() + (size_t)k * nq;
            HIP_TRY(hipMemcpyAsync(dst, src[k], (size_t)nq * 8, hipMemcpyHostToDevice, st));
            qin[k] = dst;
        }
        double *dd = q->qstage.as<double>() + (size_t)8 * nq;
        HIP_TRY(hipMemcpyAsync(dd, d, (size_t)nq * 8, hipMemcpyHostToDevice, st));
        din = dd;
    } else {
        for (int k = 0; k < 8; ++k) qin[k] = src[k];
    }

    DevBatch &b = q->b;
    batch_scalars(b, o, nq, nbuckets);
    b.rec = q->rec.as<QRec64>();
    b.box = q->box.as<QCube32>();
    b.first = q->first.as<int32_t>();
    b.last = q->last.as<int32_t>();
    b.first_s = q->first_s.as<int32_t>();
    b.last_s = q->last_s.as<int32_t>();
    b.key = q->key.as<int32_t>();
    b.perm = q->perm.as<int32_t>();
    b.bcount = q->bcount.as<int32_t>();
    b.bj2 = q->bj2.as<int32_t>();
    b.qrank = q->qrank.as<int32_t>();
    b.bq_off = q->bq_off.as<int32_t>();
    b.tiles = q->tiles.as<Tile>();
    b.units = q->units.as<long long>();
    b.unit_off = q->unit_off.as<long long>();
    b.cost_off = q->cost_off.as<long long>();
    b.ctr = q->ctr.as<Counters>() + q->ctr_slot;
    // the last kernel of this batch clears the next batch's counters
    q->next = NextClear{q->ctr.as<Counters>() + (q->ctr_slot ^ 1), q->bcount.as<int32_t>(),
                        q->bj2.as<int32_t>(), q->cap_buckets, 0};

    // Periodic and the greedy tilings walk the segments in exact
    // (t_start, caller index) order, sorted within each t_start bin
    const bool greedy = o.tiling == TDS_TILE_GREEDY_MIN || o.tiling == TDS_TILE_GREEDY_MAX;
    const bool sorted = greedy || o.tiling == TDS_TILE_PERIODIC;
    GreedyBufs gb{};
    b.skey = b.tkey = nullptr;
    b.sidx = b.tidx = nullptr;
    if (sorted && nq > 0) {
        rc = greedy_buffers(q, nq, o.batch_size, o.tiling == TDS_TILE_GREEDY_MAX, greedy, &gb);
        if (rc) return rc;
        b.skey = gb.kin;
        b.sidx = gb.vout;
        b.tkey = gb.tkey;
        b.tidx = gb.tidx;
    }

    const bool timing = (o.flags & TDS_QF_TIMING) != 0;
    const bool zero = q->clear_needed;
    q->clear_needed = true;  // until the whole batch is enqueued
    rc = enqueue_tiles(b, gb, ix, qin, din, o, st, timing ? q->ev[0] : nullptr, zero);
    if (rc) return rc;
    rc = launch_search(q);
    if (rc) return rc;
    // a batch without segments launches no k_emit, which would clear
    q->clear_needed = nq == 0;
    q->ctr_slot ^= 1;
    q->pending = true;
    q->fetched = false;
    q->traj_valid = false;
    std::memset(&q->stats, 0, sizeof q->stats);
    q->stats.n_query = nq;
    return TDS_OK;
}

int tds_query_reserve(tds_query *q, int64_t n_query, int64_t capacity, const tds_query_opts *opts) {
    if (!q || !opts || n_query < 0 || capacity < 0)
        return fail(TDS_EINVAL, "tds_query_reserve: invalid argument");
    if (q->pending) return fail(TDS_ESTATE, "tds_query_reserve: a batch is pending");
    if (n_query >= (int64_t)INT32_MAX / 2)
        return fail(TDS_EINVAL, "tds_query_reserve: n_query = %lld out of range", (long long)n_query);
    tds_segments none{};
    none.mem = TDS_MEM_DEVICE;
    tds_query_opts o;
    int rc = check_batch(&none, nullptr, opts, &o, "tds_query_reserve");
    if (rc) return rc;
    const int32_t nq = std::max<int32_t>((int32_t)n_query, 1);
    const tds_index *ix = q->ix;
    rc = ensure_capacity(q, nq, nbuckets_for(o.tiling, ix->dev.nb, ix->dev.m));
    if (rc) return rc;
    const int kovl = (o.flags & TDS_QF_KERNEL_OVERLAP) ? 1 : 0;
    const int grid = pair_grid(o.mode, o.block_size, o.grid, kovl);
    if (grid < 1 || (long long)grid * (o.block_size / 64) > INT32_MAX / kSlab)
        return fail(TDS_EINVAL, "tds_query_reserve: grid %d not supported", grid);
    const unsigned long long sel = capacity > 0 ? (unsigned long long)capacity : (1ull << 20);
    rc = ensure_slabs(q, grid * (o.block_size / 64), (sel + kSlab - 1) / kSlab);
    if (rc) return rc;
    const bool greedy = o.tiling == TDS_TILE_GREEDY_MIN || o.tiling == TDS_TILE_GREEDY_MAX;
    if (greedy || o.tiling == TDS_TILE_PERIODIC) {
        GreedyBufs gb{};
        rc = greedy_buffers(q, nq, o.batch_size, o.tiling == TDS_TILE_GREEDY_MAX, greedy, &gb);
        if (rc) return rc;
    }
    // host output is staged on the device: room for `capacity` records
    HIP_TRY(q->out_stage.ensure((size_t)sel * sizeof(tds_hit)));
    return TDS_OK;
}

int tds_query_device_bytes(const tds_query *q, int64_t *bytes) {
    if (!q || !bytes) return fail(TDS_EINVAL, "tds_query_device_bytes: null argument");
    size_t t = 0;
    for (const DBuf *b : {&q->rec, &q->box, &q->first, &q->last, &q->first_s, &q->last_s, &q->key,
                          &q->perm, &q->qrank, &q->bcount, &q->bj2, &q->bq_off, &q->tiles, &q->units,
                          &q->unit_off, &q->cost_off, &q->ctr, &q->qstage, &q->cand, &q->hits,
                          &q->slab_n, &q->slab_h, &q->hit_off, &q->wave_ovl, &q->out_stage,
                          &q->tr_qtraj, &q->tr_work, &q->tr_temp, &q->tr_out, &q->gs_work,
                          &q->gs_jump})
        t += b->bytes;
    *bytes = (int64_t)t;
    return TDS_OK;
}

// Wait for the pending batch, re-run it on overflow, and fill the stats
// (shared by the fetch calls). `who` names the caller in error messages.
// Waits for the work the handle has enqueued so far on its stream.
static hipError_t wait_own(tds_query *q) {
    const hipError_t e = hipEventRecord(q->ev_wait, q->stream);
    return e != hipSuccess ? e : hipEventSynchronize(q->ev_wait);
}

static int complete_batch(tds_query *q, const char *who) {
    hipStream_t st = q->stream;
    if (q->pending) {
        if (!q->emitted) {
            int rc = enqueue_emit(q, nullptr, 0);
            if (rc) return rc;
        }
        HIP_TRY(wait_own(q));
        Counters c = *q->host_ctr;
        if (c.err) {
            q->pending = false;
            q->clear_needed = true;
            return fail(TDS_EINVAL, "%s: the batch holds an invalid query "
                                    "segment (non-finite value, t_end <= t_start, or d < 0)", who);
        }
        // Overflow (Sec. 5: re-attempt with more memory): selections beyond
        // the slabs were counted, not stored; grow and run the search again.
        int retries = 0;
        while (c.spill > spill_capacity(q->sl)) {
            if (retries >= q->opts.max_retries) {
                q->pending = false;
                q->clear_needed = true;
                return fail(TDS_EOVERFLOW,
                            "%s: the selections needed %llu spill slabs of %d records "
                            "beyond the wave slabs; capacity %llu",
                            who, c.spill, kSlab, spill_capacity(q->sl));
            }
            ++retries;
            // the count is exact (a wave's slabs depend only on its own
            // selections), so this size suffices for the re-run
            q->clear_needed = true;  // until the re-run is enqueued
            int rc = ensure_slabs(q, q->sl.nwaves, c.spill);
            if (rc) return rc;
            HIP_TRY(launch_reset_counters(q->b.ctr, 1, st));
            rc = launch_search(q);
            if (rc) return rc;
            rc = enqueue_emit(q, nullptr, 0);
            if (rc) return rc;
            q->clear_needed = false;
            HIP_TRY(wait_own(q));
            c = *q->host_ctr;
        }
        tds_stats &s = q->stats;
        s.n_eval = (int64_t)c.n_eval;
        s.n_overlap = (q->opts.flags & TDS_QF_COUNT_OVERLAP) ? (int64_t)c.n_overlap_exact : -1;
        s.n_overlap_k = (q->opts.flags & TDS_QF_KERNEL_OVERLAP) ? (int64_t)c.overlap : -1;
        s.n_refine = (int64_t)c.cand;
        s.n_hit = (int64_t)c.hits;
        s.n_tiles = (int64_t)c.n_tiles;
        q->n_sorted = (int64_t)c.n_sorted;
        s.n_items = (int64_t)c.n_units;
        s.grid = q->grid;
        s.chunk = q->b.chunk;
        s.retries = retries;
        // timing: the event times are read by tds_query_stats, outside the batch's path
        q->fetch_timed = false;
        q->pending = false;
        q->fetched = true;
    }
    return TDS_OK;
}

int tds_fetch_results(tds_query *q, tds_hit *out, int64_t cap, int32_t out_mem, int64_t *n_total) {
    CallStream call_stream_scope(q ? (void *)q->stream : nullptr);
    if (!q || !n_total || cap < 0 || (cap > 0 && !out))
        return fail(TDS_EINVAL, "tds_fetch_results: invalid argument");
    if (out_mem != TDS_MEM_HOST && out_mem != TDS_MEM_DEVICE)
        return fail(TDS_EINVAL, "tds_fetch_results: bad out_mem");
    if (!q->pending && !q->fetched) return fail(TDS_ESTATE, "tds_fetch_results: no batch");
    hipStream_t st = q->stream;
    const bool timing = (q->opts.flags & TDS_QF_TIMING) != 0;
    // Host output in pinned memory (hipHostMalloc) is written by the kernel
    // directly; other host output is staged on the device and copied.
    void *direct = nullptr;
    if (out_mem == TDS_MEM_HOST && cap > 0) {
        hipPointerAttribute_t a{};
        if (hipPointerGetAttributes(&a, out) == hipSuccess && a.type == hipMemoryTypeHost)
            direct = a.devicePointer ? a.devicePointer : (void *)out;
        (void)hipGetLastError();  // pageable memory: the query fails, nothing is pending
    }
    void *dst = out_mem == TDS_MEM_DEVICE ? (void *)out : direct;  // written by the kernel
    // A pending batch: its last kernel (offsets, at most cap records, the
    // counters) is enqueued before the host waits, so the device does not
    // idle while the host wakes up. It runs again below if the batch had to
    // be re-run. The early run only uses staging that is already large
    // enough (a generous cap allocates nothing before the count is known).
    bool early = false;
    const bool stage_fits = (size_t)cap * sizeof(tds_hit) <= q->out_stage.bytes;
    if (q->pending && cap > 0 && (dst || stage_fits)) {
        int rc = enqueue_emit(q, dst ? dst : q->out_stage.p, cap);
        if (rc) return rc;
        early = true;
    }
    if (q->pending) {
        int rc = complete_batch(q, "tds_fetch_results");
        if (rc) return rc;
    }
    const int64_t n = q->stats.n_hit;
    *n_total = n;
    const int64_t m = std::min<int64_t>(cap, n);
    if (m > 0) {
        const bool again = !early || q->stats.retries > 0;
        if (again) {  // the records now
            if (!dst) HIP_TRY(q->out_stage.ensure((size_t)m * sizeof(tds_hit)));
            int rc = enqueue_emit(q, dst ? dst : q->out_stage.p, m);
            if (rc) return rc;
        }
        if (out_mem == TDS_MEM_HOST) {
            if (!direct)
                HIP_TRY(hipMemcpyAsync(out, q->out_stage.p, (size_t)m * sizeof(tds_hit),
                                       hipMemcpyDeviceToHost, st));
            // host output is complete on return (the early kernel finished
            // before the wait for the batch)
            if (!direct || again) HIP_TRY(wait_own(q));
        }
        // device output is ordered on the batch's stream (fetch timing is
        // read by tds_query_stats)
        if (timing) q->fetch_timed = true;
    }
    return TDS_OK;
}

// min(cap, total) merged records of the batch from the handle to `out`.
static int copy_traj(tds_query *q, tds_traj_hit *out, int64_t cap, int32_t out_mem,
                     int64_t *n_total) {
    *n_total = q->traj_total;
    const int64_t m = std::min<int64_t>(cap, q->traj_total);
    if (m > 0) {
        HIP_TRY(hipMemcpyAsync(out, q->tr_out.p, (size_t)m * sizeof(tds_traj_hit),
                               out_mem == TDS_MEM_HOST ? hipMemcpyDeviceToHost
                                                       : hipMemcpyDeviceToDevice,
                               q->stream));
        if (out_mem == TDS_MEM_HOST) HIP_TRY(wait_own(q));
    }
    return TDS_OK;
}

int tds_fetch_trajectories(tds_query *q, const int64_t *query_traj, int32_t traj_mem,
                           tds_traj_hit *out, int64_t cap, int32_t out_mem, int64_t *n_total) {
    CallStream call_stream_scope(q ? (void *)q->stream : nullptr);
    if (!q || !n_total || cap < 0 || (cap > 0 && !out))
        return fail(TDS_EINVAL, "tds_fetch_trajectories: invalid argument");
    if ((traj_mem != TDS_MEM_HOST && traj_mem != TDS_MEM_DEVICE) ||
        (out_mem != TDS_MEM_HOST && out_mem != TDS_MEM_DEVICE))
        return fail(TDS_EINVAL, "tds_fetch_trajectories: bad memory space");
    if (!q->pending && !q->fetched) return fail(TDS_ESTATE, "tds_fetch_trajectories: no batch");
    if (q->pending) {
        int rc = complete_batch(q, "tds_fetch_trajectories");
        if (rc) return rc;
    }
    const long long n = q->stats.n_hit;
    const int32_t nq = q->b.nq;
    hipStream_t st = q->stream;
    if (!query_traj) {  // copy the records of the last merge of this batch
        if (!q->traj_valid)
            return fail(TDS_ESTATE, "tds_fetch_trajectories: no merge of this batch to copy");
        return copy_traj(q, out, cap, out_mem, n_total);
    }
    *n_total = 0;
    q->traj_valid = false;
    if (n == 0) {
        q->traj_valid = true;
        q->traj_total = 0;
        return TDS_OK;
    }
    const int64_t *qt = query_traj;
    if (traj_mem == TDS_MEM_HOST) {
        HIP_TRY(q->tr_qtraj.ensure((size_t)nq * sizeof(int64_t)));
        HIP_TRY(hipMemcpyAsync(q->tr_qtraj.p, query_traj, (size_t)nq * sizeof(int64_t),
                               hipMemcpyHostToDevice, st));
        qt = q->tr_qtraj.as<int64_t>();
    }
    // work arrays: the whole keys of a small merge (2 x 32 B), the running
    // maximum's input and output (2 x 16 B), then the 8-byte ones: qt, et,
    // ta, tb, key_a, key_b, sta (7 x 8 B), then idx_a, idx_b, flag, start,
    // mid (5 x 4 B)
    const size_t nn = (size_t)n;
    const bool one = n <= kTrajOneSortMax;
    const size_t kbytes = one ? nn * 2 * sizeof(TrajKey) : 0;
    HIP_TRY(q->tr_work.ensure(kbytes + nn * (2 * sizeof(SegMax) + 7 * 8 + 5 * 4) + 64));
    char *w = q->tr_work.as<char>();
    auto take8 = [&](void *&dst) { dst = w; w += nn * 8; };
    auto take4 = [&](void *&dst) { dst = w; w += nn * 4; };
    TrajBufs t{};
    if (one) {
        t.kin = reinterpret_cast<TrajKey *>(w);
        t.kout = t.kin + nn;
        w += kbytes;
    }
    t.seg_in = reinterpret_cast<SegMax *>(w);
    t.seg_out = t.seg_in + nn;
    w += nn * 2 * sizeof(SegMax);
    take8((void *&)t.qt); take8((void *&)t.et); take8((void *&)t.ta); take8((void *&)t.tb);
    take8((void *&)t.key_a); take8((void *&)t.key_b); take8((void *&)t.sta);
    take4((void *&)t.idx_a); take4((void *&)t.idx_b); take4((void *&)t.flag);
    take4((void *&)t.start); take4((void *&)t.mid);
    // the library sorts (all but the smallest merges) need temporary storage
    const size_t temp = n <= kTrajRankMax ? 0 : traj_temp_bytes(n);
    if (n > kTrajRankMax && temp == 0)
        return fail(TDS_EDEVICE, "tds_fetch_trajectories: sort sizing failed");
    if (temp) HIP_TRY(q->tr_temp.ensure(temp));
    HIP_TRY(q->tr_out.ensure(nn * sizeof(tds_traj_hit) + sizeof(long long)));
    tds_traj_hit *recs = q->tr_out.as<tds_traj_hit>();
    long long *total_dev = reinterpret_cast<long long *>(recs + nn);
    HIP_TRY(launch_traj_merge(q->sl, q->b.ctr, n, qt, q->ix->dev, t, q->tr_temp.p,
                              q->tr_temp.bytes, recs, total_dev, st));
    // the record count to pinned host memory (after the handle's counters)
    long long *host_total = reinterpret_cast<long long *>(reinterpret_cast<char *>(q->host_ctr) + sizeof(Counters));
    HIP_TRY(hipMemcpyAsync(host_total, total_dev, sizeof(long long), hipMemcpyDeviceToHost, st));
    HIP_TRY(wait_own(q));
    q->traj_total = *host_total;
    q->traj_valid = true;
    return copy_traj(q, out, cap, out_mem, n_total);
}

int tds_query_stats(const tds_query *q, tds_stats *out) {
    if (!q || !out) return fail(TDS_EINVAL, "tds_query_stats: null argument");
    if (!q->fetched) return fail(TDS_ESTATE, "tds_query_stats: no fetched batch");
    *out = q->stats;
    // events of the last batch (complete after its fetch)
    if (q->opts.flags & (TDS_QF_TIMING | TDS_QF_TIMING_PAIR))
        HIP_TRY(hipEventElapsedTime(&out->ms_pair, q->ev[1], q->ev[2]));
    if (q->opts.flags & TDS_QF_TIMING) {
        HIP_TRY(hipEventElapsedTime(&out->ms_prep, q->ev[0], q->ev[1]));
        HIP_TRY(hipEventElapsedTime(&out->ms_refine, q->ev[2], q->ev[3]));
        if (q->fetch_timed) {
            HIP_TRY(hipEventSynchronize(q->ev[5]));
            HIP_TRY(hipEventElapsedTime(&out->ms_fetch, q->ev[4], q->ev[5]));
        }
    }
    return TDS_OK;
}

int tds_query_tiles(const tds_query *q, tds_tile_info *tiles, int64_t cap, int32_t *members,
                    int64_t member_cap, int64_t *n_tiles, int64_t *n_members) {
    if (!q || !n_tiles || !n_members || cap < 0 || member_cap < 0 || (cap > 0 && !tiles) ||
        (member_cap > 0 && !members))
        return fail(TDS_EINVAL, "tds_query_tiles: invalid argument");
    if (!q->fetched) return fail(TDS_ESTATE, "tds_query_tiles: no fetched batch");
    *n_tiles = q->stats.n_tiles;
    *n_members = q->n_sorted;
    const int64_t nt = std::min<int64_t>(cap, q->stats.n_tiles);
    if (nt > 0) {
        std::vector<Tile> t((size_t)nt);
        HIP_TRY(hipMemcpy(t.data(), q->tiles.p, (size_t)nt * sizeof(Tile), hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < nt; ++k) {
            tiles[k].q_first = t[k].q0;
            tiles[k].n_query = t[k].nq;
            tiles[k].e_first = t[k].e0;
            tiles[k].n_entry = t[k].ne;
        }
    }
    const int64_t nm = std::min<int64_t>(member_cap, q->n_sorted);
    if (nm > 0)
        HIP_TRY(hipMemcpy(members, q->perm.p, (size_t)nm * 4, hipMemcpyDeviceToHost));
    return TDS_OK;
}

int tds_query_ranges(const tds_query *q, int64_t *first, int64_t *last, int64_t n) {
    if (!q || (n > 0 && (!first || !last))) return fail(TDS_EINVAL, "tds_query_ranges: null argument");
    if (!q->fetched) return fail(TDS_ESTATE, "tds_query_ranges: no fetched batch");
    if (n != q->b.nq) return fail(TDS_EINVAL, "tds_query_ranges: n must equal the batch size");
    if (n == 0) return TDS_OK;
    std::vector<int32_t> f(n), l(n);
    HIP_TRY(hipMemcpy(f.data(), q->b.first, n * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(l.data(), q->b.last, n * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i) {
        first[i] = f[i];
        last[i] = l[i];
    }
    return TDS_OK;
}

// The per-batch buffers of one search laid out in `c` (sizes only when its
// base is null): the same arrays tds_query_batch keeps in its handle, and
// result slabs for nwaves waves plus `spill` spill slabs.
static void carve_batch(Carver &c, DevBatch &b, GreedyBufs &gb, Slabs &sl, int32_t nq, int nbuckets,
                        const tds_query_opts &o, const GreedySize *gz, int32_t nwaves,
                        long long spill) {
    const size_t n = (size_t)std::max<int32_t>(nq, 1), n1 = n + 1;
    b.rec = c.take<QRec64>(n * sizeof(QRec64));
    b.box = c.take<QCube32>(n * sizeof(QCube32));
    b.first = c.take<int32_t>(n * 4);
    b.last = c.take<int32_t>(n * 4);
    b.first_s = c.take<int32_t>(n * 4);
    b.last_s = c.take<int32_t>(n * 4);
    b.key = c.take<int32_t>(n * 4);
    b.qrank = c.take<int32_t>(n * 4);
    b.perm = c.take<int32_t>((n + 2) * 4);  // read-ahead slots
    b.tiles = c.take<Tile>(n1 * sizeof(Tile));
    b.units = c.take<long long>(n1 * 8);
    b.unit_off = c.take<long long>(n1 * 8);
    b.cost_off = c.take<long long>(n1 * 8);
    b.ctr = c.take<Counters>(sizeof(Counters));
    b.bcount = c.take<int32_t>((size_t)nbuckets * kBucketSub * 4);
    b.bq_off = c.take<int32_t>((size_t)nbuckets * kBucketSub * 4);
    b.bj2 = c.take<int32_t>((size_t)nbuckets * 4);
    b.skey = b.tkey = nullptr;
    b.sidx = b.tidx = nullptr;
    if (gz) {
        char *w = c.take<char>(gz->work);
        int32_t *j = gz->jump ? c.take<int32_t>(gz->jump) : nullptr;
        if (c.base) {
            carve_greedy(w, j, nq, *gz, &gb);
            b.skey = gb.kin;
            b.sidx = gb.vout;
            b.tkey = gb.tkey;
            b.tidx = gb.tidx;
        }
    }
    const long long ns = (long long)nwaves + 1 + spill;
    sl.wave_ovl = c.take<unsigned long long>((size_t)nwaves * 8);
    sl.cand = c.take<Cand>((size_t)ns * kSlab * sizeof(Cand));
    sl.hits = c.take<Hit24>((size_t)ns * kSlab * sizeof(Hit24));
    sl.slab_n = c.take<int32_t>((size_t)ns * 4);
    sl.slab_h = c.take<int32_t>((size_t)ns * 4);
    sl.hit_off = c.take<long long>((size_t)(ns + 1) * 8);
    sl.nwaves = nwaves;
    sl.pad = 0;
    sl.nslabs = ns;
    (void)o;
}

int tds_search_noalloc(const tds_index *ix, const tds_segments *qs, const double *d,
                       const tds_query_opts *opts, tds_hit *out, int64_t cap, int64_t *n_total,
                       void *stream) {
    const char *who = "tds_search_noalloc";
    if (!ix || !n_total || cap < 0 || (cap > 0 && !out)) return fail(TDS_EINVAL, "%s: invalid argument", who);
    *n_total = 0;
    tds_query_opts o;
    int rc = check_batch(qs, d, opts, &o, who);
    if (rc) return rc;
    if (qs->mem != TDS_MEM_DEVICE)
        return fail(TDS_EINVAL, "%s: query segments and thresholds must be in device memory", who);
    const int32_t nq = (int32_t)qs->n;
    const int nbuckets = nbuckets_for(o.tiling, ix->dev.nb, ix->dev.m);
    const int kovl = (o.flags & TDS_QF_KERNEL_OVERLAP) ? 1 : 0;
    const int grid = pair_grid(o.mode, o.block_size, o.grid, kovl);
    if (grid < 1 || (long long)grid * (o.block_size / 64) > INT32_MAX / kSlab)
        return fail(TDS_EINVAL, "%s: grid %d not supported", who, grid);
    const int32_t nwaves = grid * (o.block_size / 64);
    const bool greedy = o.tiling == TDS_TILE_GREEDY_MIN || o.tiling == TDS_TILE_GREEDY_MAX;
    const bool sorted = greedy || o.tiling == TDS_TILE_PERIODIC;
    GreedySize gz{};
    if (sorted && nq > 0) gz = greedy_size(nq, o.batch_size, o.tiling == TDS_TILE_GREEDY_MAX, greedy);

    // Layout: the fixed part with one spill slab, then as many spill slabs as fit.
    DevBatch b{};
    GreedyBufs gb{};
    Slabs sl{};
    Carver sizing{nullptr};
    carve_batch(sizing, b, gb, sl, nq, nbuckets, o, sorted && nq > 0 ? &gz : nullptr, nwaves, 1);
    const size_t fixed = sizing.used;
    if (fixed > (size_t)TDS_NOALLOC_SCRATCH_BYTES)
        return fail(TDS_EINVAL,
                    "%s: a batch of %d query segments with %d workgroups of %d threads needs %zu bytes "
                    "of scratch, more than the %zu available (TDS_NOALLOC_SCRATCH_BYTES); use "
                    "tds_query_batch or a smaller batch",
                    who, nq, grid, o.block_size, fixed, (size_t)TDS_NOALLOC_SCRATCH_BYTES);
    // each further spill slab: its candidates, hits, two counts and an offset;
    // 6 x 256 bytes cover the alignment of the regions that grow
    const size_t per_slab = kSlab * (sizeof(Cand) + sizeof(Hit24)) + 4 + 4 + 8;
    const size_t room = (size_t)TDS_NOALLOC_SCRATCH_BYTES - fixed;
    const long long spill = 1 + (room > 6 * 256 ? (long long)((room - 6 * 256) / per_slab) : 0);
    void *base = nullptr;
    rc = scratch_ptr(&base, who);
    if (rc) return rc;
    Carver c{static_cast<char *>(base)};
    carve_batch(c, b, gb, sl, nq, nbuckets, o, sorted && nq > 0 ? &gz : nullptr, nwaves,
                std::max<long long>(spill, 1));
    if (c.used > (size_t)TDS_NOALLOC_SCRATCH_BYTES)
        return fail(TDS_EINVAL, "%s: scratch layout of %zu bytes exceeds the maximum", who, c.used);
    batch_scalars(b, o, nq, nbuckets);

    hipStream_t st = (hipStream_t)stream;
    const double *qin[8] = {qs->x0, qs->y0, qs->z0, qs->t0, qs->x1, qs->y1, qs->z1, qs->t1};
    rc = enqueue_tiles(b, gb, ix, qin, d, o, st, nullptr);
    if (rc) return rc;
    if (nq > 0) {
        HIP_TRY(launch_pair(b, ix->dev, o.mode, o.block_size, o.grid, kovl, sl, st));
        HIP_TRY(launch_refine(b, ix->dev, sl, st));
        // offsets, counters and the first cap records in one kernel
        HIP_TRY(launch_emit(sl, b.ctr, cap, ix->dev, cap > 0 ? (void *)out : nullptr, kovl, nullptr,
                            NextClear{}, st));
    }
    Counters ctr{};
    HIP_TRY(hipMemcpyAsync(&ctr, b.ctr, sizeof ctr, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (ctr.err)
        return fail(TDS_EINVAL, "%s: the batch holds an invalid query segment (non-finite value, "
                                "t_end <= t_start, or d < 0)", who);
    if (ctr.spill > (unsigned long long)(sl.nslabs - sl.nwaves))
        return fail(TDS_EOVERFLOW,
                    "%s: the selections needed %llu spill slabs of %d records beyond the wave slabs; "
                    "the scratch holds %lld",
                    who, ctr.spill, kSlab, (long long)(sl.nslabs - sl.nwaves));
    *n_total = (int64_t)ctr.hits;
    return TDS_OK;
}

}  // extern "C"
