// Host runtime of the C ABI declared in include/tds.h: argument checks,
// index construction (sort by t_start, temporal bins, upload), query-batch
// orchestration on a HIP stream, overflow retry and result translation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/tds.h"
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
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need) {
        if (need <= bytes) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            bytes = 0;
        }
        size_t nb = std::max<size_t>(need, 256);
        hipError_t e = hipMalloc(&p, nb);
        if (e == hipSuccess) bytes = nb;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
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
        *t_first = *t_last = *width = 0.0;
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

}  // namespace

struct tds_index {
    int device = 0;
    int64_t n = 0;
    int32_t m = 0;
    double t_first = 0, t_last = 0, width = 0;
    std::vector<tds_bin> bins;
    DBuf t0, t1, x0, y0, z0, vx, vy, vz, boxa, boxb, orig, traj, t1s;
    DBuf bstart, bpend, bfirst, blast;
    DevIndex dev{};
    int64_t device_bytes = 0;
    int live_queries = 0;
};

struct tds_query {
    tds_index *ix = nullptr;
    int32_t cap_q = 0;  // query slots allocated
    DBuf rec, box, rec_s, box_s, first, last, first_s, last_s, key_in, key_out, val_in, perm;
    DBuf head, tile_of_head, tiles, items, item_off, ctr, sort_tmp, scan_tmp;
    DBuf qstage, hits, out_stage;
    size_t sort_bytes = 0, scan_bytes = 0;
    unsigned long long cap_hits = 0;
    Counters *host_ctr = nullptr;  // pinned
    hipStream_t stream = nullptr;
    DevBatch b{};
    tds_query_opts opts{};
    int block = 256, grid = 0;
    bool pending = false, fetched = false;
    tds_stats stats{};
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

extern "C" {

const char *tds_last_error(void) { return g_err.c_str(); }
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
    std::vector<double> pend(nb);
    for (int64_t k = 0; k < nb; ++k) pend[k] = k ? std::max(pend[k - 1], bins[k].end) : bins[k].end;
    for (int64_t i = 0; i < nq; ++i) {
        int64_t j1 = std::upper_bound(pend.begin(), pend.end(), t0[i]) - pend.begin();
        int64_t lo = 0, hi = nb;  // number of bins with start < t1
        while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (bins[mid].start < t1[i]) lo = mid + 1; else hi = mid;
        }
        int64_t j2 = lo - 1;
        if (j1 <= j2) {
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
    if (!db || !opts || !out) return fail(TDS_EINVAL, "tds_build_index: null argument");
    *out = nullptr;
    if (db->n < 0 || db->n >= (int64_t)INT32_MAX)
        return fail(TDS_EINVAL, "tds_build_index: n = %lld out of range", (long long)db->n);
    if (opts->num_bins < 1) return fail(TDS_EINVAL, "tds_build_index: num_bins must be >= 1");
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
    std::vector<int64_t> traj_h;
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
    const int64_t *traj_src = db->traj_id;
    if (traj_src && db->mem == TDS_MEM_DEVICE && n > 0) {
        traj_h.resize(n);
        HIP_TRY(hipMemcpy(traj_h.data(), traj_src, n * sizeof(int64_t), hipMemcpyDeviceToHost));
        traj_src = traj_h.data();
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
    double ext_max = 0.0, mag_max = 0.0;
    for (int64_t p = 0; p < n; ++p) {
        int32_t i = perm[p];
        t0s[p] = h[3][i];
        t1p[p] = h[7][i];
        ext_max = std::max(ext_max, std::fabs(h[4][i] - h[0][i]) + std::fabs(h[5][i] - h[1][i]) +
                                        std::fabs(h[6][i] - h[2][i]));
        for (int k : {0, 1, 2, 4, 5, 6}) mag_max = std::max(mag_max, std::fabs(h[k][i]));
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

    size_t d8 = (size_t)std::max<int64_t>(n, 1) * 8;
    for (DBuf *b : {&ix->t0, &ix->t1, &ix->x0, &ix->y0, &ix->z0, &ix->vx, &ix->vy, &ix->vz,
                    &ix->traj, &ix->t1s})
        IX_TRY(b->ensure(d8));
    IX_TRY(ix->boxa.ensure((size_t)std::max<int64_t>(n, 1) * 16));
    IX_TRY(ix->boxb.ensure((size_t)std::max<int64_t>(n, 1) * 16));
    IX_TRY(ix->orig.ensure((size_t)std::max<int64_t>(n, 1) * 4));
    size_t b8 = (size_t)std::max<int64_t>(nb, 1) * 8, b4 = (size_t)std::max<int64_t>(nb, 1) * 4;
    IX_TRY(ix->bstart.ensure(b8));
    IX_TRY(ix->bpend.ensure(b8));
    IX_TRY(ix->bfirst.ensure(b4));
    IX_TRY(ix->blast.ensure(b4));

    std::vector<double> bs(nb), bp(nb);
    std::vector<int32_t> bf(nb), bl(nb);
    for (int64_t k = 0; k < nb; ++k) {
        bs[k] = ix->bins[k].start;
        bp[k] = k ? std::max(bp[k - 1], ix->bins[k].end) : ix->bins[k].end;
        bf[k] = (int32_t)ix->bins[k].first;
        bl[k] = (int32_t)ix->bins[k].last;
    }

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
        IX_TRY(launch_ingest(rawp, n, dperm.as<int32_t>(), traj_dev, DevIndex{}, ix->t0.as<double>(),
                             ix->t1.as<double>(), ix->x0.as<double>(), ix->y0.as<double>(),
                             ix->z0.as<double>(), ix->vx.as<double>(), ix->vy.as<double>(),
                             ix->vz.as<double>(), ix->boxa.as<float4>(), ix->boxb.as<float4>(),
                             ix->orig.as<int32_t>(), ix->traj.as<int64_t>(), st));
        IX_TRY(hipMemcpyAsync(ix->t1s.p, t1s.data(), n * 8, hipMemcpyHostToDevice, st));
        IX_TRY(hipMemcpyAsync(ix->bstart.p, bs.data(), nb * 8, hipMemcpyHostToDevice, st));
        IX_TRY(hipMemcpyAsync(ix->bpend.p, bp.data(), nb * 8, hipMemcpyHostToDevice, st));
        IX_TRY(hipMemcpyAsync(ix->bfirst.p, bf.data(), nb * 4, hipMemcpyHostToDevice, st));
        IX_TRY(hipMemcpyAsync(ix->blast.p, bl.data(), nb * 4, hipMemcpyHostToDevice, st));
        IX_TRY(hipStreamSynchronize(st));
        raw.release();
        dperm.release();
        dtraj.release();
    }
#undef IX_TRY

    DevIndex &d = ix->dev;
    d.n = n;
    d.nb = (int32_t)nb;
    d.t0 = ix->t0.as<double>();
    d.t1 = ix->t1.as<double>();
    d.x0 = ix->x0.as<double>();
    d.y0 = ix->y0.as<double>();
    d.z0 = ix->z0.as<double>();
    d.vx = ix->vx.as<double>();
    d.vy = ix->vy.as<double>();
    d.vz = ix->vz.as<double>();
    d.boxa = ix->boxa.as<float4>();
    d.boxb = ix->boxb.as<float4>();
    d.orig = ix->orig.as<int32_t>();
    d.traj = ix->traj.as<int64_t>();
    d.t0s = d.t0;  // entries are sorted by t_start
    d.t1s = ix->t1s.as<double>();
    d.bstart = ix->bstart.as<double>();
    d.bpend = ix->bpend.as<double>();
    d.bfirst = ix->bfirst.as<int32_t>();
    d.blast = ix->blast.as<int32_t>();
    // Box slack: a binary64 hit implies the exact distance is within
    // d + 8 sqrt(eps) (d + relative travel) at some common time; 2^-20 keeps
    // a factor > 10 over that. Positions carry a few ulps of their magnitude;
    // 2^-40 per unit of magnitude covers it by a wide margin.
    d.band_rel = std::ldexp(1.0, -20);
    d.band_abs = std::ldexp(1.0, -40);
    d.ext_max = ext_max;
    d.mag_max = mag_max;
    ix->device_bytes = (int64_t)(n * (8 * 8 + 32 + 4 + 8 + 8) + nb * 24);
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
    out->bin_width = ix->width;
    out->device_bytes = ix->device_bytes;
    return TDS_OK;
}

int tds_index_bins(const tds_index *ix, tds_bin *out, int64_t cap, int64_t *n_out) {
    if (!ix || !n_out || (cap > 0 && !out)) return fail(TDS_EINVAL, "tds_index_bins: null argument");
    *n_out = (int64_t)ix->bins.size();
    for (int64_t k = 0; k < *n_out && k < cap; ++k) out[k] = ix->bins[k];
    return TDS_OK;
}

void tds_index_destroy(tds_index *ix) {
    if (!ix) return;
    for (DBuf *b : {&ix->t0, &ix->t1, &ix->x0, &ix->y0, &ix->z0, &ix->vx, &ix->vy, &ix->vz,
                    &ix->boxa, &ix->boxb, &ix->orig, &ix->traj, &ix->t1s, &ix->bstart, &ix->bpend,
                    &ix->bfirst, &ix->blast})
        b->release();
    delete ix;
}

int tds_query_create(tds_index *ix, tds_query **out) {
    if (!ix || !out) return fail(TDS_EINVAL, "tds_query_create: null argument");
    tds_query *q = new tds_query();
    q->ix = ix;
    hipError_t e = hipHostMalloc((void **)&q->host_ctr, sizeof(Counters), hipHostMallocDefault);
    if (e != hipSuccess) {
        delete q;
        return fail(TDS_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    std::memset(q->host_ctr, 0, sizeof(Counters));
    for (auto &ev : q->ev) {
        e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            tds_query_destroy(q);
            return fail(TDS_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
        }
    }
    ix->live_queries++;
    *out = q;
    return TDS_OK;
}

void tds_query_destroy(tds_query *q) {
    if (!q) return;
    if (q->pending && q->stream) (void)hipStreamSynchronize(q->stream);
    for (DBuf *b : {&q->rec, &q->box, &q->rec_s, &q->box_s, &q->first, &q->last, &q->first_s,
                    &q->last_s, &q->key_in, &q->key_out, &q->val_in, &q->perm, &q->head,
                    &q->tile_of_head, &q->tiles, &q->items, &q->item_off, &q->ctr, &q->sort_tmp,
                    &q->scan_tmp, &q->qstage, &q->hits, &q->out_stage})
        b->release();
    if (q->host_ctr) (void)hipHostFree(q->host_ctr);
    for (auto &ev : q->ev)
        if (ev) (void)hipEventDestroy(ev);
    if (q->ix) q->ix->live_queries--;
    delete q;
}

static int ensure_query_capacity(tds_query *q, int32_t nq) {
    if (nq <= q->cap_q && q->ctr.p) return TDS_OK;
    int32_t c = std::max<int32_t>(nq, std::max<int32_t>(1024, q->cap_q + q->cap_q / 2));
    size_t n = (size_t)c;
    HIP_TRY(q->rec.ensure(n * sizeof(QRec64)));
    HIP_TRY(q->rec_s.ensure(n * sizeof(QRec64)));
    HIP_TRY(q->box.ensure(n * sizeof(QBox32)));
    HIP_TRY(q->box_s.ensure(n * sizeof(QBox32)));
    for (DBuf *b : {&q->first, &q->last, &q->first_s, &q->last_s, &q->val_in, &q->perm, &q->head,
                    &q->tile_of_head, &q->items, &q->item_off})
        HIP_TRY(b->ensure(n * 4));
    HIP_TRY(q->key_in.ensure(n * 8));
    HIP_TRY(q->key_out.ensure(n * 8));
    HIP_TRY(q->tiles.ensure(n * sizeof(Tile)));
    HIP_TRY(q->ctr.ensure(sizeof(Counters)));
    size_t sb = 0, cb = 0;
    HIP_TRY(sort_temp_bytes(c, &sb));
    HIP_TRY(scan_temp_bytes(c, &cb));
    HIP_TRY(q->sort_tmp.ensure(sb));
    HIP_TRY(q->scan_tmp.ensure(cb));
    q->sort_bytes = q->sort_tmp.bytes;
    q->scan_bytes = q->scan_tmp.bytes;
    q->cap_q = c;
    return TDS_OK;
}

static int default_grid(int block) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return cus * std::max(1, 2048 / block);
}

static int launch_pair_now(tds_query *q) {
    HIP_TRY(launch_pair(q->b, q->ix->dev, q->opts.mode, q->block, q->grid,
                        (q->opts.flags & TDS_QF_COUNT_OVERLAP) ? 1 : 0, q->hits.as<Hit24>(),
                        q->cap_hits, q->stream));
    return TDS_OK;
}

int tds_query_batch(tds_query *q, const tds_segments *qs, const double *d,
                    const tds_query_opts *opts, void *stream) {
    if (!q || !qs || !opts || (qs->n > 0 && !d)) return fail(TDS_EINVAL, "tds_query_batch: null argument");
    if (q->pending) return fail(TDS_ESTATE, "tds_query_batch: previous batch not fetched");
    if (qs->n < 0 || qs->n >= (int64_t)INT32_MAX / 2)
        return fail(TDS_EINVAL, "tds_query_batch: n = %lld out of range", (long long)qs->n);
    if (qs->mem != TDS_MEM_HOST && qs->mem != TDS_MEM_DEVICE)
        return fail(TDS_EINVAL, "tds_query_batch: bad mem");
    tds_query_opts o = *opts;
    if (o.mode != TDS_MODE_FP64 && o.mode != TDS_MODE_FP32_REFINE)
        return fail(TDS_EINVAL, "tds_query_batch: unknown mode %d", o.mode);
    if (o.tiling != TDS_TILE_PERIODIC && o.tiling != TDS_TILE_RANGE)
        return fail(TDS_EINVAL, "tds_query_batch: unknown tiling %d", o.tiling);
    if (o.batch_size == 0) o.batch_size = 128;
    if (o.batch_size < 1 || o.batch_size > 4096)
        return fail(TDS_EINVAL, "tds_query_batch: batch_size %d out of 1..4096", o.batch_size);
    if (o.block_size == 0) o.block_size = 256;
    if (o.block_size != 64 && o.block_size != 128 && o.block_size != 256 && o.block_size != 512 &&
        o.block_size != 1024)
        return fail(TDS_EINVAL, "tds_query_batch: block_size %d not supported", o.block_size);
    if (o.max_retries < 0) o.max_retries = 4;
    if (o.capacity < 0 || o.grid < 0) return fail(TDS_EINVAL, "tds_query_batch: negative option");
    const double *src[8] = {qs->x0, qs->y0, qs->z0, qs->t0, qs->x1, qs->y1, qs->z1, qs->t1};
    const int32_t nq = (int32_t)qs->n;
    if (nq > 0)
        for (int k = 0; k < 8; ++k)
            if (!src[k]) return fail(TDS_EINVAL, "tds_query_batch: null coordinate array");
    if (qs->mem == TDS_MEM_HOST) {  // host inputs are checked here, device ones by the kernel
        for (int32_t i = 0; i < nq; ++i)
            if (!seg_ok(src, i) || !std::isfinite(d[i]) || !(d[i] >= 0.0))
                return fail(TDS_EINVAL, "tds_query_batch: query segment %d is invalid", i);
    }

    hipStream_t st = (hipStream_t)stream;
    q->stream = st;
    q->opts = o;
    q->block = o.block_size;
    q->grid = o.grid ? o.grid : default_grid(o.block_size);
    int rc = ensure_query_capacity(q, std::max<int32_t>(nq, 1));
    if (rc) return rc;
    unsigned long long want = o.capacity > 0 ? (unsigned long long)o.capacity : (1ull << 20);
    if (q->cap_hits < want || !q->hits.p) {
        HIP_TRY(q->hits.ensure(want * sizeof(Hit24)));
        q->cap_hits = q->hits.bytes / sizeof(Hit24);
    }

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
    b.nq = nq;
    b.s = o.batch_size;
    b.tiling = o.tiling;
    b.chunk = chunk_for(o.mode, o.block_size);
    b.rec = q->rec.as<QRec64>();
    b.box = q->box.as<QBox32>();
    b.rec_s = q->rec_s.as<QRec64>();
    b.box_s = q->box_s.as<QBox32>();
    b.first = q->first.as<int32_t>();
    b.last = q->last.as<int32_t>();
    b.first_s = q->first_s.as<int32_t>();
    b.last_s = q->last_s.as<int32_t>();
    b.key_in = q->key_in.as<unsigned long long>();
    b.key_out = q->key_out.as<unsigned long long>();
    b.val_in = q->val_in.as<int32_t>();
    b.perm = q->perm.as<int32_t>();
    b.head = q->head.as<int32_t>();
    b.tile_of_head = q->tile_of_head.as<int32_t>();
    b.tiles = q->tiles.as<Tile>();
    b.items = q->items.as<int32_t>();
    b.item_off = q->item_off.as<int32_t>();
    b.ctr = q->ctr.as<Counters>();

    const bool timing = (o.flags & TDS_QF_TIMING) != 0;
    if (timing) HIP_TRY(hipEventRecord(q->ev[0], st));
    HIP_TRY(launch_zero_counters(b.ctr, st));
    if (nq > 0) {
        const tds_index *ix = q->ix;
        double span = ix->t_last - ix->t_first;
        if (!(span > 0.0)) span = 1.0;
        HIP_TRY(launch_qprep(qin, din, b, ix->dev, ix->t_first, span, st));
        int end_bit = 32;
        if (o.tiling == TDS_TILE_RANGE) {
            unsigned long long maxkey =
                (unsigned long long)ix->dev.nb * ((unsigned long long)ix->dev.nb + 1ull);
            end_bit = 1;
            while (end_bit < 64 && (maxkey >> end_bit) != 0ull) ++end_bit;
        }
        HIP_TRY(launch_sort(q->sort_tmp.p, q->sort_bytes, b, end_bit, st));
        HIP_TRY(launch_gather(b, ix->dev, st));
        if (o.tiling == TDS_TILE_RANGE)
            HIP_TRY(launch_scan(q->scan_tmp.p, q->scan_bytes, b.head, b.tile_of_head, nq, st));
        HIP_TRY(launch_tiles(b, st));
        HIP_TRY(launch_scan(q->scan_tmp.p, q->scan_bytes, b.items, b.item_off, nq, st));
        if (timing) HIP_TRY(hipEventRecord(q->ev[1], st));
        rc = launch_pair_now(q);
        if (rc) return rc;
        if (timing) HIP_TRY(hipEventRecord(q->ev[2], st));
    } else if (timing) {
        HIP_TRY(hipEventRecord(q->ev[1], st));
        HIP_TRY(hipEventRecord(q->ev[2], st));
    }
    HIP_TRY(hipMemcpyAsync(q->host_ctr, b.ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
    q->pending = true;
    q->fetched = false;
    std::memset(&q->stats, 0, sizeof q->stats);
    q->stats.n_query = nq;
    q->stats.grid = q->grid;
    return TDS_OK;
}

int tds_fetch_results(tds_query *q, tds_hit *out, int64_t cap, int32_t out_mem, int64_t *n_total) {
    if (!q || !n_total || cap < 0 || (cap > 0 && !out))
        return fail(TDS_EINVAL, "tds_fetch_results: invalid argument");
    if (out_mem != TDS_MEM_HOST && out_mem != TDS_MEM_DEVICE)
        return fail(TDS_EINVAL, "tds_fetch_results: bad out_mem");
    if (!q->pending && !q->fetched) return fail(TDS_ESTATE, "tds_fetch_results: no batch");
    hipStream_t st = q->stream;
    if (q->pending) {
        HIP_TRY(hipStreamSynchronize(st));
        Counters c = *q->host_ctr;
        if (c.err) {
            q->pending = false;
            return fail(TDS_EINVAL, "tds_fetch_results: the batch holds an invalid query segment "
                                    "(non-finite value, t_end <= t_start, or d < 0)");
        }
        int retries = 0;
        while (c.hits > q->cap_hits) {
            if (retries >= q->opts.max_retries) {
                q->pending = false;
                return fail(TDS_EOVERFLOW, "tds_fetch_results: %llu hits exceed capacity %llu",
                            c.hits, q->cap_hits);
            }
            ++retries;
            unsigned long long need = c.hits + c.hits / 4 + 1024;
            HIP_TRY(q->hits.ensure(need * sizeof(Hit24)));
            q->cap_hits = q->hits.bytes / sizeof(Hit24);
            // Counters the pair kernel accumulates start again from zero.
            Counters keep = c;
            keep.hits = keep.refine = keep.overlap = 0;
            HIP_TRY(hipMemcpyAsync(q->b.ctr, &keep, sizeof(Counters), hipMemcpyHostToDevice, st));
            HIP_TRY(hipStreamSynchronize(st));
            if (q->opts.flags & TDS_QF_TIMING) HIP_TRY(hipEventRecord(q->ev[1], st));
            int rc = launch_pair_now(q);
            if (rc) return rc;
            if (q->opts.flags & TDS_QF_TIMING) HIP_TRY(hipEventRecord(q->ev[2], st));
            HIP_TRY(hipMemcpyAsync(q->host_ctr, q->b.ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            c = *q->host_ctr;
        }
        tds_stats &s = q->stats;
        s.n_eval = (int64_t)c.n_eval;
        s.n_overlap = (int64_t)c.n_overlap_exact;
        s.n_overlap_k = (q->opts.flags & TDS_QF_COUNT_OVERLAP) ? (int64_t)c.overlap : -1;
        s.n_refine = q->opts.mode == TDS_MODE_FP32_REFINE ? (int64_t)c.refine : -1;
        s.n_hit = (int64_t)c.hits;
        s.n_tiles = (int64_t)c.n_tiles;
        s.retries = retries;
        s.n_items = (int64_t)c.n_items;
        if (q->opts.flags & TDS_QF_TIMING) {
            HIP_TRY(hipEventElapsedTime(&s.ms_prep, q->ev[0], q->ev[1]));
            HIP_TRY(hipEventElapsedTime(&s.ms_pair, q->ev[1], q->ev[2]));
        }
        q->pending = false;
        q->fetched = true;
    }
    int64_t n = q->stats.n_hit;
    *n_total = n;
    int64_t m = std::min<int64_t>(cap, n);
    if (m > 0) {
        bool timing = (q->opts.flags & TDS_QF_TIMING) != 0;
        if (timing) HIP_TRY(hipEventRecord(q->ev[0], st));
        if (out_mem == TDS_MEM_DEVICE) {
            HIP_TRY(launch_translate(q->hits.as<Hit24>(), m, q->b.perm, q->ix->dev, out, st));
        } else {
            HIP_TRY(q->out_stage.ensure((size_t)m * sizeof(tds_hit)));
            HIP_TRY(launch_translate(q->hits.as<Hit24>(), m, q->b.perm, q->ix->dev, q->out_stage.p, st));
            HIP_TRY(hipMemcpyAsync(out, q->out_stage.p, (size_t)m * sizeof(tds_hit),
                                   hipMemcpyDeviceToHost, st));
        }
        if (timing) HIP_TRY(hipEventRecord(q->ev[3], st));
        HIP_TRY(hipStreamSynchronize(st));
        if (timing) HIP_TRY(hipEventElapsedTime(&q->stats.ms_fetch, q->ev[0], q->ev[3]));
    }
    return TDS_OK;
}

int tds_query_stats(const tds_query *q, tds_stats *out) {
    if (!q || !out) return fail(TDS_EINVAL, "tds_query_stats: null argument");
    if (!q->fetched) return fail(TDS_ESTATE, "tds_query_stats: no fetched batch");
    *out = q->stats;
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

}  // extern "C"
