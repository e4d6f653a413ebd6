// Serving runtime of the C ABI (tds_server_*): a resident index answering a
// stream of requests with continuous batching over several HIP streams.
//
// Threads: one scheduler and one executor per stream. The scheduler moves
// requests whose arrival time has come into the ready queue, and whenever an
// executor is free it takes ready requests, in arrival order, into one batch
// while their estimated result bytes fit the pool (Sec. 3: concurrent users
// compete for GPU memory; Sec. 5: result memory is reserved before the
// kernel). The executor packs the batch's segments into pinned staging,
// uploads them with one copy, runs tds_query_batch + tds_fetch_results on
// its own stream and query handle, splits the hits per request by a
// counting sort on the request of each hit's query segment, and updates the
// per-epoch hit fraction (Sec. 8's alpha) from the batch's hits and
// candidate counts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <queue>
#include <string>
#include <thread>
#include <vector>

#include "tds.h"
#include "tds_internal.h"

namespace {

// Device bytes a hit is expected to take: its result-slab records (8-byte
// selection + 24-byte hit) and its 40-byte staged output record.
constexpr double kHitBytes = 72.0;
// Device bytes a query segment takes in a handle's per-batch buffers.
constexpr double kSegBytes = 200.0;
constexpr int kMaxStreams = 8;

using Clock = std::chrono::steady_clock;

struct Request {
    int64_t id = 0;
    int64_t n = 0;
    const double *src[8] = {};  // borrowed caller arrays x0 y0 z0 t0 x1 y1 z1 t1
    const double *d = nullptr;
    double arrival = 0, admit = -1, done = -1;
    int32_t status = TDS_OK;
    bool finished = false;
    int64_t batch = -1;
    int32_t n_batch_requests = 0;
    std::vector<std::pair<int32_t, double>> epoch_eval;  // (epoch, candidate entries)
    std::vector<int32_t> seg_epoch;                      // epoch of each segment
    std::vector<double> seg_eval;                        // candidate entries of each segment
    std::vector<tds_hit> hits;
};

struct Batch {
    std::vector<Request *> reqs;
    int64_t nseg = 0;
    double est_bytes = 0;  // estimated device bytes its results need
    double est_hits = 0;
    int64_t number = 0;
};

struct Executor {
    int k = 0;
    hipStream_t stream = nullptr;
    tds_query *qh = nullptr;
    double *pin_in = nullptr;  // pinned: 9 arrays of n doubles
    int64_t pin_in_cap = 0;    // doubles
    double *dev_in = nullptr;
    int64_t dev_in_cap = 0;
    tds_hit *pin_out = nullptr;
    int64_t pin_out_cap = 0;   // records
    double reserved = 0;       // device bytes its query handle holds
    std::unique_ptr<Batch> work;
    bool busy = false;
    std::thread th;
};

int64_t grow(int64_t need, int64_t cur) { return std::max<int64_t>(need, cur + cur / 2); }

}  // namespace

struct tds_server {
    tds_index *ix = nullptr;
    tds_server_opts o{};
    Clock::time_point t0;
    std::vector<tds_bin> bins;
    double t_first = 0, t_last = 1;

    std::mutex mu;
    std::condition_variable cv_sched;  // scheduler wake-ups
    std::condition_variable cv_exec;   // executor wake-ups
    std::condition_variable cv_done;   // request completions
    std::vector<std::unique_ptr<Request>> reqs;  // by id
    // requests not yet arrived, earliest arrival first
    std::priority_queue<std::pair<double, int64_t>, std::vector<std::pair<double, int64_t>>,
                        std::greater<>> future;
    std::deque<Request *> ready;
    std::vector<std::unique_ptr<Executor>> ex;
    std::vector<double> alpha;
    bool stop = false;
    bool failed = false;
    std::string fail_msg;
    int64_t n_finished = 0, n_batches = 0, n_retries = 0, n_segments = 0;
    double busy_s = 0, stage_s = 0, wait_s = 0, split_s = 0;
    std::thread sched;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    Clock::time_point at(double s) const {
        return t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(s));
    }
    int32_t epoch_of(double t) const {
        const double span = std::max(t_last - t_first, 1e-300);
        double e = std::floor((t - t_first) / span * o.epochs);
        if (!(e >= 0)) e = 0;
        return (int32_t)std::min<double>(e, o.epochs - 1);
    }
    double est_hits(const Request &r) const {
        double h = 0;
        for (const auto &p : r.epoch_eval) h += alpha[p.first] * p.second;
        return h;
    }
    double est_bytes(const Request &r) const {
        return kHitBytes * o.k_safety * std::max(1.0, est_hits(r)) + kSegBytes * (double)r.n;
    }
    // Moves the requests whose arrival time has come into the ready queue, in
    // arrival order; one that finds max_waiting requests ready is refused
    // (status TDS_EBUSY). Caller holds mu.
    void move_arrivals(double t) {
        while (!future.empty() && future.top().first <= t) {
            Request *r = reqs[future.top().second].get();
            future.pop();
            if (o.max_waiting > 0 && (int64_t)ready.size() >= o.max_waiting) {
                r->status = TDS_EBUSY;
                r->admit = r->done = t;
                r->finished = true;
                ++n_finished;
                cv_done.notify_all();
                continue;
            }
            ready.push_back(r);
        }
    }
    void scheduler();
    void executor(Executor *e);
    void run_batch(Executor *e, Batch &b);
    void finish(Batch &b, int32_t status);
};

// ---------------------------------------------------------------- scheduler
void tds_server::scheduler() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        const double t = now();
        move_arrivals(t);
        // one batch per free executor while ready requests fit the pool
        for (auto &eptr : ex) {
            if (ready.empty()) break;
            Executor &e = *eptr;
            if (e.busy) continue;
            double others = 0;
            bool any_busy = false;
            for (auto &x : ex)
                if (x.get() != &e) {
                    others += x->reserved + (x->busy ? std::max(0.0, x->work->est_bytes - x->reserved) : 0.0);
                    any_busy |= x->busy;
                }
            auto b = std::make_unique<Batch>();
            while (!ready.empty()) {
                Request *r = ready.front();
                const double need = b->est_bytes + est_bytes(*r);
                const bool fits = others + std::max(e.reserved, need) <= o.pool_bytes;
                if (!b->reqs.empty() && (b->nseg + r->n > o.max_batch_segments || !fits)) break;
                if (b->reqs.empty() && !fits && any_busy) break;  // wait for memory to free
                ready.pop_front();
                r->admit = t;
                b->reqs.push_back(r);
                b->nseg += r->n;
                b->est_bytes = need;
                b->est_hits += est_hits(*r);
            }
            if (b->reqs.empty()) break;
            b->number = n_batches++;
            for (Request *r : b->reqs) {
                r->batch = b->number;
                r->n_batch_requests = (int32_t)b->reqs.size();
            }
            e.work = std::move(b);
            e.busy = true;
            cv_exec.notify_all();
        }
        const bool idle = future.empty() && ready.empty();
        bool all_free = true;
        for (auto &x : ex) all_free &= !x->busy;
        if (stop && idle && all_free) break;
        if (!future.empty())
            cv_sched.wait_until(lk, at(future.top().first));
        else
            cv_sched.wait(lk);
    }
    cv_exec.notify_all();
}

// ---------------------------------------------------------------- executors
void tds_server::executor(Executor *e) {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        cv_exec.wait(lk, [&] { return e->work != nullptr || (stop && !e->busy && future.empty() && ready.empty()); });
        if (!e->work) return;
        Batch &b = *e->work;
        lk.unlock();
        const double ts = now();
        run_batch(e, b);
        lk.lock();
        busy_s += now() - ts;
        e->work.reset();
        e->busy = false;
        cv_sched.notify_all();
    }
}

// Marks a batch's requests done with `status` (caller holds no lock).
void tds_server::finish(Batch &b, int32_t status) {
    std::lock_guard<std::mutex> lk(mu);
    const double t = now();
    for (Request *r : b.reqs) {
        r->status = status;
        r->done = t;
        r->finished = true;
        ++n_finished;
    }
    cv_done.notify_all();
}

void tds_server::run_batch(Executor *e, Batch &b) {
    const double t_start = now();
    const int64_t n = b.nseg;
    int rc = TDS_OK;
    auto fail_batch = [&](int code, const char *what) {
        {
            std::lock_guard<std::mutex> lk(mu);
            if (code == TDS_EDEVICE || code == TDS_ENOMEM) {
                failed = true;
                fail_msg = std::string(what) + ": " + tds_last_error();
            }
        }
        finish(b, code);
    };
    // pinned staging: x0 y0 z0 t0 x1 y1 z1 t1 d, n values each
    if (9 * n > e->pin_in_cap) {
        const int64_t c = grow(9 * n, e->pin_in_cap);
        if (e->pin_in) (void)hipHostFree(e->pin_in);
        e->pin_in = nullptr;
        if (hipHostMalloc((void **)&e->pin_in, (size_t)c * 8, hipHostMallocDefault) != hipSuccess) {
            e->pin_in_cap = 0;
            return fail_batch(TDS_ENOMEM, "hipHostMalloc");
        }
        e->pin_in_cap = c;
    }
    if (9 * n > e->dev_in_cap) {
        const int64_t c = grow(9 * n, e->dev_in_cap);
        (void)hipStreamSynchronize(e->stream);
        if (e->dev_in) (void)hipFree(e->dev_in);
        e->dev_in = nullptr;
        if (hipMalloc((void **)&e->dev_in, (size_t)c * 8) != hipSuccess) {
            e->dev_in_cap = 0;
            return fail_batch(TDS_ENOMEM, "hipMalloc");
        }
        e->dev_in_cap = c;
    }
    std::vector<int64_t> off(b.reqs.size() + 1, 0);
    for (size_t i = 0; i < b.reqs.size(); ++i) {
        const Request &r = *b.reqs[i];
        off[i + 1] = off[i] + r.n;
        for (int k = 0; k < 8; ++k)
            std::memcpy(e->pin_in + (size_t)k * n + off[i], r.src[k], (size_t)r.n * 8);
        std::memcpy(e->pin_in + (size_t)8 * n + off[i], r.d, (size_t)r.n * 8);
    }
    if (hipMemcpyAsync(e->dev_in, e->pin_in, (size_t)9 * n * 8, hipMemcpyHostToDevice, e->stream) != hipSuccess)
        return fail_batch(TDS_EDEVICE, "hipMemcpyAsync");
    tds_segments seg{};
    seg.n = n;
    seg.mem = TDS_MEM_DEVICE;
    const double **fld[8] = {&seg.x0, &seg.y0, &seg.z0, &seg.t0, &seg.x1, &seg.y1, &seg.z1, &seg.t1};
    for (int k = 0; k < 8; ++k) *fld[k] = e->dev_in + (size_t)k * n;
    tds_query_opts qo = o.query;
    qo.capacity = std::max<int64_t>((int64_t)(o.k_safety * std::max(1.0, b.est_hits)), 1 << 16);
    rc = tds_query_batch(e->qh, &seg, e->dev_in + (size_t)8 * n, &qo, e->stream);
    if (rc) return fail_batch(rc, "tds_query_batch");
    const double t_enq = now();
    int64_t total = 0;
    rc = tds_fetch_results(e->qh, e->pin_out, e->pin_out_cap, TDS_MEM_HOST, &total);
    if (rc) return fail_batch(rc, "tds_fetch_results");
    if (total > e->pin_out_cap) {  // more hits than the staging holds: grow, copy again
        const int64_t c = grow(total, e->pin_out_cap);
        if (e->pin_out) (void)hipHostFree(e->pin_out);
        e->pin_out = nullptr;
        if (hipHostMalloc((void **)&e->pin_out, (size_t)c * sizeof(tds_hit), hipHostMallocDefault) != hipSuccess) {
            e->pin_out_cap = 0;
            return fail_batch(TDS_ENOMEM, "hipHostMalloc");
        }
        e->pin_out_cap = c;
        rc = tds_fetch_results(e->qh, e->pin_out, e->pin_out_cap, TDS_MEM_HOST, &total);
        if (rc) return fail_batch(rc, "tds_fetch_results");
    }
    const double t_fetched = now();
    tds_stats st{};
    (void)tds_query_stats(e->qh, &st);
    int64_t dev_bytes = 0;
    (void)tds_query_device_bytes(e->qh, &dev_bytes);

    // split per request: the request of each hit's segment by a search over
    // the batch's segment offsets (work in the hits, not in the segments),
    // then a counting sort that keeps each request's hits in their order
    const size_t nr = b.reqs.size();
    std::vector<int32_t> hreq((size_t)total);
    std::vector<int64_t> cnt(nr, 0);
    for (int64_t h = 0; h < total; ++h) {
        const int64_t qi = e->pin_out[h].query_idx;
        const int32_t ri = (int32_t)(std::upper_bound(off.begin(), off.end(), qi) - off.begin()) - 1;
        hreq[(size_t)h] = ri;
        ++cnt[ri];
    }
    for (size_t i = 0; i < nr; ++i) b.reqs[i]->hits.resize((size_t)cnt[i]);
    std::fill(cnt.begin(), cnt.end(), 0);
    // per-epoch hit fraction of this batch -> alpha (running average): the
    // requests' candidate counts per epoch were summed at submission
    std::vector<double> ev(o.epochs, 0.0), hv(o.epochs, 0.0);
    for (int64_t h = 0; h < total; ++h) {
        tds_hit x = e->pin_out[h];
        const int32_t ri = hreq[(size_t)h];
        Request &r = *b.reqs[ri];
        x.query_idx -= off[ri];
        hv[r.seg_epoch[(size_t)x.query_idx]] += 1.0;
        r.hits[(size_t)cnt[ri]++] = x;
    }
    for (size_t i = 0; i < nr; ++i)
        for (const auto &pe : b.reqs[i]->epoch_eval) ev[pe.first] += pe.second;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (int32_t k = 0; k < o.epochs; ++k)
            if (ev[k] > 0) alpha[k] = 0.5 * alpha[k] + 0.5 * (hv[k] / ev[k]);
        e->reserved = (double)dev_bytes;
        n_retries += st.retries;
        n_segments += n;
        stage_s += t_enq - t_start;
        wait_s += t_fetched - t_enq;
        split_s += now() - t_fetched;
    }
    finish(b, TDS_OK);
}

// ---------------------------------------------------------------- C ABI
extern "C" {

int tds_server_create(tds_index *ix, const tds_server_opts *opts, tds_server **out) {
    if (!ix || !opts || !out) return tds::set_error(TDS_EINVAL, "tds_server_create: null argument");
    tds_server_opts o = *opts;
    if (o.streams == 0) o.streams = 4;
    if (o.max_batch_segments == 0) o.max_batch_segments = 65536;
    if (o.pool_bytes == 0) o.pool_bytes = 256.0 * (1 << 20);
    if (o.k_safety == 0) o.k_safety = 4.0;
    if (o.epochs == 0) o.epochs = 50;
    if (o.reserve_segments == 0) o.reserve_segments = o.max_batch_segments;
    if (o.alpha_prior == 0) o.alpha_prior = 1e-4;
    if (o.streams < 1 || o.streams > kMaxStreams || o.max_batch_segments < 1 ||
        o.max_batch_segments >= INT32_MAX / 2 || o.max_waiting < 0 || !(o.pool_bytes > 0) ||
        !(o.k_safety > 0) || o.epochs < 1 || o.epochs > 1 << 20 || o.reserve_segments < 0 ||
        !(o.alpha_prior > 0 && o.alpha_prior <= 1))
        return tds::set_error(TDS_EINVAL, "tds_server_create: option out of range");
    auto s = std::make_unique<tds_server>();
    s->ix = ix;
    s->o = o;
    tds_index_info info{};
    int rc = tds_index_info_get(ix, &info);
    if (rc) return rc;
    s->t_first = info.t_first;
    s->t_last = info.t_last;
    int64_t nb = 0;
    rc = tds_index_bins(ix, nullptr, 0, &nb);
    if (rc) return rc;
    s->bins.resize((size_t)nb);
    if (nb > 0 && (rc = tds_index_bins(ix, s->bins.data(), nb, &nb))) return rc;
    s->alpha.assign((size_t)o.epochs, o.alpha_prior);
    auto cleanup = [&] {
        for (auto &x : s->ex) {
            if (x->qh) tds_query_destroy(x->qh);
            if (x->pin_out) (void)hipHostFree(x->pin_out);
            if (x->stream) (void)hipStreamDestroy(x->stream);
        }
    };
    for (int k = 0; k < o.streams; ++k) {
        auto e = std::make_unique<Executor>();
        e->k = k;
        // default priority (no priority argument): one stream per executor
        if (hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking) != hipSuccess) {
            cleanup();
            return tds::set_error(TDS_EDEVICE, "tds_server_create: hipStreamCreateWithFlags failed");
        }
        rc = tds_query_create(ix, &e->qh);
        const int64_t cap = std::max<int64_t>((int64_t)(o.k_safety * 65536), 1 << 16);
        if (!rc) rc = tds_query_reserve(e->qh, o.reserve_segments, cap, &o.query);
        int64_t bytes = 0;
        if (!rc) rc = tds_query_device_bytes(e->qh, &bytes);
        e->reserved = (double)bytes;
        if (!rc && hipHostMalloc((void **)&e->pin_out, (size_t)cap * sizeof(tds_hit), hipHostMallocDefault) != hipSuccess)
            rc = tds::set_error(TDS_ENOMEM, "tds_server_create: hipHostMalloc failed");
        if (!rc) e->pin_out_cap = cap;
        s->ex.push_back(std::move(e));
        if (rc) {
            cleanup();
            return rc;
        }
    }
    s->t0 = Clock::now();
    tds_server *p = s.release();
    for (auto &e : p->ex) e->th = std::thread([p, ex = e.get()] { p->executor(ex); });
    p->sched = std::thread([p] { p->scheduler(); });
    *out = p;
    return TDS_OK;
}

double tds_server_now(const tds_server *s) { return s ? s->now() : 0.0; }

int tds_server_submit(tds_server *s, const tds_segments *q, const double *d, double arrival, int64_t *id) {
    if (!s || !q || !d || !id) return tds::set_error(TDS_EINVAL, "tds_server_submit: null argument");
    if (q->n < 1 || q->n >= INT32_MAX / 2 || q->mem != TDS_MEM_HOST || !std::isfinite(arrival))
        return tds::set_error(TDS_EINVAL, "tds_server_submit: n, memory space or arrival invalid");
    const double *src[8] = {q->x0, q->y0, q->z0, q->t0, q->x1, q->y1, q->z1, q->t1};
    for (int k = 0; k < 8; ++k)
        if (!src[k]) return tds::set_error(TDS_EINVAL, "tds_server_submit: null coordinate array");
    const int64_t n = q->n;
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 8; ++k)
            if (!std::isfinite(src[k][i]))
                return tds::set_error(TDS_EINVAL, "tds_server_submit: non-finite value");
        if (!(src[7][i] > src[3][i]) || !std::isfinite(d[i]) || !(d[i] >= 0.0))
            return tds::set_error(TDS_EINVAL, "tds_server_submit: invalid segment or threshold");
    }
    auto r = std::make_unique<Request>();
    r->n = n;
    for (int k = 0; k < 8; ++k) r->src[k] = src[k];
    r->d = d;
    // candidate entries per segment (Sec. 4 ranges) and their epochs
    std::vector<int64_t> f((size_t)n), l((size_t)n);
    int rc = tds_plan_ranges(s->bins.data(), (int64_t)s->bins.size(), src[3], src[7], n, f.data(), l.data());
    if (rc) return rc;
    r->seg_epoch.resize((size_t)n);
    r->seg_eval.resize((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        r->seg_epoch[i] = s->epoch_of(src[3][i]);
        r->seg_eval[i] = (double)std::max<int64_t>(l[i] - f[i] + 1, 0);
    }
    std::vector<double> per((size_t)s->o.epochs, 0.0);
    std::vector<char> seen((size_t)s->o.epochs, 0);
    std::vector<int32_t> order;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t e = r->seg_epoch[i];
        if (!seen[e]) {
            seen[e] = 1;
            order.push_back(e);
        }
        per[e] += r->seg_eval[i];
    }
    for (int32_t e : order) r->epoch_eval.emplace_back(e, per[e]);

    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failed) return tds::set_error(TDS_ESTATE, ("tds_server_submit: server stopped after " + s->fail_msg).c_str());
    if (s->stop) return tds::set_error(TDS_ESTATE, "tds_server_submit: server is stopping");
    const double t = s->now();
    // a request that has already arrived joins the ready queue here (earlier
    // arrivals first), so a full queue is reported to this caller
    const bool now_arrived = arrival <= t;
    if (now_arrived) {
        s->move_arrivals(t);
        if (s->o.max_waiting > 0 && (int64_t)s->ready.size() >= s->o.max_waiting)
            return tds::set_error(TDS_EBUSY, "tds_server_submit: waiting queue is full");
    }
    r->id = (int64_t)s->reqs.size();
    r->arrival = std::max(arrival, 0.0);
    *id = r->id;
    Request *rp = r.get();
    s->reqs.push_back(std::move(r));
    if (now_arrived)
        s->ready.push_back(rp);
    else
        s->future.emplace(rp->arrival, rp->id);
    s->cv_sched.notify_all();
    return TDS_OK;
}

int tds_server_wait(tds_server *s, int64_t id, double timeout_s, tds_request_info *info) {
    if (!s || !info) return tds::set_error(TDS_EINVAL, "tds_server_wait: null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    if (id < 0 || id >= (int64_t)s->reqs.size()) return tds::set_error(TDS_EINVAL, "tds_server_wait: unknown id");
    Request *r = s->reqs[(size_t)id].get();
    auto ready = [&] { return r->finished; };
    if (timeout_s < 0)
        s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready))
        return tds::set_error(TDS_ESTATE, "tds_server_wait: timed out");
    info->arrival = r->arrival;
    info->admit = r->admit;
    info->done = r->done;
    info->n_hit = (int64_t)r->hits.size();
    info->batch = r->batch;
    info->status = r->status;
    info->n_batch_requests = r->n_batch_requests;
    if (r->status != TDS_OK && r->status != TDS_EBUSY && !s->fail_msg.empty())
        tds::set_error(r->status, s->fail_msg.c_str());
    return TDS_OK;
}

int tds_server_results(tds_server *s, int64_t id, tds_hit *out, int64_t cap, int64_t *n_total) {
    if (!s || !n_total || cap < 0 || (cap > 0 && !out))
        return tds::set_error(TDS_EINVAL, "tds_server_results: invalid argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (id < 0 || id >= (int64_t)s->reqs.size()) return tds::set_error(TDS_EINVAL, "tds_server_results: unknown id");
    Request *r = s->reqs[(size_t)id].get();
    if (!r->finished) return tds::set_error(TDS_ESTATE, "tds_server_results: request not done");
    *n_total = (int64_t)r->hits.size();
    const int64_t m = std::min<int64_t>(cap, *n_total);
    if (m > 0) std::memcpy(out, r->hits.data(), (size_t)m * sizeof(tds_hit));
    return TDS_OK;
}

int tds_server_release(tds_server *s, int64_t id) {
    if (!s) return tds::set_error(TDS_EINVAL, "tds_server_release: null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (id < 0 || id >= (int64_t)s->reqs.size()) return tds::set_error(TDS_EINVAL, "tds_server_release: unknown id");
    Request *r = s->reqs[(size_t)id].get();
    if (!r->finished) return tds::set_error(TDS_ESTATE, "tds_server_release: request not done");
    std::vector<tds_hit>().swap(r->hits);
    std::vector<int32_t>().swap(r->seg_epoch);
    std::vector<double>().swap(r->seg_eval);
    return TDS_OK;
}

int tds_server_stats_get(const tds_server *s, tds_server_stats *out) {
    if (!s || !out) return tds::set_error(TDS_EINVAL, "tds_server_stats_get: null argument");
    tds_server *m = const_cast<tds_server *>(s);
    std::lock_guard<std::mutex> lk(m->mu);
    out->batches = m->n_batches;
    out->requests_done = m->n_finished;
    out->retries = m->n_retries;
    out->segments = m->n_segments;
    double b = 0;
    for (auto &e : m->ex) b += e->reserved;
    out->device_bytes = (int64_t)b;
    out->busy_s = m->busy_s;
    out->stage_s = m->stage_s;
    out->wait_s = m->wait_s;
    out->split_s = m->split_s;
    return TDS_OK;
}

int tds_server_alpha(const tds_server *s, double *alpha, int32_t cap, int32_t *n) {
    if (!s || !n || cap < 0 || (cap > 0 && !alpha)) return tds::set_error(TDS_EINVAL, "tds_server_alpha: invalid argument");
    tds_server *m = const_cast<tds_server *>(s);
    std::lock_guard<std::mutex> lk(m->mu);
    *n = (int32_t)m->alpha.size();
    for (int32_t k = 0; k < std::min(cap, *n); ++k) alpha[k] = m->alpha[(size_t)k];
    return TDS_OK;
}

void tds_server_destroy(tds_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_sched.notify_all();
        s->cv_exec.notify_all();
    }
    if (s->sched.joinable()) s->sched.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->cv_exec.notify_all();
    }
    for (auto &e : s->ex)
        if (e->th.joinable()) e->th.join();
    for (auto &e : s->ex) {
        if (e->qh) tds_query_destroy(e->qh);
        if (e->stream) (void)hipStreamSynchronize(e->stream);
        if (e->dev_in) (void)hipFree(e->dev_in);
        if (e->pin_in) (void)hipHostFree(e->pin_in);
        if (e->pin_out) (void)hipHostFree(e->pin_out);
        if (e->stream) (void)hipStreamDestroy(e->stream);
    }
    delete s;
}

}  // extern "C"
