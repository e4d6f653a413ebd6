/*
 * Oracle for the distance-threshold search over trajectory line segments.
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
 * CPU-baseline leg are the only callers. It shares no code with the GPU
 * library and the library never calls it.
 *
 * What it computes (paper, Sec. 3 "Problem Definition"; Sec. 5, Alg. 1,
 * temporalIntersection() and calcTimeInterval()): for every query segment q
 * and every entry segment e -- brute force over all |Q| x n pairs, with no
 * index -- the times within the common time span of q and e at which the two
 * linearly moving points are within Euclidean distance d of each other in
 * the three spatial dimensions. A pair with a non-empty set is reported once,
 * with that set as one closed interval [t_a, t_b] (the squared distance is a
 * convex quadratic in time, so the set is one interval).
 *
 * Readings where the paper is silent:
 *  - the common time span is (max t_start, min t_end) and pairs whose spans
 *    only touch at an instant (max t_start >= min t_end) are not compared;
 *  - "within d" is closed: distance <= d, so tangency gives [t*, t*];
 *  - each segment's velocity is (p_end - p_start) / (t_end - t_start),
 *    computed once, and positions are evaluated from p_start along it;
 *  - the hit decision uses no division and no square root; the roots of the
 *    quadratic are computed only for hits, to place the interval ends.
 *
 * Arithmetic: IEEE binary64, round to nearest even, every operation below
 * written out in the order shown; a fused multiply-add appears only where
 * fma() is called. Build with -ffp-contract=off and without fast-math.
 *
 * Per pair, with dd = d*d of the query segment:
 *   tlo = max(q.t0, e.t0), thi = min(q.t1, e.t1); no comparison unless tlo < thi
 *   T = thi - tlo, tq = tlo - q.t0, te = tlo - e.t0
 *   Pq_k = fma(q.v_k, tq, q.p0_k), Pe_k = fma(e.v_k, te, e.p0_k)    (k = x, y, z)
 *   D_k = Pq_k - Pe_k, V_k = q.v_k - e.v_k
 *   the squared distance at tlo + tau is f(tau) = a tau^2 + 2 B tau + c with
 *     a = fma(Vz, Vz, fma(Vy, Vy, Vx*Vx))
 *     B = fma(Dz, Vz, fma(Dy, Vy, Dx*Vx))
 *     c = fma(Dz, Dz, fma(Dy, Dy, fma(Dx, Dx, -dd)))
 *   in0 = c <= 0                                    (within d at tlo)
 *   inT = fma(fma(a, T, B + B), T, c) <= 0          (within d at thi)
 *   vtx = B < 0 && fma(a, T, B) > 0 && fma(B, B, -(a*c)) >= 0
 *                                   (closest approach inside and within d)
 *   hit = in0 || inT || vtx
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double x0, y0, z0, t0, t1;
    double vx, vy, vz;
} oseg;

/* a[0..7] = x0, y0, z0, t0, x1, y1, z1, t1 arrays */
static void load_seg(const double *const *a, int64_t i, oseg *s)
{
    double dt = a[7][i] - a[3][i];
    s->x0 = a[0][i];
    s->y0 = a[1][i];
    s->z0 = a[2][i];
    s->t0 = a[3][i];
    s->t1 = a[7][i];
    s->vx = (a[4][i] - a[0][i]) / dt;
    s->vy = (a[5][i] - a[1][i]) / dt;
    s->vz = (a[6][i] - a[2][i]) / dt;
}

static int seg_valid(const double *const *a, int64_t i)
{
    for (int k = 0; k < 8; ++k)
        if (!isfinite(a[k][i])) return 0;
    return a[7][i] > a[3][i];
}

static double dmax(double a, double b) { return a > b ? a : b; }
static double dmin(double a, double b) { return a < b ? a : b; }

/*
 * Returns -1 when the time spans do not overlap, 0 when they overlap but the
 * points never come within d, 1 for a hit (then *ta <= *tb are written).
 */
static int pair_eval(const oseg *q, const oseg *e, double dd, double *ta, double *tb)
{
    double tlo = dmax(q->t0, e->t0);
    double thi = dmin(q->t1, e->t1);
    if (!(tlo < thi)) return -1;

    double T = thi - tlo;
    double tq = tlo - q->t0;
    double te = tlo - e->t0;

    double Dx = fma(q->vx, tq, q->x0) - fma(e->vx, te, e->x0);
    double Dy = fma(q->vy, tq, q->y0) - fma(e->vy, te, e->y0);
    double Dz = fma(q->vz, tq, q->z0) - fma(e->vz, te, e->z0);
    double Vx = q->vx - e->vx;
    double Vy = q->vy - e->vy;
    double Vz = q->vz - e->vz;

    double a = fma(Vz, Vz, fma(Vy, Vy, Vx * Vx));
    double B = fma(Dz, Vz, fma(Dy, Vy, Dx * Vx));
    double c = fma(Dz, Dz, fma(Dy, Dy, fma(Dx, Dx, -dd)));

    int in0 = c <= 0.0;
    int inT = fma(fma(a, T, B + B), T, c) <= 0.0;
    int vtx = (B < 0.0) && (fma(a, T, B) > 0.0) && (fma(B, B, -(a * c)) >= 0.0);
    if (!(in0 || inT || vtx)) return 0;

    if (in0 && inT) {           /* convex: within d over the whole span */
        *ta = tlo;
        *tb = thi;
        return 1;
    }
    /* Here a > 0: with a == 0 the distance is constant and in0 == inT. */
    double h = fma(B, B, -(a * c));
    if (h < 0.0) h = 0.0;
    double s = sqrt(h);
    double qq = (B >= 0.0) ? -(B + s) : (s - B);   /* -(B + sign(B) s) */
    double r1 = qq / a;
    double r2 = (qq != 0.0) ? c / qq : r1;
    double lo = dmin(r1, r2);
    double hi = dmax(r1, r2);
    double a_ = in0 ? tlo : tlo + dmax(lo, 0.0);
    double b_ = inT ? thi : tlo + dmin(hi, T);
    if (a_ > b_) {              /* rounding at tangency: collapse to the vertex */
        double tv = dmin(dmax(-B / a, 0.0), T);
        a_ = tlo + tv;
        b_ = a_;
    }
    *ta = a_;
    *tb = b_;
    return 1;
}

typedef struct {
    int64_t n, cap;
    int64_t *e;
    double *ta, *tb;
} hitlist;

static int push(hitlist *h, int64_t e, double ta, double tb)
{
    if (h->n == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 8;
        int64_t *ne = realloc(h->e, (size_t)nc * sizeof(int64_t));
        if (!ne) return -1;
        h->e = ne;
        double *na = realloc(h->ta, (size_t)nc * sizeof(double));
        if (!na) return -1;
        h->ta = na;
        double *nb = realloc(h->tb, (size_t)nc * sizeof(double));
        if (!nb) return -1;
        h->tb = nb;
        h->cap = nc;
    }
    h->e[h->n] = e;
    h->ta[h->n] = ta;
    h->tb[h->n] = tb;
    h->n++;
    return 0;
}

/*
 * Brute-force search. e[8] / q[8] are the x0,y0,z0,t0,x1,y1,z1,t1 arrays of
 * the entries and the query segments, qd[i] the threshold of query i.
 * Hits are written in (query, entry) order into the out_* arrays, at most
 * cap of them; the return value is the total number of hits, or -1 for an
 * invalid input (a non-finite value, t_end <= t_start, d < 0 or NaN) and -2
 * when memory runs out. *n_overlap receives the number of pairs with a
 * non-empty common time span. nthreads <= 0 uses the OpenMP default.
 */
int64_t oracle_search(int64_t ne, const double *const *e, int64_t nq,
                      const double *const *q, const double *qd, int64_t cap,
                      int64_t *out_q, int64_t *out_e, double *out_ta,
                      double *out_tb, int64_t *n_overlap, int nthreads)
{
    if (ne < 0 || nq < 0) return -1;
    for (int64_t i = 0; i < ne; ++i)
        if (!seg_valid(e, i)) return -1;
    for (int64_t i = 0; i < nq; ++i)
        if (!seg_valid(q, i) || !(qd[i] >= 0.0) || !isfinite(qd[i])) return -1;

    oseg *es = malloc((size_t)(ne > 0 ? ne : 1) * sizeof(oseg));
    hitlist *hl = calloc((size_t)(nq > 0 ? nq : 1), sizeof(hitlist));
    if (!es || !hl) {
        free(es);
        free(hl);
        return -2;
    }
    for (int64_t i = 0; i < ne; ++i) load_seg(e, i, &es[i]);

    int64_t novl = 0;
    int failed = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : novl)
    for (int64_t i = 0; i < nq; ++i) {
        oseg qs;
        load_seg(q, i, &qs);
        double dd = qd[i] * qd[i];
        for (int64_t j = 0; j < ne; ++j) {
            double ta, tb;
            int r = pair_eval(&qs, &es[j], dd, &ta, &tb);
            if (r >= 0) novl++;
            if (r == 1 && push(&hl[i], j, ta, tb) != 0) failed = 1;
        }
    }

    int64_t total = 0;
    for (int64_t i = 0; i < nq; ++i) {
        for (int64_t k = 0; k < hl[i].n; ++k, ++total) {
            if (total < cap) {
                out_q[total] = i;
                out_e[total] = hl[i].e[k];
                out_ta[total] = hl[i].ta[k];
                out_tb[total] = hl[i].tb[k];
            }
        }
        free(hl[i].e);
        free(hl[i].ta);
        free(hl[i].tb);
    }
    free(hl);
    free(es);
    if (n_overlap) *n_overlap = novl;
    return failed ? -2 : total;
}

/*
 * One pair. qs[8], es[8]: x0,y0,z0,t0,x1,y1,z1,t1 of the query and entry
 * segment. Returns -1 (no common time span), 0 (never within d) or 1 (hit,
 * out[0] = t_a, out[1] = t_b).
 */
int oracle_pair(const double *qs, const double *es, double d, double *out)
{
    const double *qa[8], *ea[8];
    for (int k = 0; k < 8; ++k) {
        qa[k] = &qs[k];
        ea[k] = &es[k];
    }
    oseg q1, e1;
    load_seg(qa, 0, &q1);
    load_seg(ea, 0, &e1);
    return pair_eval(&q1, &e1, d * d, &out[0], &out[1]);
}

int oracle_abi_version(void) { return 1; }
