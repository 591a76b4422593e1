/*
 * CPU oracle for the first-level J/psi trigger-station triplet selection.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline of the benchmark load it.  It shares no source with the GPU
 * library: its structs, constants and arithmetic are written here from the
 * paper.
 *
 * What it computes (paper, Sec. 3.2 "Algorithm", steps 1-3):
 *   1. every triplet (i, j, k) with one hit from each of the three
 *      trigger-station layers;
 *   2. (a) a straight-line fit through the event vertex, separately in the
 *      x-z and y-z planes (x = m0 z, y = m1 z);
 *      (b) the mean square deviation of that fit per degree of freedom; the
 *      triplet is rejected if it exceeds the plane's threshold;
 *   3. the event is selected if at least two triplets pass.
 *
 * Floating point.  The paper fixes no precision.  The decision is taken in
 * IEEE-754 binary32 (round to nearest even, subnormals kept, no fused
 * multiply-add: build with -ffp-contract=off and without -ffast-math), in the
 * operation order written out below, so that an independent implementation
 * can reproduce every decision bit for bit.  The exact-arithmetic definition
 * of the same fit lives in reference.py and pins these decisions.
 *
 * Three tests are provided:
 *   MSD (default)  the fit of Sec. 3.2 step 2 written out: slope
 *                  m = sum(c z) / sum(z^2) through the vertex (the division
 *                  taken as a product with w = 1 / sum(z^2), rounded once),
 *                  residuals r_l = c_l - m z_l, Q = sum r_l^2.
 *   MSD_BASIS      the same fit's Q evaluated as the squared length of the
 *                  measurement vector's component orthogonal to the layer
 *                  vector z = (z0, z1, z2), in the orthonormal basis (u, v)
 *                  of that plane with u = (z1, -z0, 0)/|(z0, z1)| and
 *                  v = (z0 z2, z1 z2, -(z0^2 + z1^2)) / (|(z0, z1)| |z|).
 *                  In exact arithmetic Q = min_m sum_l (c_l - m z_l)^2, the
 *                  same number; in binary32 the two orders round differently.
 *   WINDOW         slope-window test: |c_l/z_l - c_0/z_0| < W for l = 1, 2.
 * For the MSD tests the triplet passes a plane iff fl(Q / ndf) <= T.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

enum { OR_TEST_MSD = 0, OR_TEST_WINDOW = 1, OR_TEST_MSD_BASIS = 2 };

typedef struct {
    int32_t test;
    float z[3];
    float msd_max[2]; /* per degree of freedom: x-z plane, y-z plane */
    int32_t ndf;
    float window[2];
    int32_t min_triplets;
} oracle_cfg;

typedef struct {
    /* MSD: layer positions and w = 1 / sum z^2 */
    float zf[3], w;
    /* MSD_BASIS: orthonormal basis of the plane orthogonal to z */
    float U0, U1, V0, V1, V2;
} oracle_consts;

static void make_consts(const oracle_cfg *c, oracle_consts *k) {
    double z0 = c->z[0], z1 = c->z[1], z2 = c->z[2];
    double s01 = z0 * z0 + z1 * z1;
    double n01 = sqrt(s01);
    double szz = s01 + z2 * z2;
    double nz = sqrt(szz);
    double d = n01 * nz;
    k->U0 = (float)(z1 / n01);
    k->U1 = (float)(-z0 / n01);
    k->V0 = (float)((z0 * z2) / d);
    k->V1 = (float)((z1 * z2) / d);
    k->V2 = (float)(-s01 / d);
    for (int l = 0; l < 3; ++l) k->zf[l] = c->z[l];
    float sz = (c->z[0] * c->z[0] + c->z[1] * c->z[1]) + c->z[2] * c->z[2];
    k->w = (float)(1.0 / (double)sz);
}

/* One plane of the MSD_BASIS test. */
static int plane_msd(float ci, float cj, float ck, const oracle_consts *k, float T, float ndf) {
    float a = k->U0 * ci + k->U1 * cj;
    float b = (k->V0 * ci + k->V1 * cj) + k->V2 * ck;
    float q = a * a + b * b;
    float msd = q / ndf;
    return msd <= T;
}

/* One plane of the MSD test: the fit through the vertex written out. */
static int plane_fit(float ci, float cj, float ck, const oracle_consts *k, float T, float ndf) {
    float p0 = ci * k->zf[0], p1 = cj * k->zf[1], p2 = ck * k->zf[2];
    float m = ((p0 + p1) + p2) * k->w;
    float r0 = ci - m * k->zf[0];
    float r1 = cj - m * k->zf[1];
    float r2 = ck - m * k->zf[2];
    float q = (r0 * r0 + r1 * r1) + r2 * r2;
    float msd = q / ndf;
    return msd <= T;
}

/* One plane of the MSD test when every hit carries its own z (staggered
 * detector modules, Sec. 3.2 last paragraph): the same fit, with the sum of
 * squares of the triplet's own z and its reciprocal taken per triplet (one
 * binary32 division). */
static int plane_fit_z(float ci, float cj, float ck, float zi, float zj, float zk, float T, float ndf) {
    float szz = (zi * zi + zj * zj) + zk * zk;
    float w = 1.0f / szz;
    float m = ((ci * zi + cj * zj) + ck * zk) * w;
    float r0 = ci - m * zi;
    float r1 = cj - m * zj;
    float r2 = ck - m * zk;
    float q = (r0 * r0 + r1 * r1) + r2 * r2;
    float msd = q / ndf;
    return msd <= T;
}

/* One plane of the slope-window test with per-hit z. */
static int plane_window_z(float ci, float cj, float ck, float zi, float zj, float zk, float W) {
    float si = ci / zi, sj = cj / zj, sk = ck / zk;
    return fabsf(sj - si) < W && fabsf(sk - si) < W;
}

/* One plane of the slope-window test. */
static int plane_window(float ci, float cj, float ck, const oracle_consts *k, float W) {
    float si = ci / k->zf[0], sj = cj / k->zf[1], sk = ck / k->zf[2];
    return fabsf(sj - si) < W && fabsf(sk - si) < W;
}

/* Whether triplet (i, j, kk) passes both planes of the configured test;
 * z (may be NULL) holds per-hit z positions. */
static int triplet_passes(const oracle_cfg *c, const oracle_consts *k, const float *x, const float *y,
                          const float *z, int64_t i, int64_t j, int64_t kk) {
    const float ndf = (float)c->ndf;
    if (z) {
        if (c->test == OR_TEST_WINDOW)
            return plane_window_z(x[i], x[j], x[kk], z[i], z[j], z[kk], c->window[0]) &&
                   plane_window_z(y[i], y[j], y[kk], z[i], z[j], z[kk], c->window[1]);
        return plane_fit_z(x[i], x[j], x[kk], z[i], z[j], z[kk], c->msd_max[0], ndf) &&
               plane_fit_z(y[i], y[j], y[kk], z[i], z[j], z[kk], c->msd_max[1], ndf);
    }
    if (c->test == OR_TEST_WINDOW)
        return plane_window(x[i], x[j], x[kk], k, c->window[0]) && plane_window(y[i], y[j], y[kk], k, c->window[1]);
    if (c->test == OR_TEST_MSD_BASIS)
        return plane_msd(x[i], x[j], x[kk], k, c->msd_max[0], ndf) &&
               plane_msd(y[i], y[j], y[kk], k, c->msd_max[1], ndf);
    return plane_fit(x[i], x[j], x[kk], k, c->msd_max[0], ndf) && plane_fit(y[i], y[j], y[kk], k, c->msd_max[1], ndf);
}

static int32_t event_count(const oracle_cfg *c, const oracle_consts *k, const int32_t *off,
                           int64_t e, int32_t n_hits, const float *x, const float *y, const float *z,
                           uint32_t *status) {
    int64_t o0 = off[3 * e], o1 = off[3 * e + 1], o2 = off[3 * e + 2], o3 = off[3 * e + 3];
    if (!(0 <= o0 && o0 <= o1 && o1 <= o2 && o2 <= o3 && o3 <= n_hits)) {
        *status |= 1u;
        return -1;
    }
    int64_t n0 = o1 - o0, n1 = o2 - o1, n2 = o3 - o2;
    /* n0*n1 <= 2^62 fits; compare the full product without forming it */
    if (n2 > 0 && n0 * n1 > (int64_t)INT32_MAX / n2) {
        *status |= 2u;
        return -2;
    }
    int32_t cnt = 0;
    for (int64_t i = o0; i < o1; ++i)
        for (int64_t j = o1; j < o2; ++j)
            for (int64_t kk = o2; kk < o3; ++kk) cnt += triplet_passes(c, k, x, y, z, i, j, kk);
    return cnt;
}

typedef struct {
    const oracle_cfg *cfg;
    const oracle_consts *k;
    const int32_t *off;
    int32_t n_hits;
    const float *x, *y, *z;
    int32_t *counts;
    uint8_t *accept;
    int64_t e0, e1;
    uint32_t status;
} worker_arg;

static void *worker(void *p) {
    worker_arg *a = (worker_arg *)p;
    uint32_t st = 0;
    for (int64_t e = a->e0; e < a->e1; ++e) {
        int32_t cnt = event_count(a->cfg, a->k, a->off, e, a->n_hits, a->x, a->y, a->z, &st);
        a->counts[e] = cnt;
        a->accept[e] = (uint8_t)(cnt >= 0 && cnt >= a->cfg->min_triplets);
    }
    a->status = st;
    return NULL;
}

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* Cost of an event for splitting work between threads (whole events per
 * thread, contiguous ranges of roughly equal triplet count). */
static int64_t event_cost(const int32_t *off, int64_t e) {
    double n0 = (double)off[3 * e + 1] - off[3 * e];
    double n1 = (double)off[3 * e + 2] - off[3 * e + 1];
    double n2 = (double)off[3 * e + 3] - off[3 * e + 2];
    if (n0 < 0 || n1 < 0 || n2 < 0) return 1;
    double c = n0 * n1 * n2;
    return 1 + (c > 1e15 ? (int64_t)1e15 : (int64_t)c);
}

/* Counts and accept flags for events [0, n_events).  Returns the elapsed
 * compute time in seconds (thread start to join), or a negative value on bad
 * arguments.  *status receives the OR of per-event error bits (1 malformed
 * CSR range, 2 triplet count not representable in int32). */
double trig_select_ref_z(int32_t n_events, const int32_t *off, int32_t n_hits, const float *x,
                         const float *y, const float *z, const oracle_cfg *cfg, int32_t *counts,
                         uint8_t *accept, uint32_t *status, int32_t n_threads);

double trig_select_ref(int32_t n_events, const int32_t *off, int32_t n_hits, const float *x,
                       const float *y, const oracle_cfg *cfg, int32_t *counts, uint8_t *accept,
                       uint32_t *status, int32_t n_threads) {
    return trig_select_ref_z(n_events, off, n_hits, x, y, NULL, cfg, counts, accept, status, n_threads);
}

/* trig_select_ref with per-hit z positions (z: n_hits floats, or NULL for
 * the configured layer positions).  The basis-form test is not defined for
 * per-hit z (-1). */
double trig_select_ref_z(int32_t n_events, const int32_t *off, int32_t n_hits, const float *x,
                         const float *y, const float *z, const oracle_cfg *cfg, int32_t *counts,
                         uint8_t *accept, uint32_t *status, int32_t n_threads) {
    if (n_events < 0 || (n_events > 0 && (!off || !counts || !accept)) || !cfg || !status)
        return -1.0;
    if (z && cfg->test == OR_TEST_MSD_BASIS) return -1.0;
    if (n_threads < 1) n_threads = 1;
    oracle_consts k;
    make_consts(cfg, &k);
    double t0 = now_s();
    if (n_threads == 1 || n_events < 2) {
        worker_arg a = {cfg, &k, off, n_hits, x, y, z, counts, accept, 0, n_events, 0};
        worker(&a);
        *status = a.status;
        return now_s() - t0;
    }
    int64_t total = 0;
    for (int64_t e = 0; e < n_events; ++e) total += event_cost(off, e);
    worker_arg *args = (worker_arg *)calloc((size_t)n_threads, sizeof(worker_arg));
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    int64_t e = 0, acc = 0;
    for (int t = 0; t < n_threads; ++t) {
        int64_t target = total * (t + 1) / n_threads;
        int64_t e0 = e;
        while (e < n_events && (acc < target || t == n_threads - 1)) acc += event_cost(off, e++);
        worker_arg a = {cfg, &k, off, n_hits, x, y, z, counts, accept, e0, e, 0};
        args[t] = a;
        pthread_create(&th[t], NULL, worker, &args[t]);
    }
    uint32_t st = 0;
    for (int t = 0; t < n_threads; ++t) {
        pthread_join(th[t], NULL);
        st |= args[t].status;
    }
    double dt = now_s() - t0;
    *status = st;
    free(args);
    free(th);
    return dt;
}

/* The MSD of one triplet in one plane, as the tests above compute it before
 * the threshold comparison (fl(Q / ndf)).  For pin tests. */
float oracle_triplet_msd(const oracle_cfg *cfg, float ci, float cj, float ck) {
    oracle_consts k;
    make_consts(cfg, &k);
    const float ndf = (float)cfg->ndf;
    if (cfg->test == OR_TEST_MSD_BASIS) {
        float a = k.U0 * ci + k.U1 * cj;
        float b = (k.V0 * ci + k.V1 * cj) + k.V2 * ck;
        return (a * a + b * b) / ndf;
    }
    float p0 = ci * k.zf[0], p1 = cj * k.zf[1], p2 = ck * k.zf[2];
    float m = ((p0 + p1) + p2) * k.w;
    float r0 = ci - m * k.zf[0], r1 = cj - m * k.zf[1], r2 = ck - m * k.zf[2];
    return ((r0 * r0 + r1 * r1) + r2 * r2) / ndf;
}

/* The fp32 basis constants (U0, U1, V0, V1, V2), for pin tests. */
void oracle_basis(const oracle_cfg *cfg, float out[5]) {
    oracle_consts k;
    make_consts(cfg, &k);
    out[0] = k.U0; out[1] = k.U1; out[2] = k.V0; out[3] = k.V1; out[4] = k.V2;
}

/* Triplets whose decision differs between the MSD and MSD_BASIS evaluations
 * of the same fit (both planes; cfg->test is ignored), for events
 * [e0, e1).  per_event[e - e0] (may be NULL) receives each event's number;
 * malformed events and events whose triplet count int32 cannot hold count 0.
 * Returns the total, or -1 on bad arguments.  One thread; callers split the
 * event range. */
int64_t trig_ref_msd_disagreements(int64_t e0, int64_t e1, const int32_t *off, int32_t n_hits,
                                   const float *x, const float *y, const oracle_cfg *cfg,
                                   int32_t *per_event) {
    if (e0 < 0 || e1 < e0 || (e1 > e0 && !off) || !cfg) return -1;
    oracle_consts k;
    make_consts(cfg, &k);
    const float ndf = (float)cfg->ndf;
    int64_t total = 0;
    for (int64_t e = e0; e < e1; ++e) {
        int64_t o0 = off[3 * e], o1 = off[3 * e + 1], o2 = off[3 * e + 2], o3 = off[3 * e + 3];
        int32_t d = 0;
        int ok = 0 <= o0 && o0 <= o1 && o1 <= o2 && o2 <= o3 && o3 <= n_hits;
        if (ok && (o3 - o2) > 0 && (o1 - o0) * (o2 - o1) > (int64_t)INT32_MAX / (o3 - o2)) ok = 0;
        if (ok)
            for (int64_t i = o0; i < o1; ++i)
                for (int64_t j = o1; j < o2; ++j)
                    for (int64_t kk = o2; kk < o3; ++kk) {
                        int fit = plane_fit(x[i], x[j], x[kk], &k, cfg->msd_max[0], ndf) &&
                                  plane_fit(y[i], y[j], y[kk], &k, cfg->msd_max[1], ndf);
                        int basis = plane_msd(x[i], x[j], x[kk], &k, cfg->msd_max[0], ndf) &&
                                    plane_msd(y[i], y[j], y[kk], &k, cfg->msd_max[1], ndf);
                        d += fit != basis;
                    }
        if (per_event) per_event[e - e0] = d;
        total += d;
    }
    return total;
}

/* Whether triplets t and u (hit indices i, j, k in layers 0, 1, 2) have no
 * hit in common. */
static int no_common_hit(const int64_t *t, const int64_t *u) {
    return t[0] != u[0] && t[1] != u[1] && t[2] != u[2];
}

/* 1 if the list of n triplets (3 hit indices each) holds two with no hit in
 * common, else 0: every pair is compared.  For pin tests as well. */
int32_t oracle_has_disjoint_pair(int64_t n, const int64_t *trip) {
    for (int64_t a = 0; a < n; ++a)
        for (int64_t b = a + 1; b < n; ++b)
            if (no_common_hit(trip + 3 * a, trip + 3 * b)) return 1;
    return 0;
}

/* Two-particle acceptance (the trigger signature of Sec. 3.1: two particles
 * in the trigger station pointing back to the target): for events [e0, e1),
 * out[e - e0] = 1 if the event's passing triplets (the test of cfg, as in
 * trig_select_ref) include two with no hit in common, else 0; malformed
 * events and events whose triplet count int32 cannot hold get 0.  The
 * passing triplets are listed, then every pair of them compared.  Returns
 * the number of accepted events, or -1 on bad arguments or memory.  One
 * thread; callers split the event range. */
int64_t trig_ref_disjoint(int64_t e0, int64_t e1, const int32_t *off, int32_t n_hits, const float *x,
                          const float *y, const float *z, const oracle_cfg *cfg, uint8_t *out) {
    if (e0 < 0 || e1 < e0 || (e1 > e0 && (!off || !out)) || !cfg) return -1;
    if (z && cfg->test == OR_TEST_MSD_BASIS) return -1;
    oracle_consts k;
    make_consts(cfg, &k);
    int64_t cap = 0, accepted = 0;
    int64_t *trip = NULL;
    for (int64_t e = e0; e < e1; ++e) {
        int64_t o0 = off[3 * e], o1 = off[3 * e + 1], o2 = off[3 * e + 2], o3 = off[3 * e + 3];
        int ok = 0 <= o0 && o0 <= o1 && o1 <= o2 && o2 <= o3 && o3 <= n_hits;
        if (ok && (o3 - o2) > 0 && (o1 - o0) * (o2 - o1) > (int64_t)INT32_MAX / (o3 - o2)) ok = 0;
        int64_t n = 0;
        if (ok)
            for (int64_t i = o0; i < o1; ++i)
                for (int64_t j = o1; j < o2; ++j)
                    for (int64_t kk = o2; kk < o3; ++kk) {
                        if (!triplet_passes(cfg, &k, x, y, z, i, j, kk)) continue;
                        if (n == cap) {
                            cap = cap ? 2 * cap : 64;
                            int64_t *grown = (int64_t *)realloc(trip, (size_t)cap * 3 * sizeof(int64_t));
                            if (!grown) {
                                free(trip);
                                return -1;
                            }
                            trip = grown;
                        }
                        trip[3 * n] = i;
                        trip[3 * n + 1] = j;
                        trip[3 * n + 2] = kk;
                        ++n;
                    }
        out[e - e0] = (uint8_t)oracle_has_disjoint_pair(n, trip);
        accepted += out[e - e0];
    }
    free(trip);
    return accepted;
}
