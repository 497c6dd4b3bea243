/*
 * Multi-core CPU comparator: the wavefront execution of a cascade of
 * second-order sections over signal block groups (Zhai & Paris Part II,
 * Sec. III-A, Fig. "wavefront").
 *
 * The signal is cut into consecutive groups of C samples. Every group is
 * followed through all K sections by one thread (groups are dealt to the
 * threads round robin). Node (g, s), section s applied to group g, needs the
 * section's state after group g-1 (handed along by the thread that ran
 * (g-1, s)) and the group's own output of section s-1 (produced just before
 * by the same thread). Within a section the groups therefore run strictly in
 * order, each from a known initial state, so the per-node work is the plain
 * serial filter; up to K nodes (one per section) run at the same time, on
 * different groups, and FIFO order is kept. Threads take the next group from
 * a shared counter, so groups start in order whatever the number of threads
 * that actually run (the calling thread is one of them).
 *
 * Per node, either the plain serial filter (transposed direct form II in
 * FP32, the precision of the data, sections normalised by a0), or the
 * multi-block node kernel of the paper's single-core function (Sec. III,
 * built on the multi-block system of Sec. II-B and PH of Sec. II-C): the
 * thread transposes its group once into blocks of LANES lanes x NB samples
 * (lane i of a block holds the block's samples i NB .. i NB + NB - 1, so a
 * vector holds one sample position of every lane), runs every section on
 * that layout with 8-wide vector arithmetic, and transposes back after the
 * last section. Per block and section: the lanes' particular solutions from
 * rest (transposed direct form II, all lanes at once), the lanes' incoming
 * states by a scan over the lanes through T^NB (FP64), and the homogeneous
 * correction g[m] s1 + g[m - 1] s2 of every sample (g the impulse response of
 * 1/A). A group's last len % (LANES NB) samples run through the serial filter.
 * Not used by the library or its tests' expected values; it is a reported
 * CPU rate beside the GPU one.
 */
#include <pthread.h>
#include <sched.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    float b0, b1, b2, a1, a2;
} coef_t;

/* multi-block node: 8-wide vectors, LANES lanes per block in VPB vectors
 * (four independent recursions interleaved per sample position: one
 * recursion's two dependent FMAs per step would otherwise leave the FMA
 * pipes idle; 4 measured 2x faster than 1 at order 16, one thread) */
typedef float v8 __attribute__((vector_size(32)));
enum { VW = 8, VPB = 4, LANES = VW * VPB, NB = 64, BLK = LANES * NB };

typedef struct {
    float b0, b1, b2, a1, a2;
    double tn[4];           /* T^NB, T = [[-a1, 1], [-a2, 0]] on TDF-II states */
    float g[NB + 1];        /* g[-1] = 0, then g[0..NB-1] */
} mbcoef_t;

typedef struct {
    const coef_t *c;
    const mbcoef_t *mc;      /* non-NULL: multi-block node kernels */
    int K;
    const float *x;
    float *y;
    int64_t n, C, G;
    int T;
    float *state;            /* K x 2: each section's state after the last group it ran */
    atomic_int_least64_t *done;   /* K: groups finished per section */
    atomic_int_least64_t next;    /* next group to start */
} wf_t;

static void run_node(const coef_t *c, const float *in, float *out, int64_t len, float *z)
{
    float z1 = z[0], z2 = z[1];
    for (int64_t i = 0; i < len; ++i) {
        const float v = in[i];
        const float y = c->b0 * v + z1;
        z1 = c->b1 * v - c->a1 * y + z2;
        z2 = c->b2 * v - c->a2 * y;
        out[i] = y;
    }
    z[0] = z1;
    z[1] = z2;
}

/* The block at X (NB vectors of each of the VPB lane sets, position-major:
 * X[m * VPB + v] holds sample m of lanes v VW .. v VW + VW - 1) through one
 * section from the block's incoming TDF-II state z, which becomes the state
 * after the block. */
static void mb_block(const mbcoef_t *c, v8 *X, float *z)
{
    const v8 b0 = {c->b0, c->b0, c->b0, c->b0, c->b0, c->b0, c->b0, c->b0};
    const v8 b1 = b0 * 0.0f + c->b1, b2 = b0 * 0.0f + c->b2;
    const v8 a1 = b0 * 0.0f + c->a1, a2 = b0 * 0.0f + c->a2;
    v8 z1[VPB], z2[VPB];
    for (int v = 0; v < VPB; ++v) z1[v] = z2[v] = b0 * 0.0f;
    /* particular solutions: every lane from rest, the VPB lane sets
     * interleaved (independent chains) */
    for (int m = 0; m < NB; ++m)
        for (int v = 0; v < VPB; ++v) {
            const v8 x = X[m * VPB + v];
            const v8 y = b0 * x + z1[v];
            z1[v] = b1 * x - a1 * y + z2[v];
            z2[v] = b2 * x - a2 * y;
            X[m * VPB + v] = y;
        }
    /* incoming state of every lane: scan over the lanes in FP64 */
    float s1f[LANES], s2f[LANES];
    double s1 = z[0], s2 = z[1];
    for (int l = 0; l < LANES; ++l) {
        s1f[l] = (float)s1;
        s2f[l] = (float)s2;
        const double t1 = z1[l / VW][l % VW], t2 = z2[l / VW][l % VW];
        const double n1 = c->tn[0] * s1 + c->tn[1] * s2 + t1;
        const double n2 = c->tn[2] * s1 + c->tn[3] * s2 + t2;
        s1 = n1;
        s2 = n2;
    }
    z[0] = (float)s1;
    z[1] = (float)s2;
    /* homogeneous correction */
    v8 S1[VPB], S2[VPB];
    for (int v = 0; v < VPB; ++v)
        for (int j = 0; j < VW; ++j) {
            S1[v][j] = s1f[v * VW + j];
            S2[v][j] = s2f[v * VW + j];
        }
    for (int m = 0; m < NB; ++m) {
        const float g0 = c->g[m + 1], gm = c->g[m];
        for (int v = 0; v < VPB; ++v) X[m * VPB + v] += g0 * S1[v] + gm * S2[v];
    }
}

/* natural order <-> blocks: in[b BLK + l NB + m] <-> X[b][m VPB + l / VW][l % VW] */
static void to_blocks(const float *in, v8 *X, int64_t nb)
{
    for (int64_t b = 0; b < nb; ++b) {
        const float *src = in + b * BLK;
        float *dst = (float *)(X + b * NB * VPB);
        for (int l = 0; l < LANES; ++l)
            for (int m = 0; m < NB; ++m) dst[(m * VPB + l / VW) * VW + l % VW] = src[l * NB + m];
    }
}

static void from_blocks(const v8 *X, float *out, int64_t nb)
{
    for (int64_t b = 0; b < nb; ++b) {
        const float *src = (const float *)(X + b * NB * VPB);
        float *dst = out + b * BLK;
        for (int l = 0; l < LANES; ++l)
            for (int m = 0; m < NB; ++m) dst[l * NB + m] = src[(m * VPB + l / VW) * VW + l % VW];
    }
}

/* Group g through all K sections with the multi-block node kernels: ws holds
 * the group's full blocks (transposed) and then its tail (natural order). */
static void run_group_mb(wf_t *w, int64_t g, v8 *ws)
{
    const int64_t off = g * w->C;
    const int64_t len = (w->n - off < w->C) ? w->n - off : w->C;
    const int64_t nb = len / BLK, tail = len - nb * BLK;
    float *wt = (float *)(ws + nb * NB * VPB);
    to_blocks(w->x + off, ws, nb);
    memcpy(wt, w->x + off + nb * BLK, sizeof(float) * (size_t)tail);
    for (int s = 0; s < w->K; ++s) {
        while (atomic_load_explicit(&w->done[s], memory_order_acquire) < g) sched_yield();
        float *z = w->state + 2 * s;
        for (int64_t b = 0; b < nb; ++b) mb_block(&w->mc[s], ws + b * NB * VPB, z);
        run_node(&w->c[s], wt, wt, tail, z);
        atomic_store_explicit(&w->done[s], g + 1, memory_order_release);
    }
    from_blocks(ws, w->y + off, nb);
    memcpy(w->y + off + nb * BLK, wt, sizeof(float) * (size_t)tail);
}

static void *worker(void *p)
{
    wf_t *w = (wf_t *)p;
    v8 *ws = NULL;
    if (w->mc) {
        /* the group's blocks, then its tail (< BLK samples); a thread that
         * cannot get its workspace takes no group */
        const size_t bytes = sizeof(float) * (size_t)(w->C + BLK);
        ws = (v8 *)aligned_alloc(32, (bytes + 31) / 32 * 32);
        if (!ws) return NULL;
    }
    for (;;) {
        const int64_t g = atomic_fetch_add_explicit(&w->next, 1, memory_order_relaxed);
        if (g >= w->G) break;
        if (w->mc) {
            run_group_mb(w, g, ws);
            continue;
        }
        const int64_t off = g * w->C;
        const int64_t len = (w->n - off < w->C) ? w->n - off : w->C;
        for (int s = 0; s < w->K; ++s) {
            /* wait for the state this section left after group g-1 */
            while (atomic_load_explicit(&w->done[s], memory_order_acquire) < g) sched_yield();
            run_node(&w->c[s], s == 0 ? w->x + off : w->y + off, w->y + off, len,
                     w->state + 2 * s);
            atomic_store_explicit(&w->done[s], g + 1, memory_order_release);
        }
    }
    free(ws);
    return NULL;
}

/* sections: K x 6 rows [b0 b1 b2 a0 a1 a2]; zi, zf: K x 2 TDF-II states (zi
 * may be NULL: zeros; zf may be NULL). group: samples per group (> 0);
 * threads: threads to use, the caller's included (> 0). y may equal x.
 * node: 0 the serial filter per node, 1 the multi-block node kernels.
 * Returns 0, -1 for invalid arguments (a0 == 0 included) or -2 when out of
 * memory. */
int sos_wavefront_nodes(const float *sections, int K, const float *x, float *y, int64_t n,
                        const float *zi, float *zf, int64_t group, int threads, int node)
{
    if (K < 0 || n < 0 || group <= 0 || threads <= 0 || (n > 0 && (!x || !y)) ||
        (K > 0 && !sections) || (node != 0 && node != 1))
        return -1;
    coef_t *c = (coef_t *)malloc(sizeof(coef_t) * (size_t)(K > 0 ? K : 1));
    mbcoef_t *mc = node ? (mbcoef_t *)malloc(sizeof(mbcoef_t) * (size_t)(K > 0 ? K : 1)) : NULL;
    float *state = (float *)calloc((size_t)(K > 0 ? 2 * K : 2), sizeof(float));
    atomic_int_least64_t *done =
        (atomic_int_least64_t *)malloc(sizeof(atomic_int_least64_t) * (size_t)(K > 0 ? K : 1));
    if (!c || !state || !done || (node && !mc)) {
        free(c);
        free(mc);
        free(state);
        free(done);
        return -2;
    }
    int rc = 0;
    for (int s = 0; s < K; ++s) {
        const float *r = sections + 6 * s;
        if (r[3] == 0.0f) rc = -1;
        const double inv = r[3] == 0.0f ? 0.0 : 1.0 / (double)r[3];
        c[s].b0 = (float)(r[0] * inv);
        c[s].b1 = (float)(r[1] * inv);
        c[s].b2 = (float)(r[2] * inv);
        c[s].a1 = (float)(r[4] * inv);
        c[s].a2 = (float)(r[5] * inv);
        if (mc) {
            const double a1 = r[4] * inv, a2 = r[5] * inv;
            mc[s].b0 = c[s].b0;
            mc[s].b1 = c[s].b1;
            mc[s].b2 = c[s].b2;
            mc[s].a1 = c[s].a1;
            mc[s].a2 = c[s].a2;
            /* T^NB by squaring (NB a power of two) */
            double t[4] = {-a1, 1.0, -a2, 0.0};
            for (int k = 1; k < NB; k *= 2) {
                const double u[4] = {t[0] * t[0] + t[1] * t[2], t[0] * t[1] + t[1] * t[3],
                                     t[2] * t[0] + t[3] * t[2], t[2] * t[1] + t[3] * t[3]};
                memcpy(t, u, sizeof t);
            }
            memcpy(mc[s].tn, t, sizeof t);
            /* impulse response of 1/A(z) */
            double gm2 = 0.0, gm1 = 0.0;
            mc[s].g[0] = 0.0f;
            for (int m = 0; m < NB; ++m) {
                const double gv = m == 0 ? 1.0 : -a1 * gm1 - a2 * gm2;
                mc[s].g[m + 1] = (float)gv;
                gm2 = gm1;
                gm1 = gv;
            }
        }
        if (zi) {
            state[2 * s] = zi[2 * s];
            state[2 * s + 1] = zi[2 * s + 1];
        }
        atomic_init(&done[s], 0);
    }
    if (rc == 0 && n > 0) {
        if (K == 0) {
            if (y != x) memmove(y, x, sizeof(float) * (size_t)n);
        } else {
            wf_t w = {c, mc, K, x, y, n, group, (n + group - 1) / group, threads, state, done, 0};
            atomic_init(&w.next, 0);
            if (w.T > w.G) w.T = (int)w.G;
            /* T - 1 helpers plus the calling thread; a helper that cannot be
             * started only lowers the parallelism */
            pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)w.T);
            int started = 0;
            for (int t = 1; th && t < w.T; ++t)
                if (pthread_create(&th[started], NULL, worker, &w) == 0) ++started;
            worker(&w);
            for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
            free(th);
            /* no thread could get a workspace: no group ran */
            if (atomic_load(&w.next) < w.G) rc = -2;
        }
    }
    if (rc == 0 && zf)
        for (int s = 0; s < 2 * K; ++s) zf[s] = state[s];
    free(c);
    free(mc);
    free(state);
    free(done);
    return rc;
}

int sos_wavefront(const float *sections, int K, const float *x, float *y, int64_t n,
                  const float *zi, float *zf, int64_t group, int threads)
{
    return sos_wavefront_nodes(sections, K, x, y, n, zi, zf, group, threads, 0);
}
