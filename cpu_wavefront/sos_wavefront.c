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
 * Per node: transposed direct form II in FP32 (the precision of the data),
 * sections normalised by a0. Not used by the library or its tests' expected
 * values; it is a reported CPU rate beside the GPU one.
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

typedef struct {
    const coef_t *c;
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

static void *worker(void *p)
{
    wf_t *w = (wf_t *)p;
    for (;;) {
        const int64_t g = atomic_fetch_add_explicit(&w->next, 1, memory_order_relaxed);
        if (g >= w->G) break;
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
    return NULL;
}

/* sections: K x 6 rows [b0 b1 b2 a0 a1 a2]; zi, zf: K x 2 TDF-II states (zi
 * may be NULL: zeros; zf may be NULL). group: samples per group (> 0);
 * threads: threads to use, the caller's included (> 0). y may equal x.
 * Returns 0, -1 for invalid arguments (a0 == 0 included) or -2 when out of
 * memory. */
int sos_wavefront(const float *sections, int K, const float *x, float *y, int64_t n,
                  const float *zi, float *zf, int64_t group, int threads)
{
    if (K < 0 || n < 0 || group <= 0 || threads <= 0 || (n > 0 && (!x || !y)) ||
        (K > 0 && !sections))
        return -1;
    coef_t *c = (coef_t *)malloc(sizeof(coef_t) * (size_t)(K > 0 ? K : 1));
    float *state = (float *)calloc((size_t)(K > 0 ? 2 * K : 2), sizeof(float));
    atomic_int_least64_t *done =
        (atomic_int_least64_t *)malloc(sizeof(atomic_int_least64_t) * (size_t)(K > 0 ? K : 1));
    if (!c || !state || !done) {
        free(c);
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
            wf_t w = {c, K, x, y, n, group, (n + group - 1) / group, threads, state, done, 0};
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
        }
    }
    if (rc == 0 && zf)
        for (int s = 0; s < 2 * K; ++s) zf[s] = state[s];
    free(c);
    free(state);
    free(done);
    return rc;
}
