/*
 * FP64 reference ("oracle") for cascaded biquad filtering.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path links, loads or calls
 * this file; it exists so that tests, the smoke check and the benchmark's CPU
 * baseline can compare the HIP kernels against a plain, slow, sequential
 * definition. It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (Zhai & Paris, Part II, Sec. II-A, Eq. (1)):
 *   a cascade of K second-order sections; the output of section k is the input
 *   of section k+1. Each section is evaluated sample by sample in transposed
 *   direct form II, in double precision, with all six coefficients
 *   [b0 b1 b2 a0 a1 a2] divided by a0 first:
 *       y    = b0*u + z1
 *       z1'  = b1*u - a1*y + z2
 *       z2'  = b2*u - a2*y
 *   zi/zf are the K x 2 TDF-II states (z1, z2) before the first and after the
 *   last sample. The multi-block system of Sec. II-B (Eqs. (2)-(3)) is an exact
 *   reformulation of this recurrence, so the parallel method must reproduce
 *   this result up to rounding.
 *
 * The gradient routine is the reverse-mode sweep of exactly this program
 * (the adjoint of each TDF-II step taken in reverse sample order, sections in
 * reverse order), plus the chain rule through the division by a0. The paper
 * does not treat gradients; this is the plain definition of the derivative of
 * the forward program above.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

/* One section over n samples; in may equal out. state[2] is read as zi and
 * written back as zf. c = normalized {b0, b1, b2, a1, a2}. */
static void tdf2_section(const double c[5], const double *in, double *out,
                         int64_t n, double state[2])
{
    const double b0 = c[0], b1 = c[1], b2 = c[2], a1 = c[3], a2 = c[4];
    double z1 = state[0], z2 = state[1];
    for (int64_t t = 0; t < n; ++t) {
        const double u = in[t];
        const double y = b0 * u + z1;
        z1 = b1 * u - a1 * y + z2;
        z2 = b2 * u - a2 * y;
        out[t] = y;
    }
    state[0] = z1;
    state[1] = z2;
}

static int normalize(const double row[6], double c[5])
{
    const double a0 = row[3];
    if (a0 == 0.0) return -2;
    c[0] = row[0] / a0;
    c[1] = row[1] / a0;
    c[2] = row[2] / a0;
    c[3] = row[4] / a0;
    c[4] = row[5] / a0;
    return 0;
}

/* sos: K x 6 rows [b0 b1 b2 a0 a1 a2]; zi, zf: K x 2 (zi may be NULL = zeros,
 * zf may be NULL). x and y may alias. Returns 0, or -2 if some a0 == 0. */
int oracle_sosfilt(const double *sos, int K, const double *x, int64_t n,
                   const double *zi, double *y, double *zf)
{
    if (K < 0 || n < 0) return -1;
    if (y != x && n > 0) memmove(y, x, (size_t)n * sizeof(double));
    for (int k = 0; k < K; ++k) {
        double c[5];
        if (normalize(sos + 6 * k, c)) return -2;
        double st[2] = {zi ? zi[2 * k] : 0.0, zi ? zi[2 * k + 1] : 0.0};
        tdf2_section(c, y, y, n, st);
        if (zf) { zf[2 * k] = st[0]; zf[2 * k + 1] = st[1]; }
    }
    return 0;
}

/*
 * Vector-Jacobian product of oracle_sosfilt.
 *   gy  : n, upstream gradient of y
 *   gzf : K x 2 upstream gradient of zf (NULL = zeros)
 * outputs
 *   gx  : n       d<gy,y>+<gzf,zf> / dx
 *   gzi : K x 2   ... / dzi          (may be NULL)
 *   gsos: K x 6   ... / d[b0 b1 b2 a0 a1 a2] (raw, un-normalized rows; may be NULL)
 * gx may alias gy. Needs O(K n) doubles of scratch for the section inputs.
 */
int oracle_sosfilt_vjp(const double *sos, int K, const double *x, int64_t n,
                       const double *zi, const double *gy, const double *gzf,
                       double *gx, double *gzi, double *gsos)
{
    if (K < 0 || n < 0) return -1;
    double *c = (double *)malloc(sizeof(double) * 5 * (K > 0 ? K : 1));
    /* acts[k] = input of section k, acts[K] = final output */
    double *acts = (double *)malloc(sizeof(double) * (size_t)(K + 1) * (size_t)(n > 0 ? n : 1));
    if (!c || !acts) { free(c); free(acts); return -4; }
    for (int k = 0; k < K; ++k)
        if (normalize(sos + 6 * k, c + 5 * k)) { free(c); free(acts); return -2; }

    if (n > 0) memcpy(acts, x, (size_t)n * sizeof(double));
    for (int k = 0; k < K; ++k) {
        double st[2] = {zi ? zi[2 * k] : 0.0, zi ? zi[2 * k + 1] : 0.0};
        tdf2_section(c + 5 * k, acts + (size_t)k * n, acts + (size_t)(k + 1) * n, n, st);
    }

    if (gx != gy && n > 0) memmove(gx, gy, (size_t)n * sizeof(double));
    for (int k = K - 1; k >= 0; --k) {
        const double *ck = c + 5 * k;
        const double b0 = ck[0], b1 = ck[1], b2 = ck[2], a1 = ck[3], a2 = ck[4];
        const double *u = acts + (size_t)k * n;        /* section input  */
        const double *v = acts + (size_t)(k + 1) * n;  /* section output */
        /* adjoints of the state after the current step */
        double g1 = gzf ? gzf[2 * k] : 0.0, g2 = gzf ? gzf[2 * k + 1] : 0.0;
        double gb0 = 0, gb1 = 0, gb2 = 0, ga1 = 0, ga2 = 0;
        for (int64_t t = n - 1; t >= 0; --t) {
            /* forward step: y = b0 u + z1p; z1n = b1 u - a1 y + z2p; z2n = b2 u - a2 y */
            const double gyt = gx[t] - a1 * g1 - a2 * g2;   /* total adjoint of y */
            const double gu = b0 * gyt + b1 * g1 + b2 * g2;
            gb0 += gyt * u[t];
            gb1 += g1 * u[t];
            gb2 += g2 * u[t];
            ga1 -= g1 * v[t];
            ga2 -= g2 * v[t];
            const double g1p = gyt;  /* adjoint of z1 before the step */
            const double g2p = g1;   /* adjoint of z2 before the step */
            g1 = g1p;
            g2 = g2p;
            gx[t] = gu;
        }
        if (gzi) { gzi[2 * k] = g1; gzi[2 * k + 1] = g2; }
        if (gsos) {
            const double a0 = sos[6 * k + 3];
            double *gs = gsos + 6 * k;
            gs[0] = gb0 / a0;
            gs[1] = gb1 / a0;
            gs[2] = gb2 / a0;
            gs[4] = ga1 / a0;
            gs[5] = ga2 / a0;
            gs[3] = -(gb0 * b0 + gb1 * b1 + gb2 * b2 + ga1 * a1 + ga2 * a2) / a0;
        }
    }
    free(c);
    free(acts);
    return 0;
}

/* ---- independent signals on a pool of host threads (CPU baseline) ---- */

typedef struct {
    int B;
    const int32_t *K;
    const int64_t *sec_off;   /* B+1, section row offsets */
    const double *sos;
    const int64_t *sig_off;   /* B+1, sample offsets */
    const double *x;
    double *y;
    const double *zi;         /* 2 * sec_off[B] or NULL */
    double *zf;               /* 2 * sec_off[B] or NULL */
    int nthreads;
    int tid;
    int rc;
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *j = (batch_job *)arg;
    for (int i = j->tid; i < j->B; i += j->nthreads) {
        const int64_t so = j->sec_off[i];
        const int64_t a = j->sig_off[i], b = j->sig_off[i + 1];
        int rc = oracle_sosfilt(j->sos + 6 * so, j->K[i], j->x + a, b - a,
                                j->zi ? j->zi + 2 * so : NULL, j->y + a,
                                j->zf ? j->zf + 2 * so : NULL);
        if (rc) j->rc = rc;
    }
    return NULL;
}

int oracle_sosfilt_batched(int B, const int32_t *K, const int64_t *sec_off,
                           const double *sos, const int64_t *sig_off,
                           const double *x, double *y, const double *zi,
                           double *zf, int nthreads)
{
    if (B < 0) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    batch_job jobs[256];
    pthread_t th[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (batch_job){B, K, sec_off, sos, sig_off, x, y, zi, zf, nthreads, t, 0};
        if (t > 0) pthread_create(&th[t], NULL, batch_worker, &jobs[t]);
    }
    batch_worker(&jobs[0]);
    int rc = jobs[0].rc;
    for (int t = 1; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        if (jobs[t].rc) rc = jobs[t].rc;
    }
    return rc;
}
