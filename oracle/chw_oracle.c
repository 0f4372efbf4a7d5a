/*
 * chw_oracle.c -- plain C statement of the Cascading Haar Wavelet cascade.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the C twin of oracle/cascade.py
 * (same algorithm, same order of operations), used where Python is too slow:
 * large parity samples and the CPU-baseline timing.  It shares no source,
 * header, table or helper with the GPU library and is never linked into it.
 *
 * Arithmetic: double with a 1/sqrt(2) per Haar level (orthonormal form of
 * eqs. 1-2), or int64 with every 1/sqrt(2) dropped (unnormalized form).
 *
 * The cascade (Sec. 2, Theorem 1 / eq. 3):
 *   1. Psi_m on the whole vector (eq. 2 read as an algorithm: levels on a
 *      shrinking block of sums, details to the upper half);
 *   2. for r = 1 .. m-1, factor F_r = I_{r-1} (x) diag(I_{m-r}, Psi_{m-r}):
 *      Psi_{m-r} on the second half of each of the 2^{r-1} blocks of
 *      2^{m-r+1}; the identity halves are not performed.
 * The adjoint applies the transposed factors in reverse order (F_{m-1}^T
 * first, Psi_m^T last), each Psi^T being the Haar synthesis.
 *
 * Batch entry points take per-signal log2 sizes and int64 element offsets,
 * and spread signals over `threads` POSIX threads (one signal per task).
 */
#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_SQRT1_2 0.70710678118654752440

/* ---- Haar building blocks ------------------------------------------------ */

/* Psi_k on v[0 .. len), double; tmp holds len/2 scratch values. */
static void haar_fwd_f64(double *v, int64_t len, double *tmp)
{
    const double c = ORC_SQRT1_2;
    while (len >= 2) {
        int64_t half = len / 2;
        for (int64_t p = 0; p < half; ++p) {
            double a = v[2 * p], b = v[2 * p + 1];
            v[p] = c * (a + b);          /* safe: p <= 2p, already read */
            tmp[p] = c * (a - b);
        }
        memcpy(v + half, tmp, (size_t)half * sizeof(double));
        len = half;
    }
}

/* Psi_k^T on v[0 .. len), double (synthesis, coarse to fine). */
static void haar_adj_f64(double *v, int64_t len, double *tmp)
{
    const double c = ORC_SQRT1_2;
    for (int64_t h = 1; h < len; h *= 2) {
        for (int64_t p = 0; p < h; ++p) {
            double a = v[p], d = v[h + p];
            tmp[2 * p] = c * (a + d);
            tmp[2 * p + 1] = c * (a - d);
        }
        memcpy(v, tmp, (size_t)(2 * h) * sizeof(double));
    }
}

static void haar_fwd_i64(int64_t *v, int64_t len, int64_t *tmp)
{
    while (len >= 2) {
        int64_t half = len / 2;
        for (int64_t p = 0; p < half; ++p) {
            int64_t a = v[2 * p], b = v[2 * p + 1];
            v[p] = a + b;
            tmp[p] = a - b;
        }
        memcpy(v + half, tmp, (size_t)half * sizeof(int64_t));
        len = half;
    }
}

static void haar_adj_i64(int64_t *v, int64_t len, int64_t *tmp)
{
    for (int64_t h = 1; h < len; h *= 2) {
        for (int64_t p = 0; p < h; ++p) {
            int64_t a = v[p], d = v[h + p];
            tmp[2 * p] = a + d;
            tmp[2 * p + 1] = a - d;
        }
        memcpy(v, tmp, (size_t)(2 * h) * sizeof(int64_t));
    }
}

/* ---- one signal ------------------------------------------------------------ */

static void chw_one_f64(double *v, int m, double *tmp, int adjoint)
{
    int64_t n = (int64_t)1 << m;
    if (!adjoint) {
        haar_fwd_f64(v, n, tmp);                       /* Psi_m */
        for (int r = 1; r < m; ++r) {                  /* F_1 .. F_{m-1} */
            int64_t big = (int64_t)1 << (m - r + 1);
            for (int64_t b = 0; b < ((int64_t)1 << (r - 1)); ++b)
                haar_fwd_f64(v + b * big + big / 2, big / 2, tmp);
        }
    } else {
        for (int r = m - 1; r >= 1; --r) {             /* F_{m-1}^T .. F_1^T */
            int64_t big = (int64_t)1 << (m - r + 1);
            for (int64_t b = ((int64_t)1 << (r - 1)) - 1; b >= 0; --b)
                haar_adj_f64(v + b * big + big / 2, big / 2, tmp);
        }
        if (m >= 1) haar_adj_f64(v, n, tmp);           /* Psi_m^T */
    }
}

static void chw_one_i64(int64_t *v, int m, int64_t *tmp, int adjoint)
{
    int64_t n = (int64_t)1 << m;
    if (!adjoint) {
        haar_fwd_i64(v, n, tmp);
        for (int r = 1; r < m; ++r) {
            int64_t big = (int64_t)1 << (m - r + 1);
            for (int64_t b = 0; b < ((int64_t)1 << (r - 1)); ++b)
                haar_fwd_i64(v + b * big + big / 2, big / 2, tmp);
        }
    } else {
        for (int r = m - 1; r >= 1; --r) {
            int64_t big = (int64_t)1 << (m - r + 1);
            for (int64_t b = ((int64_t)1 << (r - 1)) - 1; b >= 0; --b)
                haar_adj_i64(v + b * big + big / 2, big / 2, tmp);
        }
        if (m >= 1) haar_adj_i64(v, n, tmp);
    }
}

/* ---- batches over threads ---------------------------------------------------- */

typedef struct {
    const void *x;
    void *y;
    const int32_t *log2_sizes;
    const int64_t *offsets;
    int64_t batch;
    int is_int;
    int adjoint;
    atomic_llong next;
    int status;
} orc_job;

static void *orc_worker(void *arg)
{
    orc_job *job = (orc_job *)arg;
    int maxm = 0;
    for (int64_t i = 0; i < job->batch; ++i)
        if (job->log2_sizes[i] > maxm) maxm = job->log2_sizes[i];
    size_t tmp_bytes = ((size_t)1 << maxm) * 8u;
    void *tmp = malloc(tmp_bytes > 8 ? tmp_bytes : 8);
    if (!tmp) { job->status = -2; return NULL; }
    for (;;) {
        long long i = atomic_fetch_add(&job->next, 1);
        if (i >= job->batch) break;
        int m = job->log2_sizes[i];
        int64_t n = (int64_t)1 << m, off = job->offsets[i];
        if (job->is_int) {
            const int64_t *src = (const int64_t *)job->x + off;
            int64_t *dst = (int64_t *)job->y + off;
            if (dst != src) memcpy(dst, src, (size_t)n * sizeof(int64_t));
            chw_one_i64(dst, m, (int64_t *)tmp, job->adjoint);
        } else {
            const double *src = (const double *)job->x + off;
            double *dst = (double *)job->y + off;
            if (dst != src) memcpy(dst, src, (size_t)n * sizeof(double));
            chw_one_f64(dst, m, (double *)tmp, job->adjoint);
        }
    }
    free(tmp);
    return NULL;
}

static int orc_run(orc_job *job, int threads)
{
    for (int64_t i = 0; i < job->batch; ++i)
        if (job->log2_sizes[i] < 0 || job->log2_sizes[i] > 30) return -1;
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    if ((int64_t)threads > job->batch) threads = job->batch > 0 ? (int)job->batch : 1;
    atomic_init(&job->next, 0);
    job->status = 0;
    if (threads == 1) {
        orc_worker(job);
        return job->status;
    }
    pthread_t tid[256];
    int started = 0;
    for (int t = 0; t < threads; ++t) {
        if (pthread_create(&tid[t], NULL, orc_worker, job) != 0) break;
        ++started;
    }
    if (started == 0) orc_worker(job);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    return job->status;
}

/* x, y: arrays of double (or int64) addressed by element offsets; y may equal x.
 * Returns 0, or -1 for a bad size, -2 when scratch memory cannot be had. */
int orc_chw_batch_f64(const double *x, double *y, const int32_t *log2_sizes,
                      const int64_t *offsets, int64_t batch, int adjoint, int threads)
{
    orc_job job = {x, y, log2_sizes, offsets, batch, 0, adjoint ? 1 : 0};
    return orc_run(&job, threads);
}

int orc_chw_batch_i64(const int64_t *x, int64_t *y, const int32_t *log2_sizes,
                      const int64_t *offsets, int64_t batch, int adjoint, int threads)
{
    orc_job job = {x, y, log2_sizes, offsets, batch, 1, adjoint ? 1 : 0};
    return orc_run(&job, threads);
}
