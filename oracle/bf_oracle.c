/*
 * FP64 oracle for the beamforming product of the paper (Section III,
 * beamforming paragraph and its equation): for every item t,
 *
 *     R_t[i][j] = sum_{k=0}^{f_t-1} W_{w_t}[i][k] * S_t[k][j]
 *
 * with W one precoder of the pool (one row per antenna), S_t the f_t x b
 * symbol matrix (one row per flow, one column per resource element) and
 * the complex product written out as (a+bi)(c+di) = (ac - bd) + (ad + bc)i.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or constant with the GPU
 * library.
 *
 * Deliberately plain: complex64 inputs are widened exactly to double,
 * the sum runs over k = 0 .. f-1 in that order, no blocking, no fusion.
 * Build with -O2 -ffp-contract=off and without fast-math so that every
 * multiply and add is a separately rounded IEEE double operation.
 *
 * ORACLE_MUTANT (compile-time, tests only) plants one plausible mistake so
 * the pin tests can show that they catch it.  The default build has none.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

typedef struct {
    int64_t begin, end;
    int m, b, ldw;
    const float *w;
    const int32_t *w_id;
    const int32_t *f;
    const float *s;
    const int64_t *s_off;
    double *r;
} job_t;

/* One product: W is m x ldw complex64 (leading f columns used), S is f x b
 * complex64, R is m x b complex128; all row-major, (re, im) interleaved. */
static void product(int m, int b, int ldw, const float *w, int f,
                    const float *s, double *r)
{
    int kend = f;
#if ORACLE_MUTANT == 3
    kend = f > 0 ? f - 1 : 0;               /* drops the last flow */
#endif
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < b; ++j) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < kend; ++k) {
#if ORACLE_MUTANT == 4
                const float *wp = w + 2 * ((int64_t)k * m + i);           /* W indexed transposed */
#else
                const float *wp = w + 2 * ((int64_t)i * ldw + k);
#endif
#if ORACLE_MUTANT == 5
                const float *sp = s + 2 * ((int64_t)j * f + k);           /* S indexed transposed */
#else
                const float *sp = s + 2 * ((int64_t)k * b + j);
#endif
                double a = wp[0], bb = wp[1];
                double c = sp[0], d = sp[1];
#if ORACLE_MUTANT == 1
                re += a * c - bb * d;
                im += a * d - bb * c;               /* wrong sign on one cross term */
#elif ORACLE_MUTANT == 2
                re += a * c + bb * d;               /* conjugated W */
                im += a * d - bb * c;
#elif ORACLE_MUTANT == 7
                re += a * c - bb * d;
                im += bb * d + a * c;               /* wrong pairing in the imaginary part */
#else
                re += a * c - bb * d;
                im += a * d + bb * c;
#endif
            }
            r[2 * ((int64_t)i * b + j)] = re;
            r[2 * ((int64_t)i * b + j) + 1] = im;
        }
    }
}

static void *run(void *arg)
{
    const job_t *jb = (const job_t *)arg;
    const int64_t w_elems = (int64_t)jb->m * jb->ldw;
    for (int64_t t = jb->begin; t < jb->end; ++t) {
#if ORACLE_MUTANT == 6
        const float *w = jb->w;                     /* ignores the W id */
#else
        const float *w = jb->w + 2 * (int64_t)jb->w_id[t] * w_elems;
#endif
        product(jb->m, jb->b, jb->ldw, w, jb->f[t],
                jb->s + 2 * jb->s_off[t], jb->r + 2 * t * (int64_t)jb->m * jb->b);
    }
    return NULL;
}

/*
 * n        number of products
 * m, b     rows of W and R, columns of S and R (64 and 60 in the paper)
 * ldw      row stride of each pool entry in complex elements (f_max)
 * n_w      number of pool entries
 * w        complex64 [n_w][m][ldw]
 * w_id, f  int32 [n]
 * s        complex64 buffer; item t's S starts at complex element s_off[t]
 * r        complex128 [n][m][b] output
 * threads  worker threads (<= 0: one)
 * Returns 0, or -1 if an argument is out of range (nothing written).
 */
int oracle_bf_apply(int64_t n, int m, int b, int ldw, int64_t n_w,
                    const float *w, const int32_t *w_id, const int32_t *f,
                    const float *s, const int64_t *s_off, double *r, int threads)
{
    if (n < 0 || m <= 0 || b <= 0 || ldw < 0)
        return -1;
    for (int64_t t = 0; t < n; ++t) {
        if (w_id[t] < 0 || w_id[t] >= n_w || f[t] < 0 || f[t] > ldw || s_off[t] < 0)
            return -1;
    }
    if (threads <= 0)
        threads = 1;
    if (threads > n)
        threads = n > 0 ? (int)n : 1;
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    job_t *jobs = (job_t *)calloc((size_t)threads, sizeof(job_t));
    if (!tid || !jobs) {
        free(tid);
        free(jobs);
        return -1;
    }
    for (int k = 0; k < threads; ++k) {
        job_t *jb = &jobs[k];
        jb->begin = n * k / threads;
        jb->end = n * (k + 1) / threads;
        jb->m = m;
        jb->b = b;
        jb->ldw = ldw;
        jb->w = w;
        jb->w_id = w_id;
        jb->f = f;
        jb->s = s;
        jb->s_off = s_off;
        jb->r = r;
    }
    int started = 0;
    for (int k = 1; k < threads; ++k) {
        if (pthread_create(&tid[k], NULL, run, &jobs[k]) != 0)
            break;
        started = k;
    }
    run(&jobs[0]);
    for (int k = started + 1; k < threads; ++k)   /* threads that failed to start: run inline */
        run(&jobs[k]);
    for (int k = 1; k <= started; ++k)
        pthread_join(tid[k], NULL);
    free(tid);
    free(jobs);
    return 0;
}
