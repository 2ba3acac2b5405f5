/*
 * CPU-parallel DialSort baseline -- test and benchmark infrastructure only.
 *
 * A multi-threaded CPU form of the method, for host-core timing context beside
 * the GPU path (the paper's own CPU variant runs on 8 threads but does not say
 * how it splits the work, so this split is ours).  Only the tests and the
 * benchmark's CPU-baseline leg load it; the product never does.
 *
 *   1. ingestion (Sec. 3.3, Eq. (1)): thread t counts its contiguous slice of
 *      the keys into a private histogram H_t[0, U);
 *   2. merge: H[k] = sum over t of H_t[k], each thread summing one range of k;
 *   3. projection (Eq. (2)): each thread takes one range of k, learns where its
 *      range starts in the output from the range totals of the threads before
 *      it, and writes k exactly H[k] times for the k of its range.
 *
 * Returns 0 on success, 1 on bad arguments or allocation failure, 2 when a key
 * is >= U (the outputs are then unspecified).  Counters are 32-bit, as in the
 * oracle, so n must be below 2^32.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    const uint32_t *keys;
    uint64_t n, U;
    uint32_t *H, *out;
    uint32_t **priv;
    uint64_t *range_total;
    int nthreads, t, bad;
    pthread_barrier_t *bar;
} job_t;

static void slice(uint64_t len, int parts, int i, uint64_t *b, uint64_t *e) {
    *b = len * (uint64_t)i / (uint64_t)parts;
    *e = len * (uint64_t)(i + 1) / (uint64_t)parts;
}

static void *worker(void *arg) {
    job_t *j = (job_t *)arg;
    uint64_t b, e, k, i;
    uint32_t *h = j->priv[j->t];
    /* 1. private counts */
    for (k = 0; k < j->U; ++k) h[k] = 0;
    slice(j->n, j->nthreads, j->t, &b, &e);
    for (i = b; i < e; ++i) {
        uint32_t x = j->keys[i];
        if (x >= j->U) { j->bad = 1; continue; }
        h[x] += 1;
    }
    pthread_barrier_wait(j->bar);
    /* 2. merge one range of bins, and its total */
    slice(j->U, j->nthreads, j->t, &b, &e);
    uint64_t tot = 0;
    for (k = b; k < e; ++k) {
        uint32_t s = 0;
        int t;
        for (t = 0; t < j->nthreads; ++t) s += j->priv[t][k];
        j->H[k] = s;
        tot += s;
    }
    j->range_total[j->t] = tot;
    pthread_barrier_wait(j->bar);
    /* 3. project the same range from its offset */
    if (j->out) {
        uint64_t pos = 0;
        int t;
        for (t = 0; t < j->t; ++t) pos += j->range_total[t];
        for (k = b; k < e; ++k) {
            uint32_t c = j->H[k];
            uint32_t r;
            for (r = 0; r < c; ++r) j->out[pos++] = (uint32_t)k;
        }
    }
    return NULL;
}

int cpu_parallel_sort(const uint32_t *keys, uint64_t n, uint64_t U, uint32_t *H, uint32_t *out, int nthreads) {
    int t, bad = 0;
    if (U == 0 || H == NULL || (n > 0 && keys == NULL) || nthreads < 1 || n > 0xFFFFFFFFull) return 1;
    uint32_t **priv = (uint32_t **)calloc((size_t)nthreads, sizeof(uint32_t *));
    uint64_t *range_total = (uint64_t *)calloc((size_t)nthreads, sizeof(uint64_t));
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    pthread_barrier_t bar;
    int ok = priv && range_total && jobs && th;
    for (t = 0; ok && t < nthreads; ++t) {
        priv[t] = (uint32_t *)malloc((size_t)U * sizeof(uint32_t));
        ok = priv[t] != NULL;
    }
    if (ok) {
        pthread_barrier_init(&bar, NULL, (unsigned)nthreads);
        for (t = 0; t < nthreads; ++t) {
            job_t j = {keys, n, U, H, out, priv, range_total, nthreads, t, 0, &bar};
            jobs[t] = j;
        }
        for (t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, worker, &jobs[t]);
        worker(&jobs[0]);
        for (t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
        pthread_barrier_destroy(&bar);
        for (t = 0; t < nthreads; ++t) bad |= jobs[t].bad;
    }
    if (priv)
        for (t = 0; t < nthreads; ++t) free(priv[t]);
    free(priv);
    free(range_total);
    free(jobs);
    free(th);
    if (!ok) return 1;
    return bad ? 2 : 0;
}
