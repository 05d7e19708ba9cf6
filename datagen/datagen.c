/*
 * Seeded synthetic inputs for the MESSI k-NN workloads.
 *
 * This module holds no arithmetic of the indexing or search method: it only
 * draws the collections and queries that both the CPU oracle and the GPU
 * library consume.  Everything is host code (C11 + pthreads).
 *
 * Random source: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), a counter-based generator.  A draw is
 * addressed by (key = seed, counter = (block, row_lo, row_hi, stream)), so any
 * row can be regenerated on its own, in any order, by any number of threads.
 *
 * Gaussian draws: Box-Muller in fp64 from two 53-bit uniforms in (0, 1].
 *
 * Random walk (paper, Experimental Evaluation / Datasets): the first point is
 * an N(0,1) draw and every later point adds a fresh N(0,1) draw to the
 * previous one.  Accumulated in fp64, stored as fp32.
 *
 * Gaussian mixture (stand-in for SALD's 200M x 128 shape): C centres drawn
 * uniformly from [0, 255]^L; a row picks a centre uniformly, adds sigma * N(0,1)
 * per dimension, is rounded half-to-even and clipped to [0, 255].
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DG_FN static inline
#include "dg_core.h"

void dg_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    dg_philox(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1], out);
}

/* The j-th N(0,1) draw of a row (j = 0, 1, ...): pair j/2 of block j/2. */
static void row_gaussians(uint64_t seed, uint32_t stream, uint64_t row, int32_t len, double* g) {
    for (int32_t j = 0; j < len; j += 2) {
        double a, b;
        dg_gauss_pair(seed, stream, row, (uint32_t)(j / 2), &a, &b);
        g[j] = a;
        if (j + 1 < len) g[j + 1] = b;
    }
}

void dg_gaussians(uint64_t seed, uint32_t stream, uint64_t row, int32_t len, double* out) {
    row_gaussians(seed, stream, row, len, out);
}

static void walk_row(uint64_t seed, uint32_t stream, uint64_t row, int32_t len, float* out, double* g) {
    row_gaussians(seed, stream, row, len, g);
    double x = 0.0;
    for (int32_t t = 0; t < len; ++t) {
        x = (t == 0) ? g[0] : x + g[t];
        out[t] = (float)x;
    }
}

/* ---- Gaussian mixture ---------------------------------------------------- */

static void mixture_row(uint64_t seed, uint32_t stream, uint64_t row, int32_t len,
                        const double* centres, int64_t n_centres, double sigma,
                        float* out, double* g) {
    uint64_t c = dg_mixture_cluster(seed, stream, row, (uint64_t)n_centres);
    row_gaussians(seed, stream, row, len, g);
    const double* mu = centres + (size_t)c * (size_t)len;
    for (int32_t j = 0; j < len; ++j) out[j] = (float)dg_round_clip(mu[j] + sigma * g[j]);
}

void dg_mixture_centres(uint64_t seed, uint32_t stream_c, int64_t n_centres, int32_t len, double* out) {
    for (int64_t c = 0; c < n_centres; ++c)
        for (int32_t j = 0; j < len; ++j)
            out[(size_t)c * (size_t)len + (size_t)j] = dg_centre_value(seed, stream_c, (uint64_t)c, j);
}

/* ---- threaded drivers ---------------------------------------------------- */

enum { KIND_WALK = 0, KIND_MIXTURE = 1 };

typedef struct {
    int kind;
    uint64_t seed;
    uint32_t stream;
    uint64_t row0;
    int64_t r_begin, r_end; /* rows of this worker, relative to row0 */
    int32_t len;
    const double* centres;
    int64_t n_centres;
    double sigma;
    float* out;
} job_t;

static void* worker(void* arg) {
    job_t* j = (job_t*)arg;
    double* g = (double*)malloc(sizeof(double) * (size_t)(j->len + 1));
    if (!g) return (void*)1;
    for (int64_t r = j->r_begin; r < j->r_end; ++r) {
        float* dst = j->out + (size_t)r * (size_t)j->len;
        if (j->kind == KIND_WALK)
            walk_row(j->seed, j->stream, j->row0 + (uint64_t)r, j->len, dst, g);
        else
            mixture_row(j->seed, j->stream, j->row0 + (uint64_t)r, j->len, j->centres, j->n_centres, j->sigma, dst, g);
    }
    free(g);
    return NULL;
}

static int run_jobs(job_t proto, int64_t nrows, int nthreads) {
    if (nrows <= 0) return 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > nrows) nthreads = (int)nrows;
    pthread_t th[256];
    job_t jobs[256];
    int rc = 0;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = proto;
        jobs[t].r_begin = nrows * t / nthreads;
        jobs[t].r_end = nrows * (t + 1) / nthreads;
        if (pthread_create(&th[t], NULL, worker, &jobs[t]) != 0) {
            worker(&jobs[t]);
            th[t] = 0;
        }
    }
    for (int t = 0; t < nthreads; ++t) {
        void* ret = NULL;
        if (th[t]) pthread_join(th[t], &ret);
        if (ret) rc = -1;
    }
    return rc;
}

/* Rows [row0, row0 + nrows) of the random-walk collection (seed, stream) into
 * out[nrows][len] (fp32, row-major). */
int dg_random_walks(uint64_t seed, uint32_t stream, uint64_t row0, int64_t nrows, int32_t len,
                    float* out, int nthreads) {
    if (len < 1 || nrows < 0 || !out) return -1;
    job_t p;
    memset(&p, 0, sizeof p);
    p.kind = KIND_WALK; p.seed = seed; p.stream = stream; p.row0 = row0; p.len = len; p.out = out;
    return run_jobs(p, nrows, nthreads);
}

/* Rows of the Gaussian-mixture collection; centres come from dg_mixture_centres. */
int dg_mixture(uint64_t seed, uint32_t stream, uint64_t row0, int64_t nrows, int32_t len,
               const double* centres, int64_t n_centres, double sigma, float* out, int nthreads) {
    if (len < 1 || nrows < 0 || !out || !centres || n_centres < 1) return -1;
    job_t p;
    memset(&p, 0, sizeof p);
    p.kind = KIND_MIXTURE; p.seed = seed; p.stream = stream; p.row0 = row0; p.len = len;
    p.centres = centres; p.n_centres = n_centres; p.sigma = sigma; p.out = out;
    return run_jobs(p, nrows, nthreads);
}

/* Noisy queries: q[i][j] = fl32(base[i][j] + sigma[i] * g), g the j-th N(0,1)
 * draw of row (row0 + i) on (seed, stream).  base is a z-normalised dataset row
 * that the caller produced; no re-normalisation afterwards. */
int dg_add_noise(uint64_t seed, uint32_t stream, uint64_t row0, int64_t nrows, int32_t len,
                 const float* base, const double* sigma, float* out) {
    if (len < 1 || nrows < 0 || !base || !sigma || !out) return -1;
    double* g = (double*)malloc(sizeof(double) * (size_t)(len + 1));
    if (!g) return -1;
    for (int64_t i = 0; i < nrows; ++i) {
        row_gaussians(seed, stream, row0 + (uint64_t)i, len, g);
        for (int32_t j = 0; j < len; ++j)
            out[(size_t)i * (size_t)len + (size_t)j] =
                (float)((double)base[(size_t)i * (size_t)len + (size_t)j] + sigma[i] * g[j]);
    }
    free(g);
    return 0;
}

/* n uniform integers in [0, bound) from (seed, stream), element i addressed by counter i. */
int dg_uniform_ints(uint64_t seed, uint32_t stream, int64_t n, uint64_t bound, uint64_t* out) {
    if (n < 0 || bound == 0 || !out) return -1;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t ctr[4] = {0xFFFFFFFEu, (uint32_t)i, (uint32_t)((uint64_t)i >> 32), stream};
        uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
        uint32_t w[4];
        dg_philox4x32_10(ctr, key, w);
        uint64_t r = ((uint64_t)w[0] << 32) | w[1];
        out[i] = dg_mulshift(r, bound);
    }
    return 0;
}

/* n uniform doubles in (0, 1] (used for Poisson inter-arrival times). */
int dg_uniforms(uint64_t seed, uint32_t stream, int64_t n, double* out) {
    if (n < 0 || !out) return -1;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t ctr[4] = {0xFFFFFFFDu, (uint32_t)i, (uint32_t)((uint64_t)i >> 32), stream};
        uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
        uint32_t w[4];
        dg_philox4x32_10(ctr, key, w);
        out[i] = dg_u53(w[0], w[1]);
    }
    return 0;
}
