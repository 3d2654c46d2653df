/*
 * Seeded synthetic binary-code generators (host side).
 *
 * This module produces inputs only.  It holds none of the search method's
 * arithmetic (no Hamming distances, no substrings, no tables): it is shared by
 * the CPU oracle and the GPU library as the common source of test data.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), used counter-based:
 *     out(seed, c) = mix64(seed + (c + 1) * GAMMA)
 * with SplitMix64's golden-ratio increment GAMMA and its 64-bit finaliser.
 * Every value is addressed by (seed, counter), so rows can be generated in any
 * order, by any number of threads, on the host or on the device, with
 * bit-identical results.
 *
 * Workload shapes follow the paper's experiments (Section 5.1): codes of
 * 64/128/256 bits, either i.i.d. uniform bits (the analysis regime of
 * Section 3) or sign-of-random-projection codes of points drawn from an
 * isotropic Gaussian mixture in 128-D (a stand-in for LSH codes of SIFT
 * descriptors, which are not available here).
 *
 * Clustered recipe (all integer, so host and device agree bit for bit):
 *   G(seed, c) = sum of twelve 16-bit uniforms taken from out(seed, c),
 *                out(seed, c+1), out(seed, c+2), minus 6 * 65536.
 *                This is the Irwin-Hall approximation of N(0, 65536^2).
 *   means      mu[c][i] = G(2, 3*(c*128 + i))           c < 1000, i < 128
 *   planes     w[j][i]  = G(3, 3*(j*128 + i))           j < bits
 *   point p    (stream seed S, 385 outputs per point starting at 385*p):
 *              component c = floor(1000 * u) with u = out(S, 385p) / 2^64
 *              eps_i = G(S, 385p + 1 + 3i)
 *              x_i   = 10 * mu[c][i] + 3 * eps_i      (= 10 * (mu + 0.3 eps))
 *              bit j = [ sum_i w[j][i] * x_i > 0 ]     (exact int64)
 * Bit j of a code is bit (j mod 64) of 64-bit word floor(j / 64).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define DG_GAMMA 0x9E3779B97F4A7C15ULL
#define DG_CLUSTERS 1000
#define DG_DIM 128
#define DG_PER_POINT (1 + 3 * DG_DIM)

static inline uint64_t dg_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t dg_splitmix(uint64_t seed, uint64_t counter)
{
    return dg_mix64(seed + (counter + 1) * DG_GAMMA);
}

static inline int64_t dg_gauss(uint64_t seed, uint64_t c)
{
    int64_t s = 0;
    for (int w = 0; w < 3; ++w) {
        uint64_t u = dg_splitmix(seed, c + (uint64_t)w);
        s += (int64_t)(u & 0xFFFF) + (int64_t)((u >> 16) & 0xFFFF) +
             (int64_t)((u >> 32) & 0xFFFF) + (int64_t)(u >> 48);
    }
    return s - 6 * 65536;
}

int64_t dg_gauss_public(uint64_t seed, uint64_t c) { return dg_gauss(seed, c); }

/* ---------------------------------------------------------------- threads */

typedef struct {
    void (*fn)(void *ctx, uint64_t lo, uint64_t hi);
    void *ctx;
    uint64_t lo, hi;
} dg_job;

static void *dg_run(void *p)
{
    dg_job *j = (dg_job *)p;
    j->fn(j->ctx, j->lo, j->hi);
    return NULL;
}

static void dg_parallel(void (*fn)(void *, uint64_t, uint64_t), void *ctx,
                        uint64_t n, int threads)
{
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    if ((uint64_t)threads > n) threads = n ? (int)n : 1;
    pthread_t tid[256];
    dg_job job[256];
    uint64_t per = (n + (uint64_t)threads - 1) / (uint64_t)threads;
    for (int t = 0; t < threads; ++t) {
        uint64_t lo = per * (uint64_t)t, hi = lo + per;
        if (lo > n) lo = n;
        if (hi > n) hi = n;
        job[t].fn = fn; job[t].ctx = ctx; job[t].lo = lo; job[t].hi = hi;
        /* the last slice runs on the calling thread, as does any slice whose
         * thread could not be started */
        if (t == threads - 1 || pthread_create(&tid[t], NULL, dg_run, &job[t]) != 0) {
            dg_run(&job[t]);
            tid[t] = 0;
        }
    }
    for (int t = 0; t < threads - 1; ++t)
        if (tid[t]) pthread_join(tid[t], NULL);
}

/* ---------------------------------------------------------------- uniform */

typedef struct {
    uint64_t *out;
    uint32_t words;
    uint64_t seed, first_row;
} dg_uniform_ctx;

static void dg_uniform_part(void *p, uint64_t lo, uint64_t hi)
{
    dg_uniform_ctx *c = (dg_uniform_ctx *)p;
    for (uint64_t i = lo; i < hi; ++i)
        for (uint32_t w = 0; w < c->words; ++w)
            c->out[i * c->words + w] =
                dg_splitmix(c->seed, (c->first_row + i) * c->words + w);
}

/* Rows [first_row, first_row + n) of the uniform stream: word w of row i is
 * out(seed, i * words + w).  Every bit is Bernoulli(1/2). */
void dg_uniform(uint64_t *out, uint64_t n, uint32_t words, uint64_t seed,
                uint64_t first_row, int threads)
{
    dg_uniform_ctx c = {out, words, seed, first_row};
    dg_parallel(dg_uniform_part, &c, n, threads);
}

/* -------------------------------------------------------------- clustered */

typedef struct {
    uint64_t *out;
    uint32_t bits;
    uint64_t seed, first_row;
    const int64_t *mu;    /* [DG_CLUSTERS][DG_DIM] */
    const int64_t *w;     /* [bits][DG_DIM] */
} dg_clustered_ctx;

static void dg_clustered_part(void *p, uint64_t lo, uint64_t hi)
{
    dg_clustered_ctx *c = (dg_clustered_ctx *)p;
    uint32_t words = c->bits / 64;
    int64_t x[DG_DIM];
    for (uint64_t i = lo; i < hi; ++i) {
        uint64_t row = c->first_row + i;
        uint64_t base = row * (uint64_t)DG_PER_POINT;
        uint64_t u = dg_splitmix(c->seed, base);
        uint64_t comp = (uint64_t)(((unsigned __int128)u * DG_CLUSTERS) >> 64);
        const int64_t *mu = c->mu + comp * DG_DIM;
        for (int d = 0; d < DG_DIM; ++d)
            x[d] = 10 * mu[d] + 3 * dg_gauss(c->seed, base + 1 + 3 * (uint64_t)d);
        for (uint32_t wd = 0; wd < words; ++wd) {
            uint64_t word = 0;
            for (uint32_t b = 0; b < 64; ++b) {
                const int64_t *wj = c->w + (uint64_t)(wd * 64 + b) * DG_DIM;
                int64_t dot = 0;
                for (int d = 0; d < DG_DIM; ++d) dot += wj[d] * x[d];
                if (dot > 0) word |= 1ULL << b;
            }
            c->out[i * words + wd] = word;
        }
    }
}

void dg_clustered_params(int64_t *mu, int64_t *w, uint32_t bits)
{
    for (uint64_t c = 0; c < DG_CLUSTERS; ++c)
        for (uint64_t d = 0; d < DG_DIM; ++d)
            mu[c * DG_DIM + d] = dg_gauss(2, 3 * (c * DG_DIM + d));
    for (uint64_t j = 0; j < bits; ++j)
        for (uint64_t d = 0; d < DG_DIM; ++d)
            w[j * DG_DIM + d] = dg_gauss(3, 3 * (j * DG_DIM + d));
}

/* Rows [first_row, first_row + n) of the clustered stream with point seed
 * `seed` (4 for database points, 5 for queries). bits must be a multiple of 64
 * and at most 256. Returns 0 on success, -1 on bad arguments or no memory. */
int dg_clustered(uint64_t *out, uint64_t n, uint32_t bits, uint64_t seed,
                 uint64_t first_row, int threads)
{
    if (bits == 0 || bits % 64 != 0 || bits > 256) return -1;
    int64_t *mu = (int64_t *)malloc(sizeof(int64_t) * DG_CLUSTERS * DG_DIM);
    int64_t *w = (int64_t *)malloc(sizeof(int64_t) * bits * DG_DIM);
    if (!mu || !w) { free(mu); free(w); return -1; }
    dg_clustered_params(mu, w, bits);
    dg_clustered_ctx c = {out, bits, seed, first_row, mu, w};
    dg_parallel(dg_clustered_part, &c, n, threads);
    free(mu);
    free(w);
    return 0;
}

/* Per-query k drawn uniformly from a list of choices: k_i = choices[floor(
 * nchoices * u_i)], u_i = out(seed, i) / 2^64. */
void dg_choice_u32(uint32_t *out, uint64_t n, const uint32_t *choices,
                   uint32_t nchoices, uint64_t seed, uint64_t first)
{
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t u = dg_splitmix(seed, first + i);
        out[i] = choices[(uint64_t)(((unsigned __int128)u * nchoices) >> 64)];
    }
}

/* Uniform doubles in (0, 1): ((x >> 11) + 0.5) * 2^-53, never 0 or 1. */
void dg_uniform_f64(double *out, uint64_t n, uint64_t seed, uint64_t first)
{
    for (uint64_t i = 0; i < n; ++i)
        out[i] = ((double)(dg_splitmix(seed, first + i) >> 11) + 0.5) *
                 (1.0 / 9007199254740992.0);
}
