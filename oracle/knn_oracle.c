/*
 * CPU oracle for exact Hamming k-nearest-neighbour search.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * execute this file; it is used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg.  It shares no code with the GPU library.
 *
 * What it computes is the plain definition of the problem (Section 1.1): for
 * a query g and database codes h_0 .. h_{n-1} of q bits, the Hamming distance
 * is d_i = sum over 64-bit words of popcount(h_i[w] XOR g[w]) (one xor per 64
 * bits followed by a population count, Section 6, "Hamming Distance"); the
 * k nearest neighbours are the first min(k, n) pairs (d_i, i) in ascending
 * lexicographic order.  The paper accepts any choice among equidistant codes
 * (Section 5.1, last paragraph); this oracle fixes the choice to the lowest
 * id, so exactly one output is correct.  Rows with fewer than k results are
 * padded with id = dist = 0xFFFFFFFF.
 *
 * Method: per query, one pass builds the histogram of distances, which gives
 * the k-th smallest distance D and how many codes at distance D are taken;
 * a second pass over ids in ascending order places every taken code at its
 * rank, which is a stable counting sort of (d, i) truncated to k entries.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORACLE_SENTINEL 0xFFFFFFFFu

static inline uint32_t hamming(const uint64_t *a, const uint64_t *b, uint32_t words)
{
    uint32_t d = 0;
    for (uint32_t w = 0; w < words; ++w) d += (uint32_t)__builtin_popcountll(a[w] ^ b[w]);
    return d;
}

/* Exact kNN of one query; hist must hold bits+1 counters, pos bits+1. */
static void knn_one(const uint64_t *codes, uint64_t n, uint32_t words, const uint64_t *g,
                    uint32_t k, uint32_t *ids, uint32_t *dists, uint64_t *hist, uint64_t *pos)
{
    const uint32_t bits = 64 * words;
    uint64_t kk = k < n ? k : n;
    for (uint32_t r = 0; r < k; ++r) { ids[r] = ORACLE_SENTINEL; dists[r] = ORACLE_SENTINEL; }
    if (kk == 0) return;

    memset(hist, 0, sizeof(uint64_t) * (bits + 1));
    for (uint64_t i = 0; i < n; ++i) hist[hamming(codes + i * words, g, words)]++;

    /* D = smallest distance whose cumulative count reaches kk */
    uint64_t cum = 0;
    uint32_t D = bits;
    for (uint32_t d = 0; d <= bits; ++d) {
        cum += hist[d];
        if (cum >= kk) { D = d; break; }
    }
    uint64_t below = cum - hist[D];       /* codes with distance < D */
    uint64_t take_at_D = kk - below;      /* lowest-id codes taken at distance D */

    /* first output rank of each distance */
    uint64_t r = 0;
    for (uint32_t d = 0; d <= bits; ++d) {
        pos[d] = r;
        if (d < D) r += hist[d];
        else if (d == D) r += take_at_D;
    }
    uint64_t taken = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t d = hamming(codes + i * words, g, words);
        if (d < D || (d == D && taken < take_at_D)) {
            if (d == D) taken++;
            ids[pos[d]] = (uint32_t)i;
            dists[pos[d]] = d;
            pos[d]++;
        }
    }
}

typedef struct {
    const uint64_t *codes;
    uint64_t n;
    uint32_t words;
    const uint64_t *queries;
    uint32_t nq;
    const uint32_t *k;          /* per-query k */
    const uint64_t *row_off;    /* output offset of each row */
    uint32_t *out_ids, *out_dists;
    volatile uint32_t next;
    pthread_mutex_t mu;
} knn_job;

static void *knn_worker(void *p)
{
    knn_job *J = (knn_job *)p;
    uint32_t bits = 64 * J->words;
    uint64_t *hist = (uint64_t *)malloc(sizeof(uint64_t) * (bits + 1));
    uint64_t *pos = (uint64_t *)malloc(sizeof(uint64_t) * (bits + 1));
    for (;;) {
        pthread_mutex_lock(&J->mu);
        uint32_t q = J->next;
        if (q < J->nq) J->next = q + 1;
        pthread_mutex_unlock(&J->mu);
        if (q >= J->nq) break;
        knn_one(J->codes, J->n, J->words, J->queries + (uint64_t)q * J->words, J->k[q],
                J->out_ids + J->row_off[q], J->out_dists + J->row_off[q], hist, pos);
    }
    free(hist);
    free(pos);
    return NULL;
}

/*
 * codes [n][words], queries [nq][words], k[nq] per-query k, row_off[nq] the
 * output offset of each row (normally the exclusive prefix sum of k).
 * Threads share the queries; the result does not depend on their number.
 * Returns the number of threads used.
 */
int oracle_knn(const uint64_t *codes, uint64_t n, uint32_t words, const uint64_t *queries,
               uint32_t nq, const uint32_t *k, const uint64_t *row_off, uint32_t *out_ids,
               uint32_t *out_dists, int threads)
{
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    if ((uint32_t)threads > nq) threads = nq ? (int)nq : 1;
    knn_job J;
    J.codes = codes; J.n = n; J.words = words; J.queries = queries; J.nq = nq;
    J.k = k; J.row_off = row_off; J.out_ids = out_ids; J.out_dists = out_dists; J.next = 0;
    pthread_mutex_init(&J.mu, NULL);
    pthread_t tid[256];
    int started = 0;
    for (int t = 1; t < threads; ++t)
        if (pthread_create(&tid[started], NULL, knn_worker, &J) == 0) started++;
    knn_worker(&J);
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    pthread_mutex_destroy(&J.mu);
    return started + 1;
}

/*
 * r-neighbour search by definition (Section 1.1, the r-neighbour problem):
 * every code with d_i <= r, in ascending (d, i) order.  Writes at most `cap`
 * entries and returns the total count (which may exceed cap).
 */
uint64_t oracle_rnn(const uint64_t *codes, uint64_t n, uint32_t words, const uint64_t *g,
                    uint32_t r, uint32_t *ids, uint32_t *dists, uint64_t cap)
{
    const uint32_t bits = 64 * words;
    uint64_t *hist = (uint64_t *)calloc(bits + 2, sizeof(uint64_t));
    uint64_t *pos = (uint64_t *)calloc(bits + 2, sizeof(uint64_t));
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t d = hamming(codes + i * words, g, words);
        if (d <= r) hist[d]++;
    }
    uint64_t total = 0;
    for (uint32_t d = 0; d <= bits; ++d) { pos[d] = total; total += hist[d]; }
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t d = hamming(codes + i * words, g, words);
        if (d <= r) {
            uint64_t p = pos[d]++;
            if (p < cap) { ids[p] = (uint32_t)i; dists[p] = d; }
        }
    }
    free(hist);
    free(pos);
    return total;
}

/* Distances of every code to one query (for statistical checks). */
void oracle_distances(const uint64_t *codes, uint64_t n, uint32_t words, const uint64_t *g,
                      uint32_t *out)
{
    for (uint64_t i = 0; i < n; ++i) out[i] = hamming(codes + i * words, g, words);
}
