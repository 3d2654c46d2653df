/*
 * MIH-CPU: a plain single-threaded CPU implementation of multi-index hashing,
 * written from the paper to cross-check the reading of its algorithms.
 *
 * TEST INFRASTRUCTURE ONLY (a second test subject beside the oracle, not the
 * oracle itself).  Nothing in the product path may call, link or execute it;
 * it shares no code with the GPU library.
 *
 * Substrings (Section 2.1 and its footnote): a q-bit code is split into m
 * disjoint runs of contiguous bits; when m does not divide q the lengths are
 * ceil(q/m) or floor(q/m).  Reading used here: the first (q mod m) substrings
 * get the longer length, substring j starts where substring j-1 ends, bit p
 * of a code is bit (p mod 64) of 64-bit word floor(p/64), and the value of a
 * substring reads its first bit as the least significant one.
 *
 * Tables (Algorithm 1): one table per substring, mapping each substring value
 * to the ids holding it.  A table here is the list of (value, id) pairs sorted
 * by value then id, probed by binary search; any exact map gives the same
 * search result.
 *
 * kNN search (Algorithm 3): steps t = 0, 1, 2, ...; step t uses table
 * a = t mod m and substring radius r' = floor(t/m) and looks up every bucket
 * whose value differs from the query's substring in exactly r' bits.  Each
 * candidate not seen before gets its full distance and joins the set N_d of
 * its distance d.  After step t the loop ends when the sets N_0 .. N_t hold
 * at least k codes.  Duplicates are removed with an n-bit bitstring cleared
 * before each query (Section 6, "Duplicate Candidates").  A guard ends the
 * loop once every table has been searched over its whole length, which only
 * matters when k exceeds the number of codes.
 *
 * r-neighbour search (Algorithm 2): with r = m r' + a, tables 1..a+1 are
 * searched within radius r' and the others within r'-1 (Proposition 2), then
 * every candidate farther than r is removed.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MIHCPU_SENTINEL 0xFFFFFFFFu

typedef struct {
    uint64_t value;
    uint32_t id;
} mihcpu_entry;

typedef struct {
    uint64_t n;
    uint32_t words, bits, m;
    uint32_t len[256], start[256];
    mihcpu_entry *table[256];
    const uint64_t *codes;   /* borrowed */
} mihcpu_index;

static uint32_t hamming(const uint64_t *a, const uint64_t *b, uint32_t words)
{
    uint32_t d = 0;
    for (uint32_t w = 0; w < words; ++w) d += (uint32_t)__builtin_popcountll(a[w] ^ b[w]);
    return d;
}

/* value of bits [start, start+len) of a code, first bit least significant */
static uint64_t substring(const uint64_t *code, uint32_t start, uint32_t len)
{
    uint64_t v = 0;
    for (uint32_t i = 0; i < len; ++i) {
        uint32_t p = start + i;
        uint64_t bit = (code[p / 64] >> (p % 64)) & 1ULL;
        v |= bit << i;
    }
    return v;
}

static int entry_cmp(const void *x, const void *y)
{
    const mihcpu_entry *a = (const mihcpu_entry *)x, *b = (const mihcpu_entry *)y;
    if (a->value != b->value) return a->value < b->value ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id);
}

/* Substring lengths and start bits for q bits split m ways. */
void mihcpu_partition(uint32_t bits, uint32_t m, uint32_t *len, uint32_t *start)
{
    uint32_t base = bits / m, extra = bits % m, s = 0;
    for (uint32_t j = 0; j < m; ++j) {
        len[j] = base + (j < extra ? 1 : 0);
        start[j] = s;
        s += len[j];
    }
}

/* Algorithm 1. Returns NULL on bad arguments (m must be in [1, min(bits,256)],
 * substrings at most 64 bits). */
mihcpu_index *mihcpu_build(const uint64_t *codes, uint64_t n, uint32_t words, uint32_t m)
{
    uint32_t bits = 64 * words;
    if (m < 1 || m > bits || m > 256) return NULL;
    if ((bits + m - 1) / m > 64) return NULL;
    mihcpu_index *ix = (mihcpu_index *)calloc(1, sizeof(mihcpu_index));
    ix->n = n; ix->words = words; ix->bits = bits; ix->m = m; ix->codes = codes;
    mihcpu_partition(bits, m, ix->len, ix->start);
    for (uint32_t j = 0; j < m; ++j) {
        mihcpu_entry *t = (mihcpu_entry *)malloc(sizeof(mihcpu_entry) * (n ? n : 1));
        for (uint64_t i = 0; i < n; ++i) {
            t[i].value = substring(codes + i * words, ix->start[j], ix->len[j]);
            t[i].id = (uint32_t)i;
        }
        qsort(t, n, sizeof(mihcpu_entry), entry_cmp);
        ix->table[j] = t;
    }
    return ix;
}

void mihcpu_free(mihcpu_index *ix)
{
    if (!ix) return;
    for (uint32_t j = 0; j < ix->m; ++j) free(ix->table[j]);
    free(ix);
}

/* [lo, hi) of the entries of table j whose value equals v */
static void bucket(const mihcpu_index *ix, uint32_t j, uint64_t v, uint64_t *lo, uint64_t *hi)
{
    const mihcpu_entry *t = ix->table[j];
    uint64_t a = 0, b = ix->n;
    while (a < b) { uint64_t c = (a + b) / 2; if (t[c].value < v) a = c + 1; else b = c; }
    *lo = a;
    b = ix->n;
    while (a < b) { uint64_t c = (a + b) / 2; if (t[c].value <= v) a = c + 1; else b = c; }
    *hi = a;
}

/* next larger integer with the same number of set bits (Gosper) */
static uint64_t next_same_popcount(uint64_t x)
{
    uint64_t c = x & (~x + 1);
    uint64_t r = x + c;
    return (((r ^ x) >> 2) / c) | r;
}

typedef struct {
    uint64_t steps;       /* search steps executed */
    uint64_t lookups;     /* buckets examined */
    uint64_t candidates;  /* ids returned by the buckets, duplicates included */
    uint64_t unique;      /* distinct candidates whose full distance was measured */
    uint64_t radius;      /* full search radius r reached when the loop ended */
} mihcpu_stats;

typedef struct {
    uint32_t d, id;
} found_t;

static int found_cmp(const void *x, const void *y)
{
    const found_t *a = (const found_t *)x, *b = (const found_t *)y;
    if (a->d != b->d) return a->d < b->d ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id);
}

/* Visit every bucket of table j whose value differs from v in exactly rho
 * bits; each id found is passed to the visitor. */
typedef struct {
    const mihcpu_index *ix;
    const uint64_t *g;
    uint8_t *seen;
    found_t *found;
    uint64_t nfound;
    uint64_t *count_d;
    mihcpu_stats *st;
} visit_ctx;

static void probe_shell(visit_ctx *C, uint32_t j, uint64_t v, uint32_t rho)
{
    const mihcpu_index *ix = C->ix;
    uint32_t s = ix->len[j];
    if (rho > s) return;
    uint64_t limit = (s == 64) ? 0 : (1ULL << s);   /* 0 means 2^64 */
    uint64_t mask = (rho == 64) ? ~0ULL : ((1ULL << rho) - 1);
    for (;;) {
        uint64_t lo, hi;
        C->st->lookups++;
        bucket(ix, j, v ^ mask, &lo, &hi);
        for (uint64_t e = lo; e < hi; ++e) {
            uint32_t id = ix->table[j][e].id;
            C->st->candidates++;
            if (C->seen[id >> 3] & (1u << (id & 7))) continue;
            C->seen[id >> 3] |= (uint8_t)(1u << (id & 7));
            C->st->unique++;
            uint32_t d = hamming(ix->codes + (uint64_t)id * ix->words, C->g, ix->words);
            C->found[C->nfound].d = d;
            C->found[C->nfound].id = id;
            C->nfound++;
            C->count_d[d]++;
        }
        if (rho == 0 || rho == s) break;
        /* stop after the largest mask of this popcount within s bits */
        uint64_t top = ((1ULL << rho) - 1) << (s - rho);
        if (mask == top) break;
        mask = next_same_popcount(mask);
        if (limit && mask >= limit) break;
    }
}

/*
 * Algorithm 3 for one query.  Writes min(k, n) results in (d, id) order to
 * ids/dists and pads up to k with the sentinel.  Returns 0, or -1 on no memory.
 */
/*
 * Algorithm 3 for one query, optionally stopped early (the approximate
 * variants of Section 7): after the step that covers radius max_step
 * (UINT32_MAX: no limit), or after the step during which the number of
 * distinct codes met reaches max_found (0: no limit).  Returns the k best
 * of the codes met, in (d, id) order, sentinel-padded.
 */
int mihcpu_knn_approx(const mihcpu_index *ix, const uint64_t *g, uint32_t k, uint32_t max_step,
                      uint64_t max_found, uint32_t *ids, uint32_t *dists, mihcpu_stats *st);

int mihcpu_knn(const mihcpu_index *ix, const uint64_t *g, uint32_t k, uint32_t *ids,
               uint32_t *dists, mihcpu_stats *st)
{
    return mihcpu_knn_approx(ix, g, k, 0xFFFFFFFFu, 0, ids, dists, st);
}

int mihcpu_knn_approx(const mihcpu_index *ix, const uint64_t *g, uint32_t k, uint32_t max_step,
                      uint64_t max_found, uint32_t *ids, uint32_t *dists, mihcpu_stats *st)
{
    mihcpu_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    for (uint32_t r = 0; r < k; ++r) { ids[r] = MIHCPU_SENTINEL; dists[r] = MIHCPU_SENTINEL; }
    if (k == 0) return 0;

    uint8_t *seen = (uint8_t *)calloc(ix->n / 8 + 1, 1);
    found_t *found = (found_t *)malloc(sizeof(found_t) * (ix->n ? ix->n : 1));
    uint64_t *count_d = (uint64_t *)calloc(ix->bits + 1, sizeof(uint64_t));
    if (!seen || !found || !count_d) { free(seen); free(found); free(count_d); return -1; }
    visit_ctx C = {ix, g, seen, found, 0, count_d, st};

    uint32_t maxlen = 0;
    for (uint32_t j = 0; j < ix->m; ++j) if (ix->len[j] > maxlen) maxlen = ix->len[j];

    uint32_t rp = 0, a = 0, r = 0;
    for (;;) {
        /* buckets of table a that differ from the query substring in exactly rp bits */
        uint64_t v = substring(g, ix->start[a], ix->len[a]);
        probe_shell(&C, a, v, rp);
        st->steps++;
        a++;
        if (a >= ix->m) { a = 0; rp++; }
        r++;
        uint64_t within = 0;
        for (uint32_t d = 0; d < r && d <= ix->bits; ++d) within += count_d[d];
        if (within >= k) break;
        if (rp > maxlen) break;   /* every table searched over its whole length */
        if (max_step != 0xFFFFFFFFu && r > max_step) break;   /* radius max_step covered */
        if (max_found && C.nfound >= max_found) break;        /* enough distinct codes met */
    }
    st->radius = r;

    qsort(found, C.nfound, sizeof(found_t), found_cmp);
    uint64_t out = C.nfound < k ? C.nfound : k;
    for (uint64_t i = 0; i < out; ++i) { ids[i] = found[i].id; dists[i] = found[i].d; }
    free(seen);
    free(found);
    free(count_d);
    return 0;
}

/*
 * Algorithm 2 for one query and radius r.  Returns the number of r-neighbours
 * (writes at most cap of them in (d, id) order), or -1 on no memory.
 */
int64_t mihcpu_rnn(const mihcpu_index *ix, const uint64_t *g, uint32_t r, uint32_t *ids,
                   uint32_t *dists, uint64_t cap, mihcpu_stats *st)
{
    mihcpu_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    uint8_t *seen = (uint8_t *)calloc(ix->n / 8 + 1, 1);
    found_t *found = (found_t *)malloc(sizeof(found_t) * (ix->n ? ix->n : 1));
    uint64_t *count_d = (uint64_t *)calloc(ix->bits + 1, sizeof(uint64_t));
    if (!seen || !found || !count_d) { free(seen); free(found); free(count_d); return -1; }
    visit_ctx C = {ix, g, seen, found, 0, count_d, st};

    uint32_t rp = r / ix->m, a = r - ix->m * rp;
    for (uint32_t j = 0; j < ix->m; ++j) {
        int32_t radius = (j <= a) ? (int32_t)rp : (int32_t)rp - 1;
        uint64_t v = substring(g, ix->start[j], ix->len[j]);
        for (int32_t rho = 0; rho <= radius; ++rho) probe_shell(&C, j, v, (uint32_t)rho);
    }
    qsort(found, C.nfound, sizeof(found_t), found_cmp);
    uint64_t total = 0;
    for (uint64_t i = 0; i < C.nfound; ++i) {
        if (found[i].d > r) break;
        if (total < cap) { ids[total] = found[i].id; dists[total] = found[i].d; }
        total++;
    }
    st->radius = r;
    free(seen);
    free(found);
    free(count_d);
    return (int64_t)total;
}

/* Substring value of one code (exposed for tests of the partition). */
uint64_t mihcpu_substring(const uint64_t *code, uint32_t start, uint32_t len)
{
    return substring(code, start, len);
}

/* Copy table j (Algorithm 1's table as (value, id) pairs sorted by value then
 * id) into values[n] and ids[n]. */
void mihcpu_table(const mihcpu_index *ix, uint32_t j, uint64_t *values, uint32_t *ids)
{
    for (uint64_t i = 0; i < ix->n; ++i) {
        values[i] = ix->table[j][i].value;
        ids[i] = ix->table[j][i].id;
    }
}
