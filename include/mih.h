/*
 * mih.h -- exact k-nearest-neighbour search in Hamming space by multi-index
 * hashing, on one AMD Instinct MI355X (gfx950).
 *
 * Problem (Section 1.1 of Norouzi, Punjani, Fleet, "Fast Exact Search in
 * Hamming Space with Multi-Index Hashing"): given a database of n binary codes
 * h_0 .. h_{n-1} of q bits and a query g, return the k codes nearest to g in
 * Hamming distance.  The paper accepts any choice among codes at equal
 * distance; this library fixes the order to ascending (distance, id), so the
 * result is unique and every entry point returns the same bits.
 *
 * Data layout shared by all calls:
 *   - a code of `bits` bits (64, 128, 192 or 256) is bits/64 uint64 words;
 *     bit p of the code is bit (p mod 64) of word floor(p / 64);
 *   - an array of codes is row-major [count][bits/64], 8-byte aligned;
 *   - ids are 0-based row numbers of the database array, as uint32
 *     (so n <= 2^32 - 2, as in Section 6 where ids take 4 bytes);
 *   - results of query i occupy entries [off_i, off_i + k_i) of out_ids and
 *     out_dists, with off_i = k_0 + ... + k_{i-1}; entry off_i + r is the
 *     (r+1)-th nearest code.  When fewer than k_i codes exist the remaining
 *     entries hold MIH_SENTINEL in both arrays.
 *
 * Pointers named device* are HIP device pointers (for example the data_ptr()
 * of a PyTorch tensor on the GPU); host* pointers are ordinary host memory.
 * `stream` is a hipStream_t (NULL for the default stream).  Every call below
 * is blocking: it returns after its work on `stream` has completed.
 *
 * Errors: every call returns a status and never aborts.  Argument errors are
 * detected before any device work or output write (MIH_ERR_INVALID).  Device
 * failures (launch or runtime errors) return MIH_ERR_DEVICE; exhausted device
 * memory returns MIH_ERR_NOMEM.  Internal buffer overflows are resolved
 * inside the library by an exact re-run and never surface.
 */
#ifndef MIH_H
#define MIH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mih_status {
    MIH_OK = 0,
    MIH_ERR_INVALID = 1,      /* bad argument: nothing was written            */
    MIH_ERR_NOMEM = 2,        /* device memory exhausted                       */
    MIH_ERR_DEVICE = 3,       /* HIP runtime or kernel failure                 */
    MIH_ERR_UNSUPPORTED = 4,  /* valid request outside the library's limits    */
    MIH_ERR_CAPACITY = 5      /* server: no free query slot or buffer memory   */
} mih_status;

#define MIH_SENTINEL 0xFFFFFFFFu
#define MIH_K_MAX 4096u        /* largest k per query                          */
#define MIH_M_MAX 64u          /* largest number of substrings                 */
#define MIH_SUBSTRING_MAX 32u  /* longest substring (direct tables, Section 6) */

/* Substring tables.  DIRECT: one offset per substring value, 2^s + 1 uint32
 * entries per table (the direct-address tables of Section 6, stored densely),
 * plus one occupancy bit per value; SORTED: the substring values kept sorted
 * beside the ids, found through a prefix directory and a binary search;
 * GROUPED: like the 32-bucket groups of Section 6, one 64-bit record per 32
 * consecutive values (their occupancy bits and the table position of the
 * group's first code, 2^s / 4 bytes per table), and a bucket is found by
 * scanning its group's codes, so GROUPED needs INLINE codes.  AUTO: for
 * 64-bit codes whose tables hold at most one code per bucket on average
 * (n <= 2^s for the shortest substring), HEADS with INLINE codes when it
 * fits the memory budget; otherwise DIRECT when it fits, else SORTED (and
 * see the codes modes). */
typedef enum mih_table_mode {
    MIH_TABLE_AUTO = 0,
    MIH_TABLE_DIRECT = 1,
    MIH_TABLE_SORTED = 2,
    MIH_TABLE_GROUPED = 3,
    MIH_TABLE_HEADS = 4      /* 64-bit codes: DIRECT whose offset and size sit
                                beside each bucket's first code in 16-byte
                                entries (2^s + 1 of them per table), so that a
                                one-code bucket costs one line; needs INLINE
                                codes */
} mih_table_mode;

/* Where candidate codes are read during verification.  INLINE: each table
 * keeps a copy of the codes in its bucket order, so a bucket's codes are
 * contiguous (m * n * bits/8 extra bytes); INDIRECT: codes are gathered from
 * the caller's array through the ids; MIXED: the first inline_tables tables
 * are INLINE, the others INDIRECT.  AUTO: INLINE when it fits, else as many
 * INLINE tables as fit (MIXED), else INDIRECT.  With AUTO tables as well,
 * SORTED is taken over DIRECT when DIRECT would not leave room for every
 * table's codes and SORTED leaves room for more of them. */
typedef enum mih_codes_mode {
    MIH_CODES_AUTO = 0,
    MIH_CODES_INLINE = 1,
    MIH_CODES_INDIRECT = 2,
    MIH_CODES_MIXED = 3
} mih_codes_mode;

typedef struct mih_build_opts {
    mih_table_mode table_mode;
    mih_codes_mode codes_mode;
    uint64_t mem_budget_bytes;   /* 0: the device memory free at build time */
    const uint16_t *bit_order;   /* host [bits] or NULL.  Substring optimisation
                                    (Section 5.5): a permutation of the code bits;
                                    substring j is made of the code bits
                                    bit_order[start_j .. start_j + s_j), and bit
                                    k of its key is code bit bit_order[start_j + k].
                                    NULL: consecutive bits (bit_order[p] = p).
                                    Results never depend on it; speed may.  Not
                                    retained after the call. */
    uint32_t inline_tables;      /* MIXED: INLINE tables, 1 <= inline_tables < m
                                    (ignored by the other modes) */
    const char *autotune_cache;  /* path of a file of autotuned launches, or
                                    NULL.  mih_autotune on this index first
                                    looks up the index's shape and the sample
                                    (n, bits, m, table and codes modes, inline
                                    tables, number of queries, k) there and, if
                                    found, takes that tuning without timing;
                                    otherwise it times its grid and stores the
                                    result.  The file is one JSON object, key:
                                    [the mih_tuning fields in order]; it is
                                    rewritten whole on a store, and a missing
                                    or unreadable file counts as empty (a store
                                    that fails is skipped).  Copied at build. */
} mih_build_opts;

typedef struct mih_index mih_index;   /* opaque, owned by the library */

typedef struct mih_index_info {
    uint64_t n;
    uint32_t bits, m;
    uint32_t table_mode;          /* MIH_TABLE_DIRECT, _SORTED, _GROUPED or _HEADS */
    uint32_t codes_mode;          /* MIH_CODES_INLINE, _INDIRECT or _MIXED  */
    uint32_t sub_len[MIH_M_MAX];  /* substring lengths s_j                  */
    uint32_t sub_start[MIH_M_MAX];/* first bit of substring j               */
    uint32_t dir_bits[MIH_M_MAX]; /* SORTED: directory bits per table       */
    uint64_t device_bytes;        /* device memory held by the index        */
    double build_ms;              /* wall time of mih_build                 */
    uint16_t bit_order[256];      /* the bit order of the substrings (the
                                     identity unless one was given)         */
    uint32_t inline_tables;       /* tables 0 .. inline_tables - 1 keep their
                                     codes inline (m for INLINE, 0 for
                                     INDIRECT)                              */
} mih_index_info;

/* Device views of one table, for inspection and tests.  Pointers are owned
 * by the index and valid until mih_free. */
typedef struct mih_table_view {
    const uint32_t *offsets;     /* DIRECT: [2^len + 1], else NULL          */
    const uint32_t *keys;        /* SORTED: [n] substring values, else NULL */
    const uint32_t *dir;         /* SORTED: [2^dir_bits + 1], else NULL     */
    const uint32_t *ids;         /* [n] ids in bucket order                 */
    const uint64_t *codes;       /* an INLINE table: [n][bits/64], else NULL */
    uint32_t len, start, dir_bits, pad;
    const uint32_t *occupancy;   /* DIRECT: [max(2^len / 32, 1)] words, bit
                                    v % 32 of word v / 32 = [bucket v is
                                    non-empty]; else NULL                   */
    const uint64_t *groups;      /* GROUPED: [max(2^len / 32, 1)] records:
                                    bits 0..31 occupancy of values 32g..32g+31,
                                    bits 32..63 position of the first code
                                    with value >= 32g; else NULL            */
    const uint64_t *heads;       /* HEADS: [2^len + 1] pairs of words: the
                                    bucket's first code (0 if empty), then its
                                    offset in the low 32 bits and its size in
                                    the high 32 bits; else NULL             */
} mih_table_view;

/* Per-call counters of the multi-index search (sums over the queries). */
typedef struct mih_query_stats {
    uint64_t probes;       /* buckets examined (Algorithm 3 lookups)          */
    uint64_t candidates;   /* bucket entries verified with the full distance   */
    uint64_t appended;     /* candidates kept as possible neighbours           */
    uint64_t steps;        /* search steps summed over queries                 */
    uint32_t rounds;       /* device rounds (one step per active query each)   */
    uint32_t reruns;       /* queries re-run with an exact buffer capacity     */
    double elapsed_ms;     /* wall time of the call                            */
    double search_kernel_ms;   /* HIP-event time of the search kernel launches */
    uint32_t search_launches;  /* number of those launches                     */
    uint32_t pad;
    double tail_ms;            /* summed over the device rounds: time from the
                                  first to the last wave (round kernel) or
                                  workgroup (sweep kernels) of a launch that
                                  took work running out of it; the one-launch
                                  path of small batches adds nothing        */
} mih_query_stats;

/* Per-call counters of the linear scan. */
typedef struct mih_scan_stats {
    uint64_t pairs;            /* (code, query) distances computed            */
    uint64_t appended;         /* candidates kept as possible neighbours      */
    uint32_t reruns;           /* queries re-run with an exact capacity       */
    uint32_t pad;
    double elapsed_ms;         /* wall time of the call                        */
    double scan_kernel_ms;     /* HIP-event time of the scan kernel launches  */
    double sample_kernel_ms;   /* HIP-event time of the initial-bound kernel  */
} mih_scan_stats;

/*
 * Build the m substring tables of Algorithm 1 on the device.
 *   device codes : [n][bits/64], borrowed; it must stay valid and unchanged
 *                  until mih_free (candidates are verified against it).
 *   n            : number of codes, 0 <= n <= 2^32 - 2.
 *   bits         : 64, 128, 192 or 256.
 *   m            : number of substrings, 1 <= m <= MIH_M_MAX, with
 *                  ceil(bits / m) <= MIH_SUBSTRING_MAX.  Substring lengths are
 *                  floor(bits/m) or ceil(bits/m), the longer ones first, each
 *                  a run of contiguous bits (Section 2.1 and its footnote).
 *   opts         : NULL for defaults (AUTO modes, budget = free memory).
 *   out          : receives the index (owned by the library; release with
 *                  mih_free).  Untouched on error.
 */
mih_status mih_build(const uint64_t *codes, uint64_t n, uint32_t bits, uint32_t m,
                     const mih_build_opts *opts, void *stream, mih_index **out);

/*
 * Exact kNN of nq queries by multi-index hashing (Algorithm 3: per query, look
 * up the buckets that differ from the query's substring in exactly r' bits,
 * one table per step, growing r' until k codes within the searched radius are
 * found; Propositions 1 and 2 make the result exact).
 *   device queries     : [nq][bits/64].
 *   k                  : neighbours per query when k_per_query is NULL.
 *   device k_per_query : [nq] per-query k, or NULL.  Each k <= MIH_K_MAX.
 *   device out_ids, out_dists : [sum of k_i] each, layout as above.
 */
mih_status mih_knn(const mih_index *idx, const uint64_t *queries, uint32_t nq, uint32_t k,
                   const uint32_t *k_per_query, uint32_t *out_ids, uint32_t *out_dists,
                   void *stream);

/* As mih_knn, also filling *stats (may be NULL). */
mih_status mih_knn_ex(const mih_index *idx, const uint64_t *queries, uint32_t nq, uint32_t k,
                      const uint32_t *k_per_query, uint32_t *out_ids, uint32_t *out_dists,
                      void *stream, mih_query_stats *stats);

/*
 * Exact kNN by linear scan (the baseline of Section 5: the distance of every
 * code to every query, one xor and one popcount per 64 bits, Section 6).
 * Arguments as in mih_build and mih_knn; no index is needed.
 */
mih_status linscan_knn(const uint64_t *codes, uint64_t n, uint32_t bits,
                       const uint64_t *queries, uint32_t nq, uint32_t k,
                       const uint32_t *k_per_query, uint32_t *out_ids, uint32_t *out_dists,
                       void *stream);

/* As linscan_knn, also filling *stats (may be NULL). */
mih_status linscan_knn_ex(const uint64_t *codes, uint64_t n, uint32_t bits,
                          const uint64_t *queries, uint32_t nq, uint32_t k,
                          const uint32_t *k_per_query, uint32_t *out_ids, uint32_t *out_dists,
                          void *stream, mih_scan_stats *stats);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): linscan_knn with
 * every device buffer taken from a fixed array of MIH_NOALLOC_SCRATCH_BYTES
 * that the library holds on each GPU it has run this call on, from the first
 * such call until the process ends.  No hipMalloc, hipFree or other
 * allocating routine is called.  Results are those of linscan_knn.
 *   Arguments as in linscan_knn; the current device must be the stream's.
 *   A batch whose buffers do not fit half the array is scanned in slices of
 *   queries (one pass over the database per slice; a query with k <= 4096
 *   always fits); the other half takes the exact re-runs of queries whose
 *   candidate buffer overflowed.
 * Errors: as linscan_knn; MIH_ERR_CAPACITY (outputs incomplete) when the
 * exact re-run of a single query does not fit, i.e. when more than about
 * 16 M codes lie at or within that query's k-th distance.
 * Every call on one GPU shares that GPU's array and leaves it holding its
 * last contents: calls that overlap on one GPU (several host threads, or
 * several streams) race, so the caller serialises them. */
#define MIH_NOALLOC_SCRATCH_BYTES (256ull << 20)
mih_status linscan_knn_noalloc(const uint64_t *codes, uint64_t n, uint32_t bits,
                               const uint64_t *queries, uint32_t nq, uint32_t k,
                               const uint32_t *k_per_query, uint32_t *out_ids, uint32_t *out_dists,
                               void *stream);

/* Approximate kNN (Section 7): Algorithm 3 stopped early, returning the k
 * best of the codes met so far.
 *   max_radius      stop after the step that covers this radius, even if
 *                   fewer than k codes lie within it (every code within
 *                   max_radius is still found); 0xFFFFFFFF: no limit
 *   max_candidates  stop after the step during which this many distinct
 *                   codes have been met; 0: no limit
 * With neither limit reached the answer is mih_knn's.  Rows with fewer than
 * k codes met are padded with MIH_SENTINEL.  Other arguments as mih_knn_ex. */
mih_status mih_knn_approx(const mih_index *idx, const uint64_t *queries, uint32_t nq, uint32_t k,
                          const uint32_t *k_per_query, uint32_t max_radius, uint32_t max_candidates,
                          uint32_t *out_ids, uint32_t *out_dists, void *stream,
                          mih_query_stats *stats);

/* Release an index and its device memory.  NULL is ignored. */
void mih_free(mih_index *idx);

/* ---------------------------------------------------------------------
 * r-neighbour search (Section 2.2, Algorithm 2): every database code within
 * Hamming distance r of each query.  The number of results varies per
 * query, so they are returned in a result object owned by the library.
 *
 * Results of query i are entries [offsets[i], offsets[i+1]) of ids and
 * dists, in ascending (distance, id) order; offsets[0] = 0 and
 * offsets[nq] = total.  The three arrays are device memory owned by the
 * result and stay valid until mih_rnn_result_free.
 */
typedef struct mih_rnn_result mih_rnn_result;   /* opaque */

typedef struct mih_rnn_view {
    uint64_t total;              /* number of (query, code) results            */
    uint32_t nq, pad;
    const uint64_t *offsets;     /* device [nq + 1]                            */
    const uint32_t *ids;         /* device [total] (at least one entry)        */
    const uint32_t *dists;       /* device [total] (at least one entry)        */
} mih_rnn_view;

/* r-neighbours through the multi-index tables.  The search runs the steps of
 * Algorithm 3 up to step r, which by Proposition 2 covers every code within
 * distance r (it is Algorithm 2 with the tighter per-table radii of
 * Proposition 2).
 *   device queries    [nq][bits/64] (borrowed during the call)
 *   r                 radius for every query, used when r_per_query is NULL
 *   device r_per_query [nq] uint32 radii, or NULL; radii above bits mean bits
 *   host out          receives the result (NULL on error)
 * Errors: MIH_ERR_INVALID for a NULL index or out, misaligned or NULL
 * queries with nq > 0; MIH_ERR_NOMEM / MIH_ERR_DEVICE as elsewhere. */
mih_status mih_rnn(const mih_index *idx, const uint64_t *queries, uint32_t nq, uint32_t r,
                   const uint32_t *r_per_query, void *stream, mih_rnn_result **out);

/* As mih_rnn, also filling *stats (may be NULL). */
mih_status mih_rnn_ex(const mih_index *idx, const uint64_t *queries, uint32_t nq, uint32_t r,
                      const uint32_t *r_per_query, void *stream, mih_rnn_result **out,
                      mih_query_stats *stats);

/* r-neighbours by the linear scan: every (code, query) distance is computed.
 * Arguments as in linscan_knn and mih_rnn. */
mih_status linscan_rnn(const uint64_t *codes, uint64_t n, uint32_t bits,
                       const uint64_t *queries, uint32_t nq, uint32_t r,
                       const uint32_t *r_per_query, void *stream, mih_rnn_result **out);

/* Pointers and sizes of a result.  MIH_ERR_INVALID for NULL arguments. */
mih_status mih_rnn_result_view(const mih_rnn_result *res, mih_rnn_view *view);

/* Release a result and its device memory.  NULL is ignored. */
void mih_rnn_result_free(mih_rnn_result *res);

/* Static, human-readable name of a status. */
const char *mih_status_str(mih_status s);

/* Launch parameters of the multi-index search.  They change speed only; the
 * result of every query is the same for all of them. */
typedef struct mih_tuning {
    uint32_t probes_per_lane;  /* shell masks per lane per iteration: 4, 8 or 16 */
    uint32_t chunk;            /* shell masks per work item: a multiple of
                                  64 * probes_per_lane, at most 2^20           */
    uint32_t blocks_per_cu;    /* persistent workgroups per CU, 0 = all that fit */
    uint32_t occupancy_filter; /* DIRECT tables: 1 = test a one-bit-per-bucket
                                  occupancy map before reading the offsets   */
    uint32_t sweep_shift;      /* 0: off.  Else a round's group of queries at
                                  one step of a table of s >= 20 bits whose
                                  probes reach 2^s >> sweep_shift is run
                                  partition by partition of the key space   */
    uint32_t sweep_bits;       /* key bits per sweep partition, 10..32        */
    uint32_t lookahead;        /* 1..MIH_LOOKAHEAD_MAX: most steps (Algorithm 3)
                                  a query may run in one round.  Above 1, a
                                  round whose steps would leave waves of the
                                  search kernel idle also runs the following
                                  steps of its queries, lowest first, while
                                  its work items fit in the resident waves
                                  and its shell masks in four passes of
                                  them.  Exact searches only: approximate
                                  ones (mih_knn_approx) always use 1        */
    uint32_t sweep_queries;    /* swept steps on tables with an occupancy map
                                  (DIRECT with the filter, HEADS): queries
                                  per work item, a multiple of 64 in
                                  64..4096; the partitions there have
                                  2^min(sweep_bits, 18) values, whose
                                  occupancy bits a workgroup keeps in LDS   */
    uint32_t buffer_mult;      /* candidate-buffer entries per kNN query:
                                  buffer_mult * max(k, 256), 1..64.  Fewer
                                  entries admit more queries at once; a query
                                  whose buffer overflows is re-run with an
                                  exact capacity (same result, more time)   */
    uint32_t small_batch;      /* exact batches of at most this many queries
                                  (0..65536) whose expected work per query
                                  is small run in one launch: a workgroup
                                  per query takes every step and writes the
                                  top-k rows, with no host round trip      */
    uint32_t round_masks;      /* work quantum: the most shell masks one query
                                  probes in one device round (0: no limit); a
                                  larger step is continued over several
                                  rounds, so that the rounds of a serving
                                  loop stay short and requests that arrive
                                  meanwhile do not wait for a whole large
                                  step of the others.  Rounded up to whole
                                  work items (chunk); only steps within one
                                  quantum are then swept */
    uint32_t spill_codes;      /* 0 (off) or 256..: a bucket holding more
                                  codes than this, met by the round kernel,
                                  is cut into pieces of 1024 codes that any
                                  wave of the kernel may walk (waves out of
                                  work take them first), so that huge buckets
                                  of clustered codes do not leave one wave
                                  searching alone at the end of a round.
                                  Exact searches only */
} mih_tuning;

#define MIH_LOOKAHEAD_MAX 32u
#define MIH_LOOKAHEAD_DEFAULT 16u

/* Current tuning of an index (defaults after mih_build: 4, 8192, 0, the
 * occupancy filter on for DIRECT and HEADS tables of substrings of 26 bits
 * or more, sweep off, 18 sweep bits, lookahead MIH_LOOKAHEAD_DEFAULT, 256
 * sweep queries, buffer_mult 8, small_batch 512, round_masks 0,
 * spill_codes 0; HEADS tables
 * of substrings of 26 bits or more start at 4 probes per lane, chunk 8192
 * and sweeps with sweep_shift 3, 17 sweep bits and 4096 sweep queries). */
mih_status mih_get_tuning(const mih_index *idx, mih_tuning *tuning);

/* Replace the tuning; MIH_ERR_INVALID (index unchanged) if a field is out of
 * range.  Not thread-safe with concurrent mih_knn calls on the same index. */
mih_status mih_set_tuning(mih_index *idx, const mih_tuning *tuning);

/* Time mih_knn over a grid of tunings (probes_per_lane 4, 8, 16; chunk of
 * 2, 8, 32 or 128 times 64 * probes_per_lane; all workgroups that fit; with and
 * without the occupancy filter on DIRECT and HEADS tables; and, for
 * substrings of 20 bits or more, sweeps: on tables with an occupancy map
 * the partition kernel with 4096 sweep queries at (probes_per_lane,
 * sweep_bits, sweep_shift) = (4, 16, 3), (4, 17, 3), (4, 18, 3), (8, 17, 3)
 * and (4, 17, 4), otherwise sweep_shift 3 with 18 or 20 sweep
 * bits; the lookahead of the current tuning) on
 * the given sample of queries, time the three fastest twice more, then the
 * fastest with buffer_mult 4 and 16 twice each, then the fastest with
 * spill_codes 4096 and 32768 twice each (these last two changes must win
 * by 3%); keep the fastest in the
 * index and write it to *chosen (may be NULL).  Results do not depend on the tuning, so the
 * sample only has to look like the real queries (how far rounds run ahead
 * depends on the batch size: a sample as large as the real batches tunes
 * best).  Arguments as mih_knn. */
mih_status mih_autotune(mih_index *idx, const uint64_t *queries, uint32_t nq, uint32_t k,
                        const uint32_t *k_per_query, void *stream, mih_tuning *chosen);

/* ---- Choosing the number of substrings (Section 3.1; Section 6) -------
 *
 * Cost model of Eq. 6 for uniform codes, in units of one lookup: for each
 * table of s bits, (1 + n / 2^s) times the buckets within substring radius
 * floor(s r / bits).  Tables of unequal length (bits not divisible by m)
 * contribute their own terms; with s = bits / m for all tables this is
 * Eq. 6.  Returns 0 for m = 0 or m > bits. */
double mih_model_cost(uint64_t n, uint32_t bits, uint32_t m, uint32_t r);

/* Model radius of a kNN query over n uniform codes: the smallest r whose
 * expected count of codes within distance r, n L(bits, r) / 2^bits (Eq. 1),
 * is at least k; 0 for k = 0, bits when k >= n. */
uint32_t mih_model_radius(uint64_t n, uint32_t bits, uint32_t k);

#define MIH_M_TRIALS_MAX 16u

/* One candidate m timed by mih_choose_m. */
typedef struct mih_m_trial {
    uint32_t m;
    mih_status status;      /* MIH_OK, or why this m could not be timed     */
    double model_cost;      /* mih_model_cost at mih_model_radius(n, bits, k) */
    double search_ms;       /* wall time of mih_knn over the validation queries */
    double build_ms;        /* mih_build of this m                           */
    uint64_t device_bytes;  /* index memory of this m                        */
} mih_m_trial;

/* Selects m by timing (Section 6, "Number of Substrings"): for each
 * candidate m an index is built over the codes, mih_knn is run once to warm
 * up and once timed over the validation queries, and the index is freed.
 *   host candidates  [ncand] values of m, or NULL with ncand = 0 for the
 *                    default set: the integers nearest bits / log2 n (one
 *                    below, nearest, one above) and the minimiser of
 *                    mih_model_cost, each with ceil(bits/m) <= 32
 *   opts             build options for every candidate (NULL = defaults)
 *   host best_m      the candidate with the smallest search time
 *   host trials      [MIH_M_TRIALS_MAX] filled for each candidate, or NULL
 *   host ntrials     number of candidates tried
 * Codes and queries as in mih_build and mih_knn; one k for all queries.
 * Errors: MIH_ERR_INVALID for n < 2, nq = 0, k = 0 or k > MIH_K_MAX, an
 * invalid candidate or more than MIH_M_TRIALS_MAX of them; when no
 * candidate could be built and timed, the status of the last failure. */
mih_status mih_choose_m(const uint64_t *codes, uint64_t n, uint32_t bits, const uint64_t *queries,
                        uint32_t nq, uint32_t k, const uint32_t *candidates, uint32_t ncand,
                        const mih_build_opts *opts, void *stream, uint32_t *best_m,
                        mih_m_trial *trials, uint32_t *ntrials);

/* ---- Substring optimisation (Section 5.5) ------------------------------
 *
 * Co-occurrence counts of the code bits over n sample codes:
 *   device codes  [n][bits/64]
 *   host counts   [bits * bits]: counts[i * bits + j] = number of codes with
 *                 bits i and j both set (the diagonal holds the bit counts)
 * n < 2^31.  Errors: MIH_ERR_INVALID for NULL counts or bad bits. */
mih_status mih_bit_cooccurrence(const uint64_t *codes, uint64_t n, uint32_t bits, void *stream,
                                uint32_t *counts);

/* The greedy bit order of Section 5.5, from the counts above (host only).
 * With |Pearson correlation| between bits taken from the counts (0 for a
 * constant bit): substring 0 starts with first_bit; substring j starts with
 * the unused bit most correlated with the first bit of substring j - 1; then
 * the substrings, in turn, take the unused bit whose largest correlation
 * with the bits they already hold is smallest, until each has its length
 * (floor or ceil of bits / m, longer ones first).  Ties go to the lowest bit.
 *   host bit_order [bits]: the order for mih_build_opts.bit_order. */
mih_status mih_greedy_bit_order(const uint32_t *counts, uint64_t n, uint32_t bits, uint32_t m,
                                uint32_t first_bit, uint16_t *bit_order);

/* ---- Serving: continuous batching over a built index ------------------
 *
 * A server keeps per-query search state for up to max_queries queries
 * resident on the device and a pool of candidate-buffer memory.  Requests
 * (each a set of queries with their k) are queued by mih_server_submit and
 * admitted first in, first out, query by query, whenever a slot and buffer
 * memory are free; every mih_server_step runs one device round that advances
 * every admitted query by one search step, so requests submitted while
 * others are in flight share the device with them.  The result of each query
 * is the same as mih_knn's, whatever else is in flight.  A server is not
 * thread-safe; one index may serve several servers and mih_knn calls. */
typedef struct mih_server mih_server;

typedef struct mih_server_opts {
    uint32_t max_queries;      /* query slots resident on the device, >= 1      */
    uint32_t use_graph;        /* 1: replay each round as a captured hipGraph    */
    uint64_t buffer_entries;   /* candidate-buffer pool in 8-byte entries;
                                  0 = 8192 per slot.  A query with k needs
                                  max(2048, 8 k) entries while in flight.        */
} mih_server_opts;

typedef struct mih_server_stats {
    uint64_t probes, candidates;   /* summed over all rounds so far             */
    uint64_t completed_requests;
    uint32_t rounds;
    uint32_t in_flight;            /* admitted queries not yet finished          */
    uint32_t pending_queries;      /* submitted queries waiting for admission    */
    uint32_t reruns;
    double search_kernel_ms;
} mih_server_stats;

/* Create a server on `stream` (a hipStream_t, used by every later call).
 * The index must outlive the server.  opts NULL: 4096 slots, graphs on. */
mih_status mih_server_create(const mih_index *idx, const mih_server_opts *opts, void *stream,
                             mih_server **out);

/* Queue a request.  device queries [nq][bits/64] must stay valid and
 * unchanged until the request completes; results go to device out_ids /
 * out_dists in the layout of mih_knn (row i at k_0 + ... + k_{i-1}).
 * host_k_per_query: per-query k in host memory, or NULL for k.  Each
 * k <= MIH_K_MAX.  Returns MIH_ERR_CAPACITY (nothing queued) when a query's
 * buffer could never fit the pool.  Does not wait for the device. */
mih_status mih_server_submit(mih_server *srv, const uint64_t *queries, uint32_t nq, uint32_t k,
                             const uint32_t *host_k_per_query, uint32_t *out_ids,
                             uint32_t *out_dists, uint64_t *ticket);

/* Admit what fits, run one round, finalize finished queries.  Writes up to
 * max_completed tickets of requests completed since the last call to
 * host `completed` and their number to *n_completed (more stay queued for
 * the next call).  Blocking: outputs of reported requests are on the device
 * when it returns. */
mih_status mih_server_step(mih_server *srv, uint64_t *completed, uint32_t max_completed,
                           uint32_t *n_completed);

/* *done = 1 when the request has completed (its outputs are written). */
mih_status mih_server_poll(const mih_server *srv, uint64_t ticket, int *done);

mih_status mih_server_get_stats(mih_server *srv, mih_server_stats *stats);

/* Release a server (pending and in-flight requests are dropped). */
void mih_server_destroy(mih_server *srv);

/* Measurement helper (not part of the search): the device's rate of
 * independent random 64-byte line reads, the kind of read the multi-index
 * search is made of, so that its fetched lines per second can be put beside
 * a ceiling.  Reads about `reads` 8-byte words, each from a pseudo-random
 * line of device array[words] (words >= 8, 8-byte aligned), every lane
 * keeping `depth` (1, 4, 8 or 16) loads in flight; the words read are
 * summed into device *sink (one 8-byte word) so that no load is dropped.
 * The lanes take a whole number of rounds of `depth` reads, so slightly more
 * than `reads` may be read: 256 x 8 x 256 lanes on 256 CUs.
 * *ms (host) receives the kernel time.  Errors: MIH_ERR_INVALID for NULL
 * pointers, words < 8, reads = 0 or another depth. */
mih_status mih_random_read_rate(const uint64_t *array, uint64_t words, uint64_t reads, uint32_t depth,
                                uint64_t *sink, void *stream, double *ms);

/* Fill *info (host memory) with the index's shape and modes. */
mih_status mih_index_get_info(const mih_index *idx, mih_index_info *info);

/* Fill *view (host memory) with device pointers to table j (0 <= j < m). */
mih_status mih_index_table(const mih_index *idx, uint32_t j, mih_table_view *view);

#ifdef __cplusplus
}
#endif

#endif /* MIH_H */
