// C-ABI entry points (include/mih.h): argument checks, device memory
// planning, the host side of the round loop, and the exact re-run of queries
// whose candidate buffer overflowed.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "engine.h"

namespace {

using clk = std::chrono::steady_clock;

double ms_since(clk::time_point t0)
{
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

// Status of a failed HIP call; with MIH_DEBUG set in the environment the
// call site and the runtime's message go to stderr.
mih_status from_hip_at(hipError_t e, int line)
{
    if (e == hipSuccess) return MIH_OK;
    static const bool debug = std::getenv("MIH_DEBUG") != nullptr;
    if (debug) std::fprintf(stderr, "libmih: api.hip:%d: %s\n", line, hipGetErrorString(e));
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return MIH_ERR_NOMEM;
    return MIH_ERR_DEVICE;
}
#define from_hip(e) from_hip_at((e), __LINE__)

#define MIH_TRY(expr)                              \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) {                    \
            (void)hipGetLastError();               \
            return from_hip(e_);                   \
        }                                          \
    } while (0)

#define MIH_TRY_STATUS(expr)                       \
    do {                                           \
        mih_status st_ = (expr);                   \
        if (st_ != MIH_OK) return st_;             \
    } while (0)

bool bits_ok(uint32_t bits) { return bits == 64 || bits == 128 || bits == 192 || bits == 256; }

// How many tables can keep an inline copy of the codes (per_table bytes
// each) once `need` bytes are committed, within `budget`.
uint32_t inline_tables_fit(uint64_t need, uint64_t budget, uint64_t per_table, uint32_t m)
{
    if (per_table == 0) return m;
    if (need >= budget) return 0;
    return (uint32_t)std::min<uint64_t>(m, (budget - need) / per_table);
}

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

uint32_t ceil_log2(uint64_t x)
{
    uint32_t b = 0;
    while ((1ull << b) < x) ++b;
    return b;
}

uint32_t num_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 256;
    return (uint32_t)cus;
}

// A device region carved into aligned pieces.  With base == nullptr it only
// measures the size that the same sequence of take() calls needs.
struct Carver {
    char *base = nullptr;
    uint64_t used = 0;
    template <class T>
    T *take(uint64_t count)
    {
        uint64_t bytes = align_up((count ? count : 1) * sizeof(T), 256);
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += bytes;
        return p;
    }
};

// Grow-only device scratch.
struct Scratch {
    void *ptr = nullptr;
    uint64_t size = 0;
    hipError_t ensure(uint64_t bytes)
    {
        if (bytes <= size) return hipSuccess;
        if (ptr) { (void)hipFree(ptr); ptr = nullptr; size = 0; }
        hipError_t e = hipMalloc(&ptr, bytes);
        if (e == hipSuccess) size = bytes;
        else (void)hipGetLastError();
        return e;
    }
    void release()
    {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        size = 0;
    }
};

// Device memory of one linear-scan call: allocated per call, or carved from
// a caller's region (base != nullptr), in which case nothing is allocated and
// a request that does not fit fails with MIH_ERR_CAPACITY.
struct Arena {
    char *base = nullptr;
    uint64_t size = 0, used = 0;
    bool fits(uint64_t bytes) const { return used <= size && bytes <= size - used; }
};

// Memory for `bytes` from the arena (marked used until release) or from a
// fresh allocation held in `own`.
mih_status arena_take(Arena *arena, Scratch &own, uint64_t bytes, char *&p)
{
    if (arena) {
        if (!arena->fits(bytes)) return MIH_ERR_CAPACITY;
        p = arena->base + arena->used;
        arena->used += bytes;
        return MIH_OK;
    }
    MIH_TRY(own.ensure(bytes));
    p = (char *)own.ptr;
    return MIH_OK;
}

// A pair of HIP events around launches on one stream (disabled unless the
// caller asked for statistics).
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    bool on = false;
    explicit EventPair(bool enable)
    {
        if (!enable) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            (void)hipGetLastError();
            return;
        }
        on = true;
    }
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    void begin(hipStream_t s) { if (on) (void)hipEventRecord(a, s); }
    void end(hipStream_t s) { if (on) (void)hipEventRecord(b, s); }
    // milliseconds between the two records (waits for the second)
    double ms()
    {
        float t = 0;
        if (!on || hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&t, a, b) != hipSuccess) {
            (void)hipGetLastError();
            return 0.0;
        }
        return t;
    }
};

// Host description of a batch of queries.
struct BatchSpec {
    const uint64_t *queries = nullptr;   // device [nq][W]
    uint32_t nq = 0;
    std::vector<uint32_t> k;             // per query
    std::vector<uint64_t> row_off;       // output offset per query
    std::vector<uint32_t> cap;           // buffer capacity per query
    const uint32_t *tau0 = nullptr;      // device, or null
    // r-neighbour batches: hits go to this collector, query i as query
    // row_off[i] of the request, instead of into top-k rows
    mih::RnnCollector *rnn = nullptr;
};

struct BatchBufs {
    QueryBatch qb;
    uint64_t *row_off;
    uint32_t *ovf_list, *ovf_count;
    uint32_t *t, *active0, *active1, *next_t;
    mih::Group *groups;
    mih::Control *ctrl;
    unsigned long long *work, *stats;
};

void carve_batch(Carver &c, const BatchSpec &b, uint32_t bits, uint32_t W, uint64_t buf_words,
                 uint32_t ngroups, BatchBufs &B)
{
    const uint32_t nq = b.nq;
    B.qb.k = c.take<uint32_t>(nq);
    B.qb.tau = c.take<uint32_t>((uint64_t)nq + 16);   // the scan reads whole batches of 16
    B.qb.count = c.take<uint32_t>(nq);
    B.qb.cap = c.take<uint32_t>(nq);
    B.qb.buf_off = c.take<uint64_t>(nq);
    B.qb.hist = c.take<uint32_t>((uint64_t)nq * (bits + 1));
    B.qb.buf = c.take<uint64_t>(buf_words);
    B.row_off = c.take<uint64_t>(nq);
    B.ovf_list = c.take<uint32_t>(nq);
    B.ovf_count = c.take<uint32_t>(1);
    B.t = c.take<uint32_t>(nq);
    B.active0 = c.take<uint32_t>(nq);
    B.active1 = c.take<uint32_t>(nq);
    B.next_t = c.take<uint32_t>(nq);
    B.groups = c.take<mih::Group>(ngroups);
    B.ctrl = c.take<mih::Control>(1);
    B.work = c.take<unsigned long long>(1);
    B.stats = c.take<unsigned long long>(4);
    B.qb.queries = b.queries;
    B.qb.nq = nq;
    B.qb.bits = bits;
    (void)W;
}

uint64_t buffer_words(const BatchSpec &b, std::vector<uint64_t> &buf_off)
{
    buf_off.resize(b.nq);
    uint64_t acc = 0;
    for (uint32_t i = 0; i < b.nq; ++i) { buf_off[i] = acc; acc += b.cap[i]; }
    return acc;
}

hipError_t upload(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (!bytes) return hipSuccess;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);   // the host vectors are freed soon after
}

hipError_t download(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (!bytes) return hipSuccess;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

// Per-query k as host vector; validates k <= MIH_K_MAX.
mih_status read_k(uint32_t nq, uint32_t k, const uint32_t *k_per_query, hipStream_t s,
                  std::vector<uint32_t> &out)
{
    out.assign(nq, k);
    if (k_per_query && nq) MIH_TRY(download(out.data(), k_per_query, sizeof(uint32_t) * nq, s));
    for (uint32_t v : out)
        if (v > MIH_K_MAX) return MIH_ERR_UNSUPPORTED;
    return MIH_OK;
}

void row_offsets(const std::vector<uint32_t> &k, std::vector<uint64_t> &off)
{
    off.resize(k.size());
    uint64_t acc = 0;
    for (size_t i = 0; i < k.size(); ++i) { off[i] = acc; acc += k[i]; }
}

uint32_t scan_cap(uint32_t k) { return k == 0 ? 0u : std::max<uint32_t>(4096u, 16u * k); }

}  // namespace

// ============================================================== the index

struct mih_rnn_result {
    mih::RnnOut out;
    ~mih_rnn_result() { mih::free_rnn_out(out); }
};

hipError_t mih_index::alloc(void **p, uint64_t bytes)
{
    hipError_t e = hipMalloc(p, bytes ? bytes : 4);
    if (e != hipSuccess) { (void)hipGetLastError(); *p = nullptr; return e; }
    allocs.push_back(*p);
    device_bytes += bytes;
    return hipSuccess;
}

mih_index::~mih_index()
{
    batch_engine.reset();
    if (small_dev) (void)hipFree(small_dev);
    if (small_host) (void)hipHostFree(small_host);
    for (void *p : allocs) (void)hipFree(p);
}

namespace {

// ---------------------------------------------------------------- linscan

mih_status linscan_batch(const uint64_t *codes, uint64_t n, uint32_t bits, BatchSpec &b,
                         uint32_t *out_ids, uint32_t *out_dists, hipStream_t s, int depth,
                         mih_scan_stats *stats, Arena *arena = nullptr);

// Bytes of device memory linscan_batch carves for a batch.
uint64_t linscan_batch_bytes(const BatchSpec &b, uint32_t bits)
{
    const uint32_t W = bits / 64;
    std::vector<uint64_t> buf_off;
    const uint64_t words = buffer_words(b, buf_off);
    BatchBufs B;
    Carver c0;
    carve_batch(c0, b, bits, W, words, 1, B);
    c0.take<uint64_t>((uint64_t)mih::linscan_pad(b.nq) * W);
    return c0.used;
}

// The queries of `rb` from position i0 on that fit the arena with one
// batch (at least one; 0 if not even one fits).
uint32_t rerun_slice(const BatchSpec &rb, uint32_t i0, uint32_t bits, const Arena &arena)
{
    uint32_t lo = 0, hi = rb.nq - i0;   // the largest count that fits, by bisection
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        BatchSpec t;
        t.nq = mid;
        t.cap.assign(rb.cap.begin() + i0, rb.cap.begin() + i0 + mid);
        if (arena.fits(linscan_batch_bytes(t, bits))) lo = mid; else hi = mid - 1;
    }
    return lo;
}

mih_status rerun_linscan(const uint64_t *codes, uint64_t n, uint32_t bits, const BatchSpec &b,
                         BatchBufs &B, uint32_t *out_ids, uint32_t *out_dists, hipStream_t s,
                         int depth, mih_scan_stats *stats, Arena *arena)
{
    uint32_t novf = 0;
    MIH_TRY(download(&novf, B.ovf_count, sizeof(uint32_t), s));
    if (novf == 0) return MIH_OK;
    if (depth > 2) return MIH_ERR_DEVICE;   // an exact re-run cannot overflow
    if (stats) stats->reruns += novf;
    const uint32_t W = bits / 64;
    std::vector<uint32_t> list(novf);
    MIH_TRY(download(list.data(), B.ovf_list, sizeof(uint32_t) * novf, s));
    Carver c0;
    c0.take<uint32_t>(novf); c0.take<uint32_t>(novf); c0.take<uint32_t>(novf);
    c0.take<uint64_t>((uint64_t)novf * W);
    Scratch tmp;
    const uint64_t arena_mark = arena ? arena->used : 0;
    Carver c;
    MIH_TRY_STATUS(arena_take(arena, tmp, c0.used, c.base));
    uint32_t *dlist = c.take<uint32_t>(novf);
    uint32_t *dtau = c.take<uint32_t>(novf);
    uint32_t *dcap = c.take<uint32_t>(novf);
    uint64_t *dq = c.take<uint64_t>((uint64_t)novf * W);
    mih_status st = MIH_OK;
    do {
        if (upload(dlist, list.data(), sizeof(uint32_t) * novf, s) != hipSuccess) { st = MIH_ERR_DEVICE; break; }
        if (mih::exact_bounds(B.qb, dlist, novf, dtau, dcap, s) != hipSuccess ||
            mih::gather_rows(b.queries, dlist, novf, W, dq, s) != hipSuccess) { st = MIH_ERR_DEVICE; break; }
        BatchSpec rb;
        rb.queries = dq;
        rb.nq = novf;
        rb.tau0 = dtau;
        rb.rnn = b.rnn;
        rb.cap.resize(novf);
        if (download(rb.cap.data(), dcap, sizeof(uint32_t) * novf, s) != hipSuccess) { st = MIH_ERR_DEVICE; break; }
        rb.k.resize(novf);
        rb.row_off.resize(novf);
        for (uint32_t i = 0; i < novf; ++i) {
            rb.k[i] = b.k[list[i]];
            rb.row_off[i] = b.row_off[list[i]];
            if (rb.cap[i] == 0 && rb.k[i]) rb.cap[i] = 1;
        }
        if (!arena) {
            st = linscan_batch(codes, n, bits, rb, out_ids, out_dists, s, depth + 1, stats);
            break;
        }
        // in a fixed region the re-run goes in slices of queries that fit
        for (uint32_t i0 = 0; i0 < novf && st == MIH_OK;) {
            const uint32_t cnt = rerun_slice(rb, i0, bits, *arena);
            if (cnt == 0) { st = MIH_ERR_CAPACITY; break; }
            BatchSpec sb;
            sb.queries = rb.queries + (uint64_t)i0 * W;
            sb.nq = cnt;
            sb.tau0 = rb.tau0 + i0;
            sb.rnn = rb.rnn;
            sb.cap.assign(rb.cap.begin() + i0, rb.cap.begin() + i0 + cnt);
            sb.k.assign(rb.k.begin() + i0, rb.k.begin() + i0 + cnt);
            sb.row_off.assign(rb.row_off.begin() + i0, rb.row_off.begin() + i0 + cnt);
            st = linscan_batch(codes, n, bits, sb, out_ids, out_dists, s, depth + 1, stats, arena);
            i0 += cnt;
        }
    } while (0);
    (void)hipStreamSynchronize(s);
    tmp.release();
    if (arena) arena->used = arena_mark;
    return st;
}

mih_status linscan_batch(const uint64_t *codes, uint64_t n, uint32_t bits, BatchSpec &b,
                         uint32_t *out_ids, uint32_t *out_dists, hipStream_t s, int depth,
                         mih_scan_stats *stats, Arena *arena)
{
    if (b.nq == 0) return MIH_OK;
    const uint32_t W = bits / 64;
    std::vector<uint64_t> buf_off;
    const uint64_t words = buffer_words(b, buf_off);
    BatchBufs B;
    const uint64_t qrows = mih::linscan_pad(b.nq);
    Scratch mem;
    const uint64_t arena_mark = arena ? arena->used : 0;
    Carver c;
    MIH_TRY_STATUS(arena_take(arena, mem, linscan_batch_bytes(b, bits), c.base));
    carve_batch(c, b, bits, W, words, 1, B);
    uint64_t *qpad = c.take<uint64_t>(qrows * W);
    mih_status st = MIH_OK;
    do {
        // the scan reads queries in whole batches: a zero-padded copy
        hipError_t e = mih::fill_u64(qpad, qrows * W, 0ull, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(qpad, b.queries, sizeof(uint64_t) * W * b.nq, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = upload((void *)B.qb.k, b.k.data(), sizeof(uint32_t) * b.nq, s);
        if (e == hipSuccess) e = upload((void *)B.qb.cap, b.cap.data(), sizeof(uint32_t) * b.nq, s);
        if (e == hipSuccess) e = upload((void *)B.qb.buf_off, buf_off.data(), sizeof(uint64_t) * b.nq, s);
        if (e == hipSuccess) e = upload(B.row_off, b.row_off.data(), sizeof(uint64_t) * b.nq, s);
        mih::LinscanArgs L;
        L.codes = codes;
        L.n = n;
        L.qb = B.qb;
        L.queries_padded = qpad;
        L.W = W;
        uint32_t kmax = 0;
        for (uint32_t v : b.k) kmax = std::max(kmax, v);
        uint64_t sample = std::min<uint64_t>(n, std::max<uint64_t>(65536, 256ull * kmax));
        if (sample > (1ull << 20)) sample = 1ull << 20;
        EventPair ev_sample(stats != nullptr), ev_scan(stats != nullptr);
        ev_sample.begin(s);
        if (e == hipSuccess) e = mih::linscan_init(L, sample, b.tau0, s);
        ev_sample.end(s);
        ev_scan.begin(s);
        if (e == hipSuccess) e = mih::linscan_run(L, num_cus(), s);
        ev_scan.end(s);
        mih::FinalArgs F;
        F.qb = B.qb;
        F.row_off = B.row_off;
        F.out_ids = out_ids;
        F.out_dists = out_dists;
        F.overflow_list = B.ovf_list;
        F.overflow_count = B.ovf_count;
        if (e == hipSuccess) e = mih::find_overflow(F, s);
        if (e == hipSuccess && !b.rnn) e = mih::finalize_topk(F, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess && b.rnn) {
            // every query that did not overflow holds all its hits
            std::vector<uint32_t> cnt(b.nq), query, count;
            std::vector<uint64_t> src;
            e = download(cnt.data(), B.qb.count, sizeof(uint32_t) * b.nq, s);
            for (uint32_t i = 0; i < b.nq && e == hipSuccess; ++i) {
                if (cnt[i] > b.cap[i]) continue;
                query.push_back((uint32_t)b.row_off[i]);
                src.push_back(buf_off[i]);
                count.push_back(cnt[i]);
            }
            if (e == hipSuccess) e = b.rnn->add(B.qb.buf, query, src, count, s);
        }
        if (e != hipSuccess) { (void)hipGetLastError(); st = from_hip(e); break; }
        if (stats) {
            stats->sample_kernel_ms += ev_sample.ms();
            stats->scan_kernel_ms += ev_scan.ms();
            stats->pairs += n * (uint64_t)b.nq;
            std::vector<uint32_t> cnt(b.nq);
            if (download(cnt.data(), B.qb.count, sizeof(uint32_t) * b.nq, s) == hipSuccess)
                for (uint32_t i = 0; i < b.nq; ++i) stats->appended += cnt[i];
        }
        st = rerun_linscan(codes, n, bits, b, B, out_ids, out_dists, s, depth, stats, arena);
    } while (0);
    (void)hipStreamSynchronize(s);
    mem.release();
    if (arena) arena->used = arena_mark;
    return st;
}

// ---------------------------------------------------------------- MIH

bool use_graphs()
{
    static const bool off = std::getenv("MIH_NO_GRAPH") != nullptr;
    return !off;
}

// Runs one request of nq queries through an engine until it completes.
mih_status engine_batch(mih::Engine &eng, const uint64_t *queries, uint32_t nq,
                        const std::vector<uint32_t> &k, const std::vector<uint64_t> &row_off,
                        uint32_t *out_ids, uint32_t *out_dists, uint32_t max_t = 0xFFFFFFFFu,
                        uint32_t budget = 0)
{
    std::vector<uint64_t> completed;
    eng.set_count_unique(budget != 0);
    eng.set_lookahead(max_t == 0xFFFFFFFFu && budget == 0);
    eng.submit(queries, nq, k.data(), row_off.data(), out_ids, out_dists, max_t, budget);
    uint64_t guard = 0;
    while (!eng.idle()) {
        MIH_TRY(eng.step(completed));
        if (++guard > (1ull << 24)) return MIH_ERR_DEVICE;   // cannot happen: every round advances
    }
    return MIH_OK;
}

void copy_stats(const mih::EngineStats &es, clk::time_point t0, mih_query_stats *stats)
{
    stats->probes = es.probes;
    stats->candidates = es.candidates;
    stats->appended = es.appended;
    stats->steps = es.steps;
    stats->rounds = es.rounds;
    stats->reruns = es.reruns;
    stats->search_kernel_ms = es.search_kernel_ms;
    stats->search_launches = es.search_launches;
    stats->tail_ms = es.tail_ms;
    stats->elapsed_ms = ms_since(t0);
}

// Per-query radius as a host vector.
mih_status read_radius(uint32_t nq, uint32_t r, const uint32_t *r_per_query, hipStream_t s,
                       std::vector<uint32_t> &out)
{
    out.assign(nq, r);
    if (r_per_query && nq) MIH_TRY(download(out.data(), r_per_query, sizeof(uint32_t) * nq, s));
    return MIH_OK;
}

mih_status check_query_args(uint32_t bits, const uint64_t *queries, uint32_t nq,
                            const uint32_t *out_ids, const uint32_t *out_dists)
{
    if (!bits_ok(bits)) return MIH_ERR_INVALID;
    if (nq && !queries) return MIH_ERR_INVALID;
    if (nq && (!out_ids || !out_dists)) return MIH_ERR_INVALID;
    if (((uintptr_t)queries & 7) != 0) return MIH_ERR_INVALID;
    return MIH_OK;
}

}  // namespace

namespace mih {

// linscan_knn with every buffer carved from [base, base + size): slices of
// queries whose first pass fits in half the region, the other half left to
// the exact re-runs of overflowed queries.  Allocates no device memory.
mih_status linscan_check_args(const uint64_t *codes, uint64_t n, uint32_t bits,
                              const uint64_t *queries, uint32_t nq, uint32_t k,
                              const uint32_t *k_per_query, const uint32_t *out_ids,
                              const uint32_t *out_dists)
{
    MIH_TRY_STATUS(check_query_args(bits, queries, nq, out_ids, out_dists));
    if (n > 0xFFFFFFFEull || (n && !codes) || ((uintptr_t)codes & 7) != 0) return MIH_ERR_INVALID;
    if (!k_per_query && k > MIH_K_MAX) return MIH_ERR_UNSUPPORTED;
    return MIH_OK;
}

mih_status linscan_knn_in_region(const uint64_t *codes, uint64_t n, uint32_t bits,
                                 const uint64_t *queries, uint32_t nq, uint32_t k,
                                 const uint32_t *k_per_query, uint32_t *out_ids,
                                 uint32_t *out_dists, hipStream_t s, char *base, uint64_t size)
{
    MIH_TRY_STATUS(linscan_check_args(codes, n, bits, queries, nq, k, k_per_query, out_ids, out_dists));
    if (!base || ((uintptr_t)base & 255) != 0) return MIH_ERR_INVALID;
    const uint32_t W = bits / 64;
    BatchSpec all;
    all.queries = queries;
    all.nq = nq;
    MIH_TRY_STATUS(read_k(nq, k, k_per_query, s, all.k));
    row_offsets(all.k, all.row_off);
    all.cap.resize(nq);
    for (uint32_t i = 0; i < nq; ++i) all.cap[i] = scan_cap(all.k[i]);
    if (n == 0) {
        const uint64_t total = all.row_off.empty() ? 0 : all.row_off.back() + all.k.back();
        MIH_TRY(mih::fill_u32(out_ids, total, MIH_SENTINEL, s));
        MIH_TRY(mih::fill_u32(out_dists, total, MIH_SENTINEL, s));
        MIH_TRY(hipStreamSynchronize(s));
        return MIH_OK;
    }
    Arena first;   // the half of the region a slice's first pass may use
    first.base = base;
    first.size = size / 2 / 256 * 256;
    for (uint32_t i0 = 0; i0 < nq;) {
        const uint32_t cnt = rerun_slice(all, i0, bits, first);
        if (cnt == 0) return MIH_ERR_CAPACITY;
        BatchSpec b;
        b.queries = queries + (uint64_t)i0 * W;
        b.nq = cnt;
        b.k.assign(all.k.begin() + i0, all.k.begin() + i0 + cnt);
        b.row_off.assign(all.row_off.begin() + i0, all.row_off.begin() + i0 + cnt);
        b.cap.assign(all.cap.begin() + i0, all.cap.begin() + i0 + cnt);
        Arena whole;
        whole.base = base;
        whole.size = size;
        MIH_TRY_STATUS(linscan_batch(codes, n, bits, b, out_ids, out_dists, s, 0, nullptr, &whole));
        i0 += cnt;
    }
    return MIH_OK;
}

}  // namespace mih

// ============================================================== C ABI

extern "C" {

const char *mih_status_str(mih_status s)
{
    switch (s) {
    case MIH_OK: return "ok";
    case MIH_ERR_INVALID: return "invalid argument";
    case MIH_ERR_NOMEM: return "out of device memory";
    case MIH_ERR_DEVICE: return "device error";
    case MIH_ERR_UNSUPPORTED: return "unsupported";
    case MIH_ERR_CAPACITY: return "no capacity";
    }
    return "unknown status";
}

mih_status linscan_knn(const uint64_t *codes, uint64_t n, uint32_t bits, const uint64_t *queries,
                       uint32_t nq, uint32_t k, const uint32_t *k_per_query, uint32_t *out_ids,
                       uint32_t *out_dists, void *stream)
{
    return linscan_knn_ex(codes, n, bits, queries, nq, k, k_per_query, out_ids, out_dists, stream,
                          nullptr);
}

mih_status linscan_knn_ex(const uint64_t *codes, uint64_t n, uint32_t bits, const uint64_t *queries,
                          uint32_t nq, uint32_t k, const uint32_t *k_per_query, uint32_t *out_ids,
                          uint32_t *out_dists, void *stream, mih_scan_stats *stats)
{
    auto t0 = clk::now();
    if (stats) std::memset(stats, 0, sizeof(*stats));
    MIH_TRY_STATUS(check_query_args(bits, queries, nq, out_ids, out_dists));
    if (n > 0xFFFFFFFEull || (n && !codes) || ((uintptr_t)codes & 7) != 0) return MIH_ERR_INVALID;
    if (!k_per_query && k > MIH_K_MAX) return MIH_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    BatchSpec b;
    b.queries = queries;
    b.nq = nq;
    MIH_TRY_STATUS(read_k(nq, k, k_per_query, s, b.k));
    row_offsets(b.k, b.row_off);
    b.cap.resize(nq);
    for (uint32_t i = 0; i < nq; ++i) b.cap[i] = scan_cap(b.k[i]);
    if (n == 0) {
        // nothing to scan: every row is padding
        uint64_t total = b.row_off.empty() ? 0 : b.row_off.back() + b.k.back();
        MIH_TRY(mih::fill_u32(out_ids, total, MIH_SENTINEL, s));
        MIH_TRY(mih::fill_u32(out_dists, total, MIH_SENTINEL, s));
        MIH_TRY(hipStreamSynchronize(s));
        return MIH_OK;
    }
    mih_status st = linscan_batch(codes, n, bits, b, out_ids, out_dists, s, 0, stats);
    if (stats) stats->elapsed_ms = ms_since(t0);
    return st;
}

mih_status mih_build(const uint64_t *codes, uint64_t n, uint32_t bits, uint32_t m,
                     const mih_build_opts *opts, void *stream, mih_index **out)
{
    auto t0 = clk::now();
    if (!out) return MIH_ERR_INVALID;
    if (!bits_ok(bits) || m < 1 || m > MIH_M_MAX || m > bits) return MIH_ERR_INVALID;
    if ((bits + m - 1) / m > MIH_SUBSTRING_MAX) return MIH_ERR_UNSUPPORTED;
    if (n > 0xFFFFFFFEull || (n && !codes) || ((uintptr_t)codes & 7) != 0) return MIH_ERR_INVALID;
    mih_build_opts o = {MIH_TABLE_AUTO, MIH_CODES_AUTO, 0, nullptr, 0, nullptr};
    if (opts) o = *opts;
    if (o.bit_order) {
        // a permutation of 0 .. bits-1
        std::vector<uint8_t> seen(bits, 0);
        for (uint32_t p = 0; p < bits; ++p) {
            if (o.bit_order[p] >= bits || seen[o.bit_order[p]]) return MIH_ERR_INVALID;
            seen[o.bit_order[p]] = 1;
        }
    }
    if (o.table_mode > MIH_TABLE_HEADS || o.codes_mode > MIH_CODES_MIXED) return MIH_ERR_INVALID;
    if (o.codes_mode == MIH_CODES_MIXED && (o.inline_tables < 1 || o.inline_tables >= m)) return MIH_ERR_INVALID;
    // GROUPED tables scan, and HEADS tables read, the codes in table order
    if ((o.table_mode == MIH_TABLE_GROUPED || o.table_mode == MIH_TABLE_HEADS) &&
        (o.codes_mode == MIH_CODES_INDIRECT || o.codes_mode == MIH_CODES_MIXED))
        return MIH_ERR_INVALID;
    if (o.table_mode == MIH_TABLE_HEADS && bits != 64) return MIH_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;

    mih_index *ix = new (std::nothrow) mih_index();
    if (!ix) return MIH_ERR_NOMEM;
    (void)hipGetDevice(&ix->device);
    if (o.autotune_cache) ix->autotune_cache = o.autotune_cache;
    ix->codes = codes;
    ix->n = n;
    ix->bits = bits;
    ix->W = bits / 64;
    ix->m = m;
    const uint32_t W = ix->W;
    {
        uint32_t base = bits / m, extra = bits % m, st = 0;
        ix->t_all = 0xFFFFFFFFu;
        for (uint32_t p = 0; p < bits; ++p) ix->bit_order[p] = o.bit_order ? o.bit_order[p] : (uint16_t)p;
        for (uint32_t j = 0; j < m; ++j) {
            ix->len[j] = base + (j < extra ? 1 : 0);
            ix->start[j] = st;
            st += ix->len[j];
            ix->t_all = std::min(ix->t_all, m * ix->len[j] + j);
        }
    }
    const uint32_t lg = ceil_log2(n + 1);
    uint64_t direct_bytes = 0, sorted_bytes = 0, grouped_bytes = 0, heads_bytes = 0, max_entries = n + 1;
    for (uint32_t j = 0; j < m; ++j) {
        uint32_t p = lg > 3 ? lg - 3 : 1;
        if (p > ix->len[j]) p = ix->len[j];
        if (p < 1) p = 1;
        ix->dir_bits[j] = p;
        direct_bytes += ((1ull << ix->len[j]) + 1) * 4 + std::max<uint64_t>((1ull << ix->len[j]) / 32, 1) * 4;
        grouped_bytes += std::max<uint64_t>((1ull << ix->len[j]) / 32, 1) * 8;
        heads_bytes += ((1ull << ix->len[j]) + 1) * sizeof(BucketHead) +
                       std::max<uint64_t>((1ull << ix->len[j]) / 32, 1) * 4;
        sorted_bytes += n * 4 + ((1ull << p) + 1) * 4;
        max_entries = std::max<uint64_t>(max_entries, (1ull << ix->len[j]) + 1);
    }
    const uint64_t ids_bytes = (uint64_t)m * n * 4;
    const uint64_t table_inline_bytes = n * 8 * W;   // one table's copy of the codes
    const uint64_t temp_bytes = 3 * n * 4 + mih::radix_tmp_words(n) * 4 +
                                mih::scan_tmp_words(max_entries) * 4 + (1 << 20);
    uint64_t budget = o.mem_budget_bytes;
    if (!budget) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) { (void)hipGetLastError(); delete ix; return MIH_ERR_DEVICE; }
        budget = fr;
    }
    const uint64_t reserve = std::min<uint64_t>(8ull << 30, budget / 10);
    uint64_t need = ids_bytes + temp_bytes + reserve;
    if (o.table_mode == MIH_TABLE_DIRECT) ix->table_mode = MIH_TABLE_DIRECT;
    else if (o.table_mode == MIH_TABLE_SORTED) ix->table_mode = MIH_TABLE_SORTED;
    else if (o.table_mode == MIH_TABLE_GROUPED) ix->table_mode = MIH_TABLE_GROUPED;
    else if (o.table_mode == MIH_TABLE_HEADS) ix->table_mode = MIH_TABLE_HEADS;
    else if (bits == 64 && (o.codes_mode == MIH_CODES_AUTO || o.codes_mode == MIH_CODES_INLINE) &&
             n <= (1ull << ix->len[m - 1]) &&
             need + heads_bytes + (max_entries + 1) * 4 + (uint64_t)m * table_inline_bytes <= budget)
        // 64-bit codes in sparse tables (at most one code per bucket on
        // average): a bucket's offset, size and first code in one entry
        ix->table_mode = MIH_TABLE_HEADS;
    else if (need + direct_bytes > budget) ix->table_mode = MIH_TABLE_SORTED;
    else {
        // DIRECT unless it would leave fewer tables room for inline codes
        // than SORTED would (their offsets take 2^s words per table)
        const uint32_t kd = inline_tables_fit(need + direct_bytes, budget, table_inline_bytes, m);
        const uint32_t ks = inline_tables_fit(need + sorted_bytes, budget, table_inline_bytes, m);
        ix->table_mode = (o.codes_mode == MIH_CODES_AUTO && kd < m && ks > kd) ? MIH_TABLE_SORTED
                                                                               : MIH_TABLE_DIRECT;
    }
    need += ix->table_mode == MIH_TABLE_DIRECT ? direct_bytes
          : ix->table_mode == MIH_TABLE_SORTED ? sorted_bytes
          : ix->table_mode == MIH_TABLE_GROUPED ? grouped_bytes : heads_bytes;
    // the plain offsets of GROUPED and HEADS tables exist only while they are built
    const uint64_t build_off_bytes =
        (ix->table_mode == MIH_TABLE_GROUPED || ix->table_mode == MIH_TABLE_HEADS) ? (max_entries + 1) * 4 : 0;
    need += build_off_bytes;
    if (o.codes_mode == MIH_CODES_INLINE || ix->table_mode == MIH_TABLE_GROUPED ||
        ix->table_mode == MIH_TABLE_HEADS)
        ix->inline_tables = m;
    else if (o.codes_mode == MIH_CODES_INDIRECT) ix->inline_tables = 0;
    else if (o.codes_mode == MIH_CODES_MIXED) ix->inline_tables = o.inline_tables;
    else ix->inline_tables = inline_tables_fit(need, budget, table_inline_bytes, m);
    ix->codes_mode = ix->inline_tables == m ? MIH_CODES_INLINE
                   : ix->inline_tables == 0 ? MIH_CODES_INDIRECT : MIH_CODES_MIXED;
    need += (uint64_t)ix->inline_tables * table_inline_bytes;
    if (o.mem_budget_bytes && need - reserve > budget) { delete ix; return MIH_ERR_NOMEM; }

    mih_status st = MIH_OK;
    Scratch tk1, tk2, ti2, tmp, toff;
    do {
        hipError_t e;
        if ((e = tk1.ensure(n * 4 + 4)) != hipSuccess || (e = tk2.ensure(n * 4 + 4)) != hipSuccess ||
            (e = ti2.ensure(n * 4 + 4)) != hipSuccess || (e = toff.ensure(build_off_bytes)) != hipSuccess ||
            (e = tmp.ensure(std::max(mih::radix_tmp_words(n), mih::scan_tmp_words(max_entries)) * 4)) !=
                hipSuccess) {
            st = from_hip(e);
            break;
        }
        for (uint32_t j = 0; j < m && st == MIH_OK; ++j) {
            TableDev &T = ix->tables_host[j];
            T.len = ix->len[j];
            T.start = ix->start[j];
            T.dir_bits = ix->dir_bits[j];
            // the substring's bits: a mask for substring distances and, when
            // they are not the consecutive run [start, start + len), the
            // order in which they form the key
            T.permuted = 0;
            for (uint32_t k = 0; k < T.len; ++k) {
                const uint32_t b = ix->bit_order[T.start + k];
                T.mask[b >> 6] |= 1ull << (b & 63);
                T.order[k] = (uint8_t)b;
                if (b != T.start + k) T.permuted = 1;
            }
            uint32_t *ids = nullptr;
            if ((e = ix->alloc((void **)&ids, n * 4)) != hipSuccess) { st = from_hip(e); break; }
            uint32_t *keys = (uint32_t *)tk1.ptr, *keys2 = (uint32_t *)tk2.ptr, *ids2 = (uint32_t *)ti2.ptr;
            uint32_t *ids_cur = ids;
            e = mih::extract_keys(codes, n, W, T, keys, ids_cur, s);
            if (e == hipSuccess)
                e = mih::radix_sort_pairs(keys, ids_cur, keys2, ids2, n, T.len, (uint32_t *)tmp.ptr, s);
            if (e == hipSuccess && ids_cur != ids)
                e = hipMemcpyAsync(ids, ids_cur, n * 4, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) { st = from_hip(e); break; }
            T.ids = ids;
            if (ix->table_mode == MIH_TABLE_DIRECT) {
                uint32_t *off = nullptr;
                const uint64_t nb = 1ull << T.len;
                if ((e = ix->alloc((void **)&off, (nb + 1) * 4)) != hipSuccess) { st = from_hip(e); break; }
                e = mih::bucket_offsets(keys, n, 0, off, nb, (uint32_t *)tmp.ptr, s);
                T.off = off;
                uint32_t *occ = nullptr;
                if (e == hipSuccess && (e = ix->alloc((void **)&occ, std::max<uint64_t>(nb / 32, 1) * 4)) == hipSuccess)
                    e = mih::occupancy_bits(off, nb, occ, s);
                T.occ = occ;
            } else if (ix->table_mode == MIH_TABLE_HEADS) {
                // offsets (kept until the codes are in table order) and the
                // occupancy map; the heads follow the inline codes below
                const uint64_t nb = 1ull << T.len;
                uint32_t *off = (uint32_t *)toff.ptr;
                e = mih::bucket_offsets(keys, n, 0, off, nb, (uint32_t *)tmp.ptr, s);
                uint32_t *occ = nullptr;
                if (e == hipSuccess && (e = ix->alloc((void **)&occ, std::max<uint64_t>(nb / 32, 1) * 4)) == hipSuccess)
                    e = mih::occupancy_bits(off, nb, occ, s);
                T.occ = occ;
            } else if (ix->table_mode == MIH_TABLE_GROUPED) {
                const uint64_t nb = 1ull << T.len;
                uint32_t *off = (uint32_t *)toff.ptr;
                uint64_t *grp = nullptr;
                e = mih::bucket_offsets(keys, n, 0, off, nb, (uint32_t *)tmp.ptr, s);
                if (e == hipSuccess && (e = ix->alloc((void **)&grp, std::max<uint64_t>(nb / 32, 1) * 8)) == hipSuccess)
                    e = mih::group_records(off, nb, grp, s);
                T.grp = grp;
            } else {
                uint32_t *skeys = nullptr, *dir = nullptr;
                const uint64_t nb = 1ull << T.dir_bits;
                if ((e = ix->alloc((void **)&skeys, n * 4)) != hipSuccess ||
                    (e = ix->alloc((void **)&dir, (nb + 1) * 4)) != hipSuccess) { st = from_hip(e); break; }
                e = hipMemcpyAsync(skeys, keys, n * 4, hipMemcpyDeviceToDevice, s);
                if (e == hipSuccess)
                    e = mih::bucket_offsets(keys, n, T.len - T.dir_bits, dir, nb, (uint32_t *)tmp.ptr, s);
                T.keys = skeys;
                T.dir = dir;
            }
            if (e != hipSuccess) { st = from_hip(e); break; }
            if (j < ix->inline_tables) {
                uint64_t *tc = nullptr;
                if ((e = ix->alloc((void **)&tc, n * 8 * W)) != hipSuccess) { st = from_hip(e); break; }
                if ((e = mih::gather_codes(codes, ids, n, W, tc, s)) != hipSuccess) { st = from_hip(e); break; }
                T.codes = tc;
            }
            if (ix->table_mode == MIH_TABLE_HEADS) {
                const uint64_t nb = 1ull << T.len;
                BucketHead *head = nullptr;
                if ((e = ix->alloc((void **)&head, (nb + 1) * sizeof(BucketHead))) != hipSuccess ||
                    (e = mih::bucket_heads((const uint32_t *)toff.ptr, nb, T.codes, head, s)) != hipSuccess) {
                    st = from_hip(e);
                    break;
                }
                T.head = head;
            }
            if ((e = hipStreamSynchronize(s)) != hipSuccess) { st = from_hip(e); break; }
        }
        if (st != MIH_OK) break;
        if ((e = ix->alloc((void **)&ix->tables_dev, sizeof(TableDev) * m)) != hipSuccess) { st = from_hip(e); break; }
        if ((e = upload(ix->tables_dev, ix->tables_host, sizeof(TableDev) * m, s)) != hipSuccess) { st = from_hip(e); break; }
    } while (0);
    (void)hipStreamSynchronize(s);
    tk1.release();
    tk2.release();
    ti2.release();
    tmp.release();
    toff.release();
    if (st != MIH_OK) { delete ix; return st; }
    // the occupancy map pays off where the offsets array outgrows the caches
    uint32_t max_len = 0;
    for (uint32_t j = 0; j < m; ++j) max_len = std::max(max_len, ix->len[j]);
    ix->tuning.occupancy_filter =
        ((ix->table_mode == MIH_TABLE_DIRECT || ix->table_mode == MIH_TABLE_HEADS) && max_len >= 26) ? 1u : 0u;
    if (ix->table_mode == MIH_TABLE_HEADS && max_len >= 26) {
        // one entry read per occupied probe leaves registers for more
        // probes in flight per lane; the large steps run in the partition
        // kernel with a partition's occupancy bits in LDS (the autotuner's
        // usual pick there)
        ix->tuning.probes_per_lane = 4;
        ix->tuning.chunk = 8192;
        ix->tuning.sweep_shift = 3;
        ix->tuning.sweep_bits = 17;
        ix->tuning.sweep_queries = 4096;
    }
    ix->build_ms = ms_since(t0);
    *out = ix;
    return MIH_OK;
}

namespace {

// kNN through the index's batch engine, exact or stopped early.
mih_status knn_common(const mih_index *cidx, const uint64_t *queries, uint32_t nq, uint32_t k,
                      const uint32_t *k_per_query, uint32_t *out_ids, uint32_t *out_dists,
                      void *stream, mih_query_stats *stats, uint32_t max_t, uint32_t budget);

}  // namespace

mih_status mih_knn_ex(const mih_index *cidx, const uint64_t *queries, uint32_t nq, uint32_t k,
                      const uint32_t *k_per_query, uint32_t *out_ids, uint32_t *out_dists,
                      void *stream, mih_query_stats *stats)
{
    return knn_common(cidx, queries, nq, k, k_per_query, out_ids, out_dists, stream, stats,
                      0xFFFFFFFFu, 0);
}

mih_status mih_knn_approx(const mih_index *cidx, const uint64_t *queries, uint32_t nq, uint32_t k,
                          const uint32_t *k_per_query, uint32_t max_radius, uint32_t max_candidates,
                          uint32_t *out_ids, uint32_t *out_dists, void *stream, mih_query_stats *stats)
{
    return knn_common(cidx, queries, nq, k, k_per_query, out_ids, out_dists, stream, stats,
                      max_radius, max_candidates);
}

}  // extern "C"

namespace {

// Expected probes of an exact query with this k over uniform codes: the
// shells of steps 0 .. r of the model radius r (Eq. 1 per step).  Used only
// to pick the one-launch path for small batches.
uint64_t model_probes(const mih_index *ix, uint32_t k)
{
    const uint32_t r = mih_model_radius(ix->n, ix->bits, k);
    uint64_t probes = 0;
    for (uint32_t t = 0; t <= r && t <= ix->t_all; ++t) {
        const uint32_t rp = t / ix->m, s = ix->len[t % ix->m];
        if (rp > s) continue;
        uint64_t c = 1;
        for (uint32_t i = 1; i <= rp; ++i) c = c * (s - rp + i) / i;
        probes += c;
    }
    return probes;
}

// Most expected probes per query for the one-launch path: beyond this a
// query's steps are better spread over many workgroups by the rounds.
constexpr uint64_t kSmallProbes = 1ull << 18;

// The batch in one launch (mih_small): the state of every query starts
// from one upload of pinned staging (arguments, zeroed counters and
// histograms); overflowed queries are returned in `ovf` for the engine's
// exact re-run.
mih_status small_batch(mih_index *ix, const uint64_t *queries, uint32_t nq, const std::vector<uint32_t> &kv,
                       const std::vector<uint64_t> &row_off, uint32_t *out_ids, uint32_t *out_dists,
                       hipStream_t s, bool timed, mih::EngineStats &es, std::vector<uint32_t> &ovf)
{
    const uint32_t nb = ix->bits + 1, nsteps = ix->t_all + 1;
    std::vector<uint64_t> buf_off(nq);
    std::vector<uint32_t> cap(nq);
    uint64_t entries = 0;
    for (uint32_t i = 0; i < nq; ++i) {
        cap[i] = mih::search_capacity(kv[i], ix->tuning.buffer_mult);
        buf_off[i] = entries;
        entries += cap[i];
    }
    // the uploaded block: 64-bit arrays first, then the 32-bit ones
    uint64_t up = 0;
    auto field = [&](uint64_t bytes) { const uint64_t o = up; up += (bytes + 7) / 8 * 8; return o; };
    const uint64_t o_bo = field(8ull * nq), o_ro = field(8ull * nq), o_st = field(32), o_oc = field(8),
                   o_k = field(4ull * nq), o_cap = field(4ull * nq), o_tau = field(4ull * nq + 64),
                   o_cnt = field(4ull * nq), o_hist = field(4ull * nq * nb), o_stop = field(4ull * nq),
                   o_exit = field(4ull * nq), o_sc = field(4ull * nq * nsteps);
    // workgroups per query: the device's resident workgroups shared in
    // proportion to each query's expected probes (uniform-code model at its
    // k), at least 1 and at most 8 each
    if (ix->small_resident_J != ix->tuning.probes_per_lane) {
        mih::MihArgs L = {};
        mih::index_args(ix, L);
        ix->small_resident = num_cus() * (uint32_t)mih::mih_small_occupancy(L.W, L.tm, L.inline_codes, L.J);
        ix->small_resident_J = ix->tuning.probes_per_lane;
    }
    const uint32_t resident = ix->small_resident;
    std::vector<uint64_t> work(nq);
    double sum = 0;
    {
        std::vector<std::pair<uint32_t, uint64_t>> seen;   // the model per distinct k
        for (uint32_t i = 0; i < nq; ++i) {
            uint64_t w = 0;
            if (kv[i]) {
                auto it = std::find_if(seen.begin(), seen.end(), [&](const auto &p) { return p.first == kv[i]; });
                if (it == seen.end()) {
                    seen.emplace_back(kv[i], model_probes(ix, kv[i]));
                    it = seen.end() - 1;
                }
                w = it->second;
            }
            work[i] = w;
            sum += (double)w;
        }
    }
    std::vector<uint32_t> first(nq + 1, 0);
    for (uint32_t i = 0; i < nq; ++i) {
        const double share = sum > 0 ? (double)resident * (double)work[i] / sum : 1.0;
        first[i + 1] = first[i] + std::min<uint32_t>(8, std::max<uint32_t>(1, (uint32_t)share));
    }
    const uint32_t blocks = first[nq];
    const uint64_t o_first = field(4ull * (nq + 1)), o_qof = field(4ull * blocks);
    // then, not uploaded: the overflow list and the candidate buffers
    const uint64_t o_ol = align_up(up, 256), o_buf = align_up(o_ol + 4ull * nq, 256);
    const uint64_t dev_bytes = o_buf + 8 * std::max<uint64_t>(entries, 1);
    if (dev_bytes > ix->small_dev_bytes) {
        if (ix->small_dev) (void)hipFree(ix->small_dev);
        ix->small_dev = nullptr;
        ix->small_dev_bytes = 0;
        MIH_TRY(hipMalloc(&ix->small_dev, dev_bytes));
        ix->small_dev_bytes = dev_bytes;
    }
    const uint64_t host_bytes = up + 48;   // the upload, then the counters read back
    if (host_bytes > ix->small_host_bytes) {
        if (ix->small_host) (void)hipHostFree(ix->small_host);
        ix->small_host = nullptr;
        ix->small_host_bytes = 0;
        MIH_TRY(hipHostMalloc(&ix->small_host, host_bytes, 0));
        ix->small_host_bytes = host_bytes;
    }
    char *h = (char *)ix->small_host, *d = (char *)ix->small_dev;
    std::memset(h, 0, up);
    std::memcpy(h + o_bo, buf_off.data(), 8ull * nq);
    std::memcpy(h + o_ro, row_off.data(), 8ull * nq);
    std::memcpy(h + o_k, kv.data(), 4ull * nq);
    std::memcpy(h + o_cap, cap.data(), 4ull * nq);
    std::memcpy(h + o_first, first.data(), 4ull * (nq + 1));
    for (uint32_t i = 0; i < nq; ++i)
        for (uint32_t b = first[i]; b < first[i + 1]; ++b) reinterpret_cast<uint32_t *>(h + o_qof)[b] = i;
    for (uint32_t i = 0; i < nq; ++i) {
        reinterpret_cast<uint32_t *>(h + o_tau)[i] = ix->bits;
        reinterpret_cast<uint32_t *>(h + o_stop)[i] = 0xFFFFFFFFu;
    }
    MIH_TRY(hipMemcpyAsync(d, h, up, hipMemcpyHostToDevice, s));

    mih::MihArgs A = {};
    mih::index_args(ix, A);
    A.qb.queries = queries;
    A.qb.k = (const uint32_t *)(d + o_k);
    A.qb.tau = (uint32_t *)(d + o_tau);
    A.qb.count = (uint32_t *)(d + o_cnt);
    A.qb.cap = (const uint32_t *)(d + o_cap);
    A.qb.buf_off = (const uint64_t *)(d + o_bo);
    A.qb.buf = (uint64_t *)(d + o_buf);
    A.qb.hist = (uint32_t *)(d + o_hist);
    A.qb.nq = nq;
    A.qb.bits = ix->bits;
    A.stats = (unsigned long long *)(d + o_st);
    mih::SmallArgs S = {};
    S.nq = nq;
    S.blocks = blocks;
    S.first = (const uint32_t *)(d + o_first);
    S.query_of = (const uint32_t *)(d + o_qof);
    S.row_off = (const uint64_t *)(d + o_ro);
    S.out_ids = out_ids;
    S.out_dists = out_dists;
    S.stop = (uint32_t *)(d + o_stop);
    S.exits = (uint32_t *)(d + o_exit);
    S.step_cnt = (uint32_t *)(d + o_sc);
    S.ovf_list = (uint32_t *)(d + o_ol);
    S.ovf_count = (uint32_t *)(d + o_oc);
    EventPair ev(timed);
    ev.begin(s);
    MIH_TRY(mih::mih_small(A, S, s));
    ev.end(s);
    // the statistics and the overflow count, read back together
    char *hb = h + up;
    MIH_TRY(hipMemcpyAsync(hb, d + o_st, 36, hipMemcpyDeviceToHost, s));   // the overflow count follows
    MIH_TRY(hipStreamSynchronize(s));
    const unsigned long long *hs = (const unsigned long long *)hb;
    const uint32_t novf = *(const uint32_t *)(hb + 32);
    es.probes += hs[0];
    es.candidates += hs[1];
    es.steps += hs[2];
    es.appended += hs[3];
    es.rounds += 1;
    es.search_launches += 1;
    if (timed) es.search_kernel_ms += ev.ms();
    ovf.assign(novf, 0u);
    if (novf) MIH_TRY(download(ovf.data(), S.ovf_list, 4ull * novf, s));
    return MIH_OK;
}

mih_status knn_common(const mih_index *cidx, const uint64_t *queries, uint32_t nq, uint32_t k,
                      const uint32_t *k_per_query, uint32_t *out_ids, uint32_t *out_dists,
                      void *stream, mih_query_stats *stats, uint32_t max_t, uint32_t budget)
{
    auto t0 = clk::now();
    if (!cidx) return MIH_ERR_INVALID;
    mih_index *ix = const_cast<mih_index *>(cidx);
    MIH_TRY_STATUS(check_query_args(ix->bits, queries, nq, out_ids, out_dists));
    if (!k_per_query && k > MIH_K_MAX) return MIH_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(ix->mu);
    if (stats) std::memset(stats, 0, sizeof(*stats));
    std::vector<uint32_t> kv;
    MIH_TRY_STATUS(read_k(nq, k, k_per_query, s, kv));
    std::vector<uint64_t> row_off;
    row_offsets(kv, row_off);
    uint32_t slots = 0, kmax = 0;
    uint64_t pool = 0;
    for (uint32_t v : kv)
        if (v) { slots++; pool += mih::search_capacity(v, ix->tuning.buffer_mult); kmax = std::max(kmax, v); }
    if (slots == 0) return MIH_OK;
    mih::EngineStats small_es;
    std::vector<uint32_t> rest;   // queries left to the rounds (all, or the overflowed)
    const bool small = max_t == 0xFFFFFFFFu && budget == 0 && nq <= ix->tuning.small_batch &&
                       model_probes(ix, kmax) <= kSmallProbes;
    if (small) {
        MIH_TRY_STATUS(small_batch(ix, queries, nq, kv, row_off, out_ids, out_dists, s, stats != nullptr,
                                   small_es, rest));
        if (rest.empty()) {
            if (stats) copy_stats(small_es, t0, stats);
            return MIH_OK;
        }
        slots = (uint32_t)rest.size();
        pool = 0;
        for (uint32_t i : rest) pool += mih::search_capacity(kv[i], ix->tuning.buffer_mult);
    }
    // one engine per index, kept while it is large enough
    if (!ix->batch_engine || ix->batch_engine->slots() < slots || ix->batch_engine->pool_entries() < pool) {
        ix->batch_engine.reset();
        std::unique_ptr<mih::Engine> e(new (std::nothrow) mih::Engine(ix, s));
        if (!e) return MIH_ERR_NOMEM;
        hipError_t he = e->init(slots, pool, use_graphs());
        if (he != hipSuccess) { (void)hipGetLastError(); return from_hip(he); }
        ix->batch_engine = std::move(e);
    }
    mih::Engine &eng = *ix->batch_engine;
    eng.set_stream(s);
    MIH_TRY(eng.reset_stats());
    mih_status st = MIH_OK;
    if (!small) {
        st = engine_batch(eng, queries, nq, kv, row_off, out_ids, out_dists, max_t, budget);
    } else {
        // the overflowed queries of the one-launch path, one request each
        const uint32_t W = ix->W;
        std::vector<uint64_t> completed;
        eng.set_count_unique(false);
        eng.set_lookahead(true);
        for (uint32_t i : rest) eng.submit(queries + (uint64_t)i * W, 1, &kv[i], &row_off[i], out_ids, out_dists);
        while (st == MIH_OK && !eng.idle()) {
            hipError_t e = eng.step(completed);
            if (e != hipSuccess) { (void)hipGetLastError(); st = from_hip(e); }
        }
    }
    if (st != MIH_OK) { ix->batch_engine.reset(); return st; }
    if (stats) {
        mih::EngineStats es;
        MIH_TRY(eng.read_stats(es));
        es.probes += small_es.probes;
        es.candidates += small_es.candidates;
        es.steps += small_es.steps;
        es.appended += small_es.appended;
        es.rounds += small_es.rounds;
        es.reruns += (uint32_t)rest.size() * (small ? 1u : 0u);
        es.search_kernel_ms += small_es.search_kernel_ms;
        es.search_launches += small_es.search_launches;
        copy_stats(es, t0, stats);
    }
    return MIH_OK;
}

}  // namespace

extern "C" {

mih_status mih_knn(const mih_index *idx, const uint64_t *queries, uint32_t nq, uint32_t k,
                   const uint32_t *k_per_query, uint32_t *out_ids, uint32_t *out_dists, void *stream)
{
    return mih_knn_ex(idx, queries, nq, k, k_per_query, out_ids, out_dists, stream, nullptr);
}

void mih_free(mih_index *idx) { delete idx; }

// ------------------------------------------------------- r-neighbour search

mih_status mih_rnn_ex(const mih_index *cidx, const uint64_t *queries, uint32_t nq, uint32_t r,
                      const uint32_t *r_per_query, void *stream, mih_rnn_result **out,
                      mih_query_stats *stats)
{
    auto t0 = clk::now();
    if (!cidx || !out) return MIH_ERR_INVALID;
    *out = nullptr;
    mih_index *ix = const_cast<mih_index *>(cidx);
    if (nq && (!queries || ((uintptr_t)queries & 7) != 0)) return MIH_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lock(ix->mu);
    if (stats) std::memset(stats, 0, sizeof(*stats));
    std::vector<uint32_t> rv;
    MIH_TRY_STATUS(read_radius(nq, r, r_per_query, s, rv));
    std::unique_ptr<mih_rnn_result> res(new (std::nothrow) mih_rnn_result);
    if (!res) return MIH_ERR_NOMEM;
    const uint32_t slots = std::min<uint32_t>(std::max<uint32_t>(nq, 1), 1u << 16);
    const uint64_t pool = (uint64_t)slots * mih::kRnnCapacity;
    if (!ix->batch_engine || ix->batch_engine->slots() < slots || ix->batch_engine->pool_entries() < pool) {
        ix->batch_engine.reset();
        std::unique_ptr<mih::Engine> e(new (std::nothrow) mih::Engine(ix, s));
        if (!e) return MIH_ERR_NOMEM;
        hipError_t he = e->init(slots, pool, use_graphs());
        if (he != hipSuccess) { (void)hipGetLastError(); return from_hip(he); }
        ix->batch_engine = std::move(e);
    }
    mih::Engine &eng = *ix->batch_engine;
    eng.set_stream(s);
    MIH_TRY(eng.reset_stats());
    eng.set_count_unique(false);
    const uint64_t ticket = eng.submit_rnn(queries, nq, rv.data());
    std::vector<uint64_t> completed;
    uint64_t guard = 0;
    while (!eng.idle()) {
        hipError_t he = eng.step(completed);
        if (he != hipSuccess) { (void)hipGetLastError(); ix->batch_engine.reset(); return from_hip(he); }
        if (++guard > (1ull << 24)) { ix->batch_engine.reset(); return MIH_ERR_DEVICE; }
    }
    if (!eng.take_rnn(ticket, res->out)) { ix->batch_engine.reset(); return MIH_ERR_DEVICE; }
    if (stats) {
        mih::EngineStats es;
        MIH_TRY(eng.read_stats(es));
        copy_stats(es, t0, stats);
    }
    *out = res.release();
    return MIH_OK;
}

mih_status mih_rnn(const mih_index *idx, const uint64_t *queries, uint32_t nq, uint32_t r,
                   const uint32_t *r_per_query, void *stream, mih_rnn_result **out)
{
    return mih_rnn_ex(idx, queries, nq, r, r_per_query, stream, out, nullptr);
}

mih_status linscan_rnn(const uint64_t *codes, uint64_t n, uint32_t bits, const uint64_t *queries,
                       uint32_t nq, uint32_t r, const uint32_t *r_per_query, void *stream,
                       mih_rnn_result **out)
{
    if (!out) return MIH_ERR_INVALID;
    *out = nullptr;
    if (!bits_ok(bits)) return MIH_ERR_INVALID;
    if (nq && (!queries || ((uintptr_t)queries & 7) != 0)) return MIH_ERR_INVALID;
    if (n > 0xFFFFFFFEull || (n && !codes) || ((uintptr_t)codes & 7) != 0) return MIH_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint32_t> rv;
    MIH_TRY_STATUS(read_radius(nq, r, r_per_query, s, rv));
    for (uint32_t &v : rv) v = std::min(v, bits);
    std::unique_ptr<mih_rnn_result> res(new (std::nothrow) mih_rnn_result);
    if (!res) return MIH_ERR_NOMEM;
    mih::RnnCollector col(nq);
    if (n > 0 && nq > 0) {
        Scratch dtau;
        MIH_TRY(dtau.ensure(4ull * nq));
        mih_status st = from_hip(upload(dtau.ptr, rv.data(), 4ull * nq, s));
        BatchSpec b;
        b.queries = queries;
        b.nq = nq;
        b.k.assign(nq, mih::kRnnK);
        b.row_off.resize(nq);
        for (uint32_t i = 0; i < nq; ++i) b.row_off[i] = i;
        b.cap.assign(nq, mih::kRnnCapacity);
        b.tau0 = (const uint32_t *)dtau.ptr;
        b.rnn = &col;
        if (st == MIH_OK) st = linscan_batch(codes, n, bits, b, nullptr, nullptr, s, 0, nullptr);
        (void)hipStreamSynchronize(s);
        dtau.release();
        MIH_TRY_STATUS(st);
    }
    MIH_TRY(col.finish(bits, s, res->out));
    *out = res.release();
    return MIH_OK;
}

mih_status mih_rnn_result_view(const mih_rnn_result *res, mih_rnn_view *view)
{
    if (!res || !view) return MIH_ERR_INVALID;
    view->total = res->out.total;
    view->nq = res->out.nq;
    view->pad = 0;
    view->offsets = res->out.offsets;
    view->ids = res->out.ids;
    view->dists = res->out.dists;
    return MIH_OK;
}

void mih_rnn_result_free(mih_rnn_result *res) { delete res; }

mih_status mih_index_get_info(const mih_index *idx, mih_index_info *info)
{
    if (!idx || !info) return MIH_ERR_INVALID;
    std::memset(info, 0, sizeof(*info));
    info->n = idx->n;
    info->bits = idx->bits;
    info->m = idx->m;
    info->table_mode = idx->table_mode;
    info->codes_mode = idx->codes_mode;
    info->inline_tables = idx->inline_tables;
    for (uint32_t j = 0; j < idx->m; ++j) {
        info->sub_len[j] = idx->len[j];
        info->sub_start[j] = idx->start[j];
        info->dir_bits[j] = idx->table_mode == MIH_TABLE_SORTED ? idx->dir_bits[j] : 0;
    }
    info->device_bytes = idx->device_bytes;
    info->build_ms = idx->build_ms;
    for (uint32_t p = 0; p < idx->bits; ++p) info->bit_order[p] = idx->bit_order[p];
    return MIH_OK;
}

mih_status mih_get_tuning(const mih_index *idx, mih_tuning *tuning)
{
    if (!idx || !tuning) return MIH_ERR_INVALID;
    *tuning = idx->tuning;
    return MIH_OK;
}

mih_status mih_set_tuning(mih_index *idx, const mih_tuning *tuning)
{
    if (!idx || !tuning) return MIH_ERR_INVALID;
    const uint32_t J = tuning->probes_per_lane;
    if (!mih::mih_probes_per_lane_ok(J)) return MIH_ERR_INVALID;
    if (tuning->chunk == 0 || tuning->chunk % (64 * J) != 0 || tuning->chunk > (1u << 20))
        return MIH_ERR_INVALID;
    if (tuning->blocks_per_cu > 64 || tuning->occupancy_filter > 1) return MIH_ERR_INVALID;
    if (tuning->sweep_shift > 32 || tuning->sweep_bits < 10 || tuning->sweep_bits > 32) return MIH_ERR_INVALID;
    if (tuning->lookahead < 1 || tuning->lookahead > MIH_LOOKAHEAD_MAX) return MIH_ERR_INVALID;
    if (tuning->sweep_queries < 64 || tuning->sweep_queries > 4096 || tuning->sweep_queries % 64 != 0)
        return MIH_ERR_INVALID;
    if (tuning->buffer_mult < 1 || tuning->buffer_mult > 64) return MIH_ERR_INVALID;
    if (tuning->small_batch > 65536) return MIH_ERR_INVALID;
    if (tuning->round_masks > (1u << 30)) return MIH_ERR_INVALID;
    if (tuning->spill_codes != 0 && tuning->spill_codes < 256) return MIH_ERR_INVALID;
    std::lock_guard<std::mutex> lock(idx->mu);
    idx->tuning = *tuning;
    idx->tuning_version++;
    return MIH_OK;
}

mih_status mih_index_table(const mih_index *idx, uint32_t j, mih_table_view *view)
{
    if (!idx || !view || j >= idx->m) return MIH_ERR_INVALID;
    const TableDev &T = idx->tables_host[j];
    view->offsets = T.off;
    view->keys = T.keys;
    view->dir = T.dir;
    view->ids = T.ids;
    view->codes = T.codes;
    view->len = T.len;
    view->start = T.start;
    view->dir_bits = idx->table_mode == MIH_TABLE_SORTED ? T.dir_bits : 0;
    view->pad = 0;
    view->occupancy = T.occ;
    view->groups = T.grp;
    view->heads = reinterpret_cast<const uint64_t *>(T.head);
    return MIH_OK;
}

}  // extern "C"

// ============================================================== serving

struct mih_server {
    mih_index *ix = nullptr;
    std::unique_ptr<mih::Engine> eng;
    std::deque<uint64_t> backlog;   // completed tickets not yet reported
    uint64_t completed = 0;
};

extern "C" {

mih_status mih_server_create(const mih_index *cidx, const mih_server_opts *opts, void *stream,
                             mih_server **out)
{
    if (!cidx || !out) return MIH_ERR_INVALID;
    mih_server_opts o = {4096, 1, 0};
    if (opts) o = *opts;
    if (o.max_queries == 0) return MIH_ERR_INVALID;
    const uint64_t pool = o.buffer_entries ? o.buffer_entries : 8192ull * o.max_queries;
    mih_server *srv = new (std::nothrow) mih_server();
    if (!srv) return MIH_ERR_NOMEM;
    srv->ix = const_cast<mih_index *>(cidx);
    srv->eng.reset(new (std::nothrow) mih::Engine(srv->ix, (hipStream_t)stream));
    if (!srv->eng) { delete srv; return MIH_ERR_NOMEM; }
    hipError_t e = srv->eng->init(o.max_queries, pool, o.use_graph != 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete srv;
        return from_hip(e);
    }
    *out = srv;
    return MIH_OK;
}

mih_status mih_server_submit(mih_server *srv, const uint64_t *queries, uint32_t nq, uint32_t k,
                             const uint32_t *host_k_per_query, uint32_t *out_ids,
                             uint32_t *out_dists, uint64_t *ticket)
{
    if (!srv || !ticket) return MIH_ERR_INVALID;
    MIH_TRY_STATUS(check_query_args(srv->ix->bits, queries, nq, out_ids, out_dists));
    std::vector<uint32_t> kv(nq, k);
    if (host_k_per_query) kv.assign(host_k_per_query, host_k_per_query + nq);
    for (uint32_t v : kv) {
        if (v > MIH_K_MAX) return MIH_ERR_UNSUPPORTED;
        if (!srv->eng->can_ever_fit(v)) return MIH_ERR_CAPACITY;
    }
    std::vector<uint64_t> row_off;
    row_offsets(kv, row_off);
    *ticket = srv->eng->submit(queries, nq, kv.data(), row_off.data(), out_ids, out_dists);
    return MIH_OK;
}

mih_status mih_server_step(mih_server *srv, uint64_t *completed, uint32_t max_completed,
                           uint32_t *n_completed)
{
    if (!srv || !n_completed || (max_completed && !completed)) return MIH_ERR_INVALID;
    std::vector<uint64_t> done;
    hipError_t e = srv->eng->step(done);
    if (e != hipSuccess) { (void)hipGetLastError(); return from_hip(e); }
    srv->completed += done.size();
    for (uint64_t t : done) srv->backlog.push_back(t);
    uint32_t n = 0;
    while (n < max_completed && !srv->backlog.empty()) {
        completed[n++] = srv->backlog.front();
        srv->backlog.pop_front();
    }
    *n_completed = n;
    return MIH_OK;
}

mih_status mih_server_poll(const mih_server *srv, uint64_t ticket, int *done)
{
    if (!srv || !done) return MIH_ERR_INVALID;
    *done = srv->eng->done(ticket) ? 1 : 0;
    return MIH_OK;
}

mih_status mih_server_get_stats(mih_server *srv, mih_server_stats *st)
{
    if (!srv || !st) return MIH_ERR_INVALID;
    mih::EngineStats es;
    MIH_TRY(srv->eng->read_stats(es));
    std::memset(st, 0, sizeof(*st));
    st->probes = es.probes;
    st->candidates = es.candidates;
    st->completed_requests = srv->completed;
    st->rounds = es.rounds;
    st->in_flight = srv->eng->in_flight();
    st->pending_queries = srv->eng->pending_queries();
    st->reruns = es.reruns;
    st->search_kernel_ms = es.search_kernel_ms;
    return MIH_OK;
}

void mih_server_destroy(mih_server *srv) { delete srv; }

}  // extern "C"

// ============================================================== autotuner

namespace {

constexpr int kTuningFields = sizeof(mih_tuning) / sizeof(uint32_t);
static_assert(sizeof(mih_tuning) == kTuningFields * sizeof(uint32_t), "mih_tuning holds uint32_t fields only");

// The key of an autotuned launch: the index's shape and the sample (one k,
// or a hash of the per-query k values).
std::string autotune_key(const mih_index *ix, uint32_t nq, const std::vector<uint32_t> &kv)
{
    bool one = true;
    uint64_t h = 1469598103934665603ull;   // FNV-1a over the k values
    for (uint32_t v : kv) {
        one &= v == kv[0];
        for (int b = 0; b < 4; ++b) { h ^= (v >> (8 * b)) & 0xFFu; h *= 1099511628211ull; }
    }
    char buf[256];
    if (one)
        std::snprintf(buf, sizeof buf, "n=%llu bits=%u m=%u table=%u codes=%u inline=%u queries=%u k=%u",
                      (unsigned long long)ix->n, ix->bits, ix->m, ix->table_mode, ix->codes_mode, ix->inline_tables,
                      nq, kv.empty() ? 0u : kv[0]);
    else
        std::snprintf(buf, sizeof buf, "n=%llu bits=%u m=%u table=%u codes=%u inline=%u queries=%u k=%016llx",
                      (unsigned long long)ix->n, ix->bits, ix->m, ix->table_mode, ix->codes_mode, ix->inline_tables,
                      nq, (unsigned long long)h);
    return buf;
}

// Entries of a cache file: lines of the form  "key": [f0, f1, ...]  (the
// other lines, braces included, carry nothing).  Entries whose field count
// is not that of mih_tuning are dropped.
std::map<std::string, std::vector<uint32_t>> read_autotune_cache(const std::string &path)
{
    std::map<std::string, std::vector<uint32_t>> out;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return out;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        const char *q0 = std::strchr(line, '"');
        const char *q1 = q0 ? std::strchr(q0 + 1, '"') : nullptr;
        const char *b0 = q1 ? std::strchr(q1, '[') : nullptr;
        if (!b0) continue;
        std::vector<uint32_t> v;
        const char *p = b0 + 1;
        while (*p && *p != ']') {
            char *end = nullptr;
            const unsigned long x = std::strtoul(p, &end, 10);
            if (end == p) { ++p; continue; }
            v.push_back((uint32_t)x);
            p = end;
        }
        if ((int)v.size() == kTuningFields) out[std::string(q0 + 1, q1)] = v;
    }
    std::fclose(f);
    return out;
}

void store_autotune_cache(const std::string &path, const std::string &key, const mih_tuning &t)
{
    auto entries = read_autotune_cache(path);
    const uint32_t *f = reinterpret_cast<const uint32_t *>(&t);
    entries[key] = std::vector<uint32_t>(f, f + kTuningFields);
    const std::string tmp = path + ".tmp";
    FILE *o = std::fopen(tmp.c_str(), "w");
    if (!o) return;
    std::fprintf(o, "{\n");
    size_t i = 0;
    for (const auto &e : entries) {
        std::fprintf(o, "  \"%s\": [", e.first.c_str());
        for (int j = 0; j < kTuningFields; ++j) std::fprintf(o, j ? ", %u" : "%u", e.second[j]);
        std::fprintf(o, "]%s\n", ++i < entries.size() ? "," : "");
    }
    std::fprintf(o, "}\n");
    const bool ok = std::fclose(o) == 0;
    if (ok) (void)std::rename(tmp.c_str(), path.c_str());
    else (void)std::remove(tmp.c_str());
}

}  // namespace

extern "C" mih_status mih_autotune(mih_index *idx, const uint64_t *queries, uint32_t nq, uint32_t k,
                                   const uint32_t *k_per_query, void *stream, mih_tuning *chosen)
{
    if (!idx) return MIH_ERR_INVALID;
    if (nq == 0) {
        if (chosen) *chosen = idx->tuning;
        return MIH_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint32_t> kv;
    MIH_TRY_STATUS(read_k(nq, k, k_per_query, s, kv));
    // a launch tuned before for the same index shape and sample
    const std::string key = idx->autotune_cache.empty() ? std::string() : autotune_key(idx, nq, kv);
    if (!key.empty()) {
        const auto entries = read_autotune_cache(idx->autotune_cache);
        const auto it = entries.find(key);
        if (it != entries.end()) {
            mih_tuning t;
            std::memcpy(&t, it->second.data(), sizeof t);
            if (mih_set_tuning(idx, &t) == MIH_OK) {
                if (chosen) *chosen = t;
                return MIH_OK;
            }
        }
    }
    uint64_t total = 0;
    for (uint32_t v : kv) total += v;
    Scratch out;
    MIH_TRY(out.ensure(8 * (total ? total : 1)));
    uint32_t *oi = (uint32_t *)out.ptr, *od = oi + total;
    const mih_tuning start = idx->tuning;
    mih_tuning best = start;
    double best_ms = 1e300;
    // warm-up: first call sizes the engine and faults in the tables' pages
    mih_status st = mih_knn(idx, queries, nq, k, k_per_query, oi, od, stream);
    // the grid: (filter, J, chunk) with whole steps, then partition-major
    // sweeps of the large steps with the occupancy filter if there is one
    std::vector<mih_tuning> grid;
    const uint32_t filters =
        (idx->table_mode == MIH_TABLE_DIRECT || idx->table_mode == MIH_TABLE_HEADS) ? 2 : 1;
    for (uint32_t f = 0; f < filters; ++f)
        for (uint32_t J : {4u, 8u, 16u})
            for (uint32_t mult : {2u, 8u, 32u, 128u}) {
                mih_tuning t = idx->tuning;
                t.probes_per_lane = J;
                t.chunk = 64 * J * mult;
                t.blocks_per_cu = 0;
                t.occupancy_filter = f;
                t.sweep_shift = 0;
                grid.push_back(t);
            }
    uint32_t max_len = 0;
    for (uint32_t j = 0; j < idx->m; ++j) max_len = std::max(max_len, idx->len[j]);
    if (max_len >= mih::kSweepMinBits) {
        if (filters == 2) {
            // tables with an occupancy map sweep in the partition kernel:
            // partition size, masks per lane of the round kernel, and which
            // steps are swept (shift 4 also takes those of a quarter the size)
            struct { uint32_t J, bits, shift; } part[] = {{4, 16, 3}, {4, 17, 3}, {4, 18, 3}, {8, 17, 3},
                                                          {4, 17, 4}};
            for (const auto &p : part) {
                mih_tuning t = idx->tuning;
                t.probes_per_lane = p.J;
                t.chunk = 64 * p.J * 32;
                t.blocks_per_cu = 0;
                t.occupancy_filter = 1;
                t.sweep_shift = p.shift;
                t.sweep_bits = p.bits;
                t.sweep_queries = 4096;
                grid.push_back(t);
            }
        } else {
            for (uint32_t J : {4u, 8u})
                for (uint32_t bits : {18u, 20u}) {
                    mih_tuning t = idx->tuning;
                    t.probes_per_lane = J;
                    t.chunk = 64 * J * 32;
                    t.blocks_per_cu = 0;
                    t.occupancy_filter = 0;
                    t.sweep_shift = 3;
                    t.sweep_bits = bits;
                    grid.push_back(t);
                }
        }
    }
    // one timing per setting, then two more of the three fastest (a single
    // call can be a few percent off); the best of a setting's timings counts
    std::vector<double> ms(grid.size(), 1e300);
    auto time_one = [&](size_t i) {
        if ((st = mih_set_tuning(idx, &grid[i])) != MIH_OK) return;
        auto t0 = clk::now();
        st = mih_knn(idx, queries, nq, k, k_per_query, oi, od, stream);
        ms[i] = std::min(ms[i], ms_since(t0));
    };
    for (size_t i = 0; i < grid.size() && st == MIH_OK; ++i) time_one(i);
    if (st == MIH_OK) {
        std::vector<size_t> order(grid.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return ms[a] < ms[b]; });
        for (int rep = 0; rep < 2 && st == MIH_OK; ++rep)
            for (size_t r = 0; r < std::min<size_t>(3, order.size()) && st == MIH_OK; ++r) time_one(order[r]);
    }
    for (size_t i = 0; i < grid.size(); ++i)
        if (ms[i] < best_ms) { best_ms = ms[i]; best = grid[i]; }
    // candidate-buffer capacity with the best launch: fewer entries admit
    // more queries per round and touch less memory, more avoid the exact
    // re-runs of overflowed queries (timed with them)
    if (st == MIH_OK) {
        const size_t base = grid.size();
        for (uint32_t mult : {4u, 16u}) {
            mih_tuning t = best;
            t.buffer_mult = mult;
            grid.push_back(t);
        }
        ms.resize(grid.size(), 1e300);
        for (int rep = 0; rep < 2 && st == MIH_OK; ++rep)
            for (size_t i = base; i < grid.size() && st == MIH_OK; ++i) time_one(i);
        // a change of capacity must win by 3%: a sample's timings vary by
        // about that much, and a smaller buffer risks re-runs on other batches
        for (size_t i = base; i < grid.size(); ++i)
            if (ms[i] < best_ms * 0.97) { best_ms = ms[i]; best = grid[i]; }
    }
    // huge buckets shared out in pieces (clustered codes): with the best
    // launch so far, two sizes from which a bucket is cut (it must win by 3%:
    // its kernel variant holds more registers)
    if (st == MIH_OK && best.spill_codes == 0) {
        const size_t base = grid.size();
        for (uint32_t sc : {4096u, 32768u}) {
            mih_tuning t = best;
            t.spill_codes = sc;
            grid.push_back(t);
        }
        ms.resize(grid.size(), 1e300);
        for (int rep = 0; rep < 2 && st == MIH_OK; ++rep)
            for (size_t i = base; i < grid.size() && st == MIH_OK; ++i) time_one(i);
        for (size_t i = base; i < grid.size(); ++i)
            if (ms[i] < best_ms * 0.97) { best_ms = ms[i]; best = grid[i]; }
    }
    mih_status st2 = mih_set_tuning(idx, st == MIH_OK ? &best : &start);
    out.release();
    if (st != MIH_OK) return st;
    if (chosen) *chosen = best;
    if (st2 == MIH_OK && !key.empty()) store_autotune_cache(idx->autotune_cache, key, best);
    return st2;
}
