// Host side of the multi-index search: the index object and the engine that
// runs queries through the device rounds.
#pragma once

#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "mih_common.h"
#include "mih_query.h"
#include "rnn.h"

namespace mih {

// A first-fit allocator of buffer entries inside one device region.
class PoolAlloc {
public:
    void reset(uint64_t size);
    bool alloc(uint64_t n, uint64_t &off);
    void release(uint64_t off, uint64_t n);
    uint64_t size() const { return size_; }
    uint64_t free_total() const { return free_total_; }
    uint64_t largest_free() const;

private:
    std::map<uint64_t, uint64_t> free_;   // offset -> length
    uint64_t size_ = 0, free_total_ = 0;
};

// Candidate-buffer capacity given to a query with this k (entries):
// mult * max(k, 256).
inline uint32_t search_capacity(uint32_t k, uint32_t mult)
{
    return k == 0 ? 0u : mult * (k > 256u ? k : 256u);
}

// The k of an r-neighbour query: no count ever reaches it, so its bound
// stays at the radius.
constexpr uint32_t kRnnK = 0xFFFFFFFFu;
// First candidate-buffer capacity of an r-neighbour query (entries); a query
// with more hits is re-run with the exact count.  (1024 re-ran every query
// of 1e8 x 64-bit at the median 1000th distance, ~1,200 hits each.)
constexpr uint32_t kRnnCapacity = 4096;

class Engine;

// The index-wide fields of the search kernels' arguments (tables, layout,
// launch tuning), shared by the engine and the one-launch search.
void index_args(const mih_index *ix, MihArgs &A);

}  // namespace mih

struct mih_index {
    int device = 0;
    std::string autotune_cache;   // file of autotuned launches ("" for none)
    const uint64_t *codes = nullptr;
    uint64_t n = 0;
    uint32_t bits = 0, W = 0, m = 0;
    uint32_t table_mode = 0, codes_mode = 0;
    uint32_t inline_tables = 0;   // tables 0 .. inline_tables - 1 keep inline codes
    uint32_t len[MIH_M_MAX] = {}, start[MIH_M_MAX] = {}, dir_bits[MIH_M_MAX] = {};
    uint16_t bit_order[256] = {};
    uint32_t t_all = 0;
    TableDev tables_host[MIH_M_MAX] = {};
    TableDev *tables_dev = nullptr;
    std::vector<void *> allocs;
    uint64_t device_bytes = 0;
    double build_ms = 0;
    mih_tuning tuning = {4, 8192, 0, 0, 0, 18, MIH_LOOKAHEAD_DEFAULT, 256, 8, 512, 0, 0};
    uint32_t tuning_version = 0;
    std::mutex mu;
    std::unique_ptr<mih::Engine> batch_engine;   // reused by mih_knn calls
    // the one-launch search of small batches: device state (grow-only) and
    // pinned host staging for its arguments and counters
    void *small_dev = nullptr;
    uint64_t small_dev_bytes = 0;
    void *small_host = nullptr;
    uint64_t small_host_bytes = 0;
    uint32_t small_resident = 0, small_resident_J = 0;   // workgroups the one-launch kernel keeps resident

    hipError_t alloc(void **p, uint64_t bytes);
    ~mih_index();
};

namespace mih {

struct EngineStats {
    uint64_t probes = 0, candidates = 0, steps = 0, appended = 0;
    uint32_t rounds = 0, reruns = 0;
    double search_kernel_ms = 0;
    uint32_t search_launches = 0;
    double tail_ms = 0;   // rounds' tails: first to last wave of a search launch running out of work
};

// Runs queries over an index in rounds.  Per-query state lives in `slots`
// device slots; candidate buffers come from a pool of `pool_entries`
// entries.  Requests are admitted first in, first out, query by query, as
// slots and buffer memory become free; every query's result is independent
// of what else is in flight.
class Engine {
public:
    Engine(mih_index *ix, hipStream_t s) : ix_(ix), s_(s) {}
    ~Engine();
    hipError_t init(uint32_t slots, uint64_t pool_entries, bool use_graph);
    uint32_t slots() const { return S_; }
    uint64_t pool_entries() const { return pool_.size(); }

    // A request of nq queries with per-query k (host), output rows at
    // row_off[i] in out_ids / out_dists (device).  Returns its ticket.
    // An approximate request (Section 7) stops each query after step max_t
    // or once `budget` distinct codes were met (budget 0: no limit); counting
    // distinct codes must be switched on first (set_count_unique).
    uint64_t submit(const uint64_t *queries, uint32_t nq, const uint32_t *k,
                    const uint64_t *row_off, uint32_t *out_ids, uint32_t *out_dists,
                    uint32_t max_t = 0xFFFFFFFFu, uint32_t budget = 0);
    // Count distinct codes per query (needed by budgets; off by default).
    // Only while the engine is idle.
    void set_count_unique(bool on) { count_unique_ = on; }
    // Let rounds run queries ahead by several steps when they would leave
    // waves idle (exact searches only: an approximate query's result depends
    // on the steps it ran).  On by default; only while the engine is idle.
    void set_lookahead(bool on) { lookahead_ = on; }
    // A request of nq r-neighbour queries with per-query radius (host).  Its
    // results are taken with take_rnn() once the ticket has completed.
    uint64_t submit_rnn(const uint64_t *queries, uint32_t nq, const uint32_t *radius);
    // Hands over the output buffers of a completed r-neighbour request.
    bool take_rnn(uint64_t ticket, RnnOut &out);
    // One round; tickets of requests completed in it are appended.
    hipError_t step(std::vector<uint64_t> &completed);
    bool idle() const { return in_flight_ == 0 && pending_.empty() && reruns_.empty(); }
    bool done(uint64_t ticket) const { return reqs_.find(ticket) == reqs_.end(); }
    uint32_t in_flight() const { return in_flight_; }
    uint32_t pending_queries() const;
    hipError_t read_stats(EngineStats &out);
    hipError_t reset_stats();
    void set_stream(hipStream_t s) { s_ = s; }
    bool can_ever_fit(uint32_t k) const { return search_capacity(k, ix_->tuning.buffer_mult) <= pool_.size(); }

private:
    struct Req {
        const uint64_t *queries;
        uint32_t nq;
        std::vector<uint32_t> k;
        std::vector<uint64_t> row_off;
        uint32_t *out_ids, *out_dists;
        uint32_t next = 0, done = 0;
        std::vector<uint32_t> radius;            // r-neighbour requests only
        uint32_t max_t = 0xFFFFFFFFu, budget = 0;  // approximate requests
        std::unique_ptr<RnnCollector> rnn;       // non-null for r-neighbour requests
    };
    struct SlotInfo {
        uint64_t ticket = 0;
        uint32_t query = 0;
        uint64_t buf_off = 0, buf_len = 0;
    };
    struct Rerun {
        uint32_t slot, tau0, cap;
    };

    hipError_t admit();
    hipError_t run_round();
    hipError_t collect_rnn(const std::vector<uint32_t> &slots);
    hipError_t finish_round(const MihArgs &A, hipStream_t s);
    hipError_t complete(uint64_t ticket, Req &r, std::vector<uint64_t> &completed);
    hipError_t capture_graph();
    void fill_args(MihArgs &A) const;

    mih_index *ix_;
    hipStream_t s_;
    uint32_t S_ = 0;
    bool use_graph_ = false;
    void *dev_ = nullptr;      // slot state, one allocation
    uint64_t *pool_mem_ = nullptr;
    PoolAlloc pool_;
    QueryBatch qb_ = {};
    uint32_t *t_ = nullptr, *active_ = nullptr, *active_tmp_ = nullptr, *next_t_ = nullptr;
    uint32_t *new_slots_ = nullptr, *done_list_ = nullptr, *ovf_list_ = nullptr;
    uint32_t *bound_tau_ = nullptr, *bound_cap_ = nullptr;
    uint32_t *tmp_list_ = nullptr, *tmp_cnt_ = nullptr;
    uint32_t *max_t_ = nullptr, *budget_ = nullptr, *uniq_ = nullptr, *cursor_ = nullptr;
    bool count_unique_ = false, graph_count_unique_ = false;
    bool lookahead_ = true, graph_lookahead_ = true;
    uint64_t *out_ids_ = nullptr, *out_dists_ = nullptr;
    Group *groups_ = nullptr;
    Control *ctrl_ = nullptr;
    unsigned long long *work_ = nullptr, *stats_ = nullptr;
    SpillRec *spill_ = nullptr;
    uint32_t *spill_flag_ = nullptr;
    unsigned long long *spill_cnt_ = nullptr;
    AdmitRec *admit_dev_ = nullptr;
    Control *ctrl_host_ = nullptr;   // pinned
    uint32_t *done_host_ = nullptr;  // pinned [slots]: the last round's done list
    hipEvent_t ev_a_ = nullptr, ev_b_ = nullptr;
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t graph_exec_ = nullptr;
    uint32_t graph_tuning_version_ = ~0u;
    uint32_t round_grid_ = 0, sweep_grid_ = 0;

    std::vector<uint32_t> free_slots_;
    std::vector<SlotInfo> slot_info_;
    std::unordered_map<uint64_t, Req> reqs_;
    std::deque<uint64_t> pending_;
    std::deque<Rerun> reruns_;
    std::unordered_map<uint64_t, RnnOut> rnn_out_;   // finished r-neighbour requests
    uint64_t next_ticket_ = 1;
    uint32_t in_flight_ = 0;       // admitted queries not yet finished
    EngineStats stats_host_;
};

}  // namespace mih
