// The engine that runs multi-index kNN queries in device rounds.
//
// A round is three kernels: regroup (surviving and newly admitted queries
// become the active list, grouped by step), the persistent search kernel (one
// step of every active query) and advance (termination tests; finished
// queries are listed).  The three, with the copy of the control block to
// pinned host memory, are captured once in a hipGraph and replayed every
// round.  Between rounds the host admits queries into free slots (first in,
// first out, as long as slots and candidate-buffer memory allow), finalizes
// the finished ones into their requests' output rows, and re-admits the rare
// query whose buffer overflowed with its exact bound and an exact capacity.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "engine.h"

namespace mih {

namespace {

uint64_t align256(uint64_t x) { return (x + 255) / 256 * 256; }

uint32_t cu_count()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return (uint32_t)cus;
}

hipError_t sync_copy(void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t s)
{
    if (!bytes) return hipSuccess;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

}  // namespace

// ------------------------------------------------------------ PoolAlloc

void PoolAlloc::reset(uint64_t size)
{
    free_.clear();
    if (size) free_[0] = size;
    size_ = size;
    free_total_ = size;
}

bool PoolAlloc::alloc(uint64_t n, uint64_t &off)
{
    if (n == 0) { off = 0; return true; }
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second >= n) {
            off = it->first;
            uint64_t rest = it->second - n;
            free_.erase(it);
            if (rest) free_[off + n] = rest;
            free_total_ -= n;
            return true;
        }
    }
    return false;
}

void PoolAlloc::release(uint64_t off, uint64_t n)
{
    if (n == 0) return;
    auto it = free_.emplace(off, n).first;
    free_total_ += n;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        free_.erase(nx);
    }
    if (it != free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            free_.erase(it);
        }
    }
}

uint64_t PoolAlloc::largest_free() const
{
    uint64_t b = 0;
    for (auto &kv : free_) b = std::max(b, kv.second);
    return b;
}

// ------------------------------------------------------------ Engine

Engine::~Engine()
{
    if (graph_exec_) (void)hipGraphExecDestroy(graph_exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    if (ev_a_) (void)hipEventDestroy(ev_a_);
    if (ev_b_) (void)hipEventDestroy(ev_b_);
    if (ctrl_host_) (void)hipHostFree(ctrl_host_);
    if (done_host_) (void)hipHostFree(done_host_);
    if (pool_mem_) (void)hipFree(pool_mem_);
    if (dev_) (void)hipFree(dev_);
    for (auto &kv : rnn_out_) free_rnn_out(kv.second);
}

hipError_t Engine::init(uint32_t slots, uint64_t pool_entries, bool use_graph)
{
    S_ = slots ? slots : 1;
    use_graph_ = use_graph;
    const uint32_t W = ix_->W, nb = ix_->bits + 1;
    uint64_t used = 0;
    auto take = [&](uint64_t bytes) { uint64_t o = used; used += align256(bytes ? bytes : 1); return o; };
    const uint64_t o_q = take(8ull * S_ * W), o_k = take(4ull * S_), o_tau = take(4ull * S_ + 64),
                   o_cnt = take(4ull * S_), o_cap = take(4ull * S_), o_boff = take(8ull * S_),
                   o_hist = take(4ull * S_ * nb), o_t = take(4ull * S_), o_oi = take(8ull * S_),
                   o_od = take(8ull * S_), o_act = take(4ull * S_), o_tmp = take(4ull * S_),
                   o_nt = take(4ull * S_), o_new = take(4ull * S_), o_done = take(4ull * S_),
                   o_ovf = take(4ull * S_), o_btau = take(4ull * S_), o_bcap = take(4ull * S_),
                   o_grp = take(sizeof(Group) * (ix_->t_all + 1)), o_ctrl = take(sizeof(Control)),
                   o_work = take(8 * (1 + kSweepXcds)), o_scnt = take(4096), o_spill = take(sizeof(SpillRec) * kSpillCap), o_sflag = take(4ull * kSpillCap), o_stats = take(8 * kStatSlots), o_adm = take(sizeof(AdmitRec) * S_),
                   o_tl = take(4ull * S_), o_tc = take(4ull * S_), o_mt = take(4ull * S_),
                   o_bg = take(4ull * S_), o_uq = take(4ull * S_), o_cur = take(4ull * S_);
    hipError_t e = hipMalloc(&dev_, used);
    if (e != hipSuccess) { dev_ = nullptr; return e; }
    char *b = (char *)dev_;
    qb_.queries = (const uint64_t *)(b + o_q);
    qb_.k = (const uint32_t *)(b + o_k);
    qb_.tau = (uint32_t *)(b + o_tau);
    qb_.count = (uint32_t *)(b + o_cnt);
    qb_.cap = (const uint32_t *)(b + o_cap);
    qb_.buf_off = (const uint64_t *)(b + o_boff);
    qb_.hist = (uint32_t *)(b + o_hist);
    qb_.nq = S_;
    qb_.bits = ix_->bits;
    t_ = (uint32_t *)(b + o_t);
    out_ids_ = (uint64_t *)(b + o_oi);
    out_dists_ = (uint64_t *)(b + o_od);
    active_ = (uint32_t *)(b + o_act);
    active_tmp_ = (uint32_t *)(b + o_tmp);
    next_t_ = (uint32_t *)(b + o_nt);
    new_slots_ = (uint32_t *)(b + o_new);
    done_list_ = (uint32_t *)(b + o_done);
    ovf_list_ = (uint32_t *)(b + o_ovf);
    bound_tau_ = (uint32_t *)(b + o_btau);
    bound_cap_ = (uint32_t *)(b + o_bcap);
    groups_ = (Group *)(b + o_grp);
    ctrl_ = (Control *)(b + o_ctrl);
    work_ = (unsigned long long *)(b + o_work);
    spill_ = (SpillRec *)(b + o_spill);
    spill_flag_ = (uint32_t *)(b + o_sflag);
    spill_cnt_ = (unsigned long long *)(b + o_scnt);
    stats_ = (unsigned long long *)(b + o_stats);
    admit_dev_ = (AdmitRec *)(b + o_adm);
    tmp_list_ = (uint32_t *)(b + o_tl);
    tmp_cnt_ = (uint32_t *)(b + o_tc);
    max_t_ = (uint32_t *)(b + o_mt);
    budget_ = (uint32_t *)(b + o_bg);
    uniq_ = (uint32_t *)(b + o_uq);
    cursor_ = (uint32_t *)(b + o_cur);

    const uint64_t pe = pool_entries ? pool_entries : 1;
    e = hipMalloc((void **)&pool_mem_, pe * 8);
    if (e != hipSuccess) { pool_mem_ = nullptr; return e; }
    pool_.reset(pe);
    qb_.buf = pool_mem_;
    e = hipHostMalloc((void **)&ctrl_host_, sizeof(Control), 0);
    if (e != hipSuccess) { ctrl_host_ = nullptr; return e; }
    std::memset(ctrl_host_, 0, sizeof(Control));
    e = hipHostMalloc((void **)&done_host_, 4ull * S_, 0);
    if (e != hipSuccess) { done_host_ = nullptr; return e; }
    if ((e = hipEventCreate(&ev_a_)) != hipSuccess || (e = hipEventCreate(&ev_b_)) != hipSuccess) return e;
    // zeroed control block, counters and statistics
    if ((e = fill_u32((uint32_t *)ctrl_, sizeof(Control) / 4, 0u, s_)) != hipSuccess) return e;
    if ((e = fill_u64((uint64_t *)work_, 1 + kSweepXcds, 0ull, s_)) != hipSuccess) return e;
    if ((e = fill_u64((uint64_t *)spill_cnt_, 512, 0ull, s_)) != hipSuccess) return e;
    if ((e = fill_u64((uint64_t *)stats_, kStatSlots, 0ull, s_)) != hipSuccess) return e;
    if ((e = fill_u32(spill_flag_, kSpillCap, 0u, s_)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s_)) != hipSuccess) return e;
    free_slots_.resize(S_);
    for (uint32_t i = 0; i < S_; ++i) free_slots_[i] = S_ - 1 - i;
    slot_info_.assign(S_, SlotInfo());
    return hipSuccess;
}

void index_args(const mih_index *ix, MihArgs &A)
{
    A.tables = ix->tables_dev;
    A.codes = ix->codes;
    A.n = ix->n;
    A.W = ix->W;
    A.m = ix->m;
    A.bits = ix->bits;
    A.t_all = ix->t_all;
    A.tm = ix->table_mode == MIH_TABLE_SORTED ? TM_SORTED
         : ix->table_mode == MIH_TABLE_GROUPED ? TM_GROUPED
         : ix->table_mode == MIH_TABLE_HEADS ? TM_HEADS : TM_DIRECT;
    A.inline_codes = ix->codes_mode == MIH_CODES_INLINE;
    A.chunk = ix->tuning.chunk;
    A.J = ix->tuning.probes_per_lane;
    // DIRECT and HEADS tables: test the occupancy map before the bucket
    // (HEADS entries also say whether a bucket is empty; the map is denser)
    A.occ_filter = ix->tuning.occupancy_filter &&
                   (ix->table_mode == MIH_TABLE_DIRECT || ix->table_mode == MIH_TABLE_HEADS);
}

void Engine::fill_args(MihArgs &A) const
{
    index_args(ix_, A);
    // the work quantum in whole work items; steps cut into portions are
    // never swept (a sweep runs a whole step): the regroup kernel sweeps
    // only steps within one quantum
    A.quantum_items = ix_->tuning.round_masks
                          ? std::max<uint32_t>(1u, (ix_->tuning.round_masks + A.chunk - 1) / A.chunk)
                          : 0u;
    A.cursor = cursor_;
    // distinct codes are counted in whole-step probing only
    A.sweep_shift = count_unique_ ? 0u : ix_->tuning.sweep_shift;
    A.count_unique = count_unique_ ? 1u : 0u;
    A.max_t = max_t_;
    A.budget = budget_;
    A.uniq = uniq_;
    A.sweep_bits = ix_->tuning.sweep_bits;
    // tables with an occupancy map sweep in the partition kernel, with the
    // partition's occupancy bits staged in LDS
    A.sweep_part = A.occ_filter && (A.tm == TM_HEADS || A.tm == TM_DIRECT) &&
                   mih_part_kernel_ok(A.W, A.tm, A.inline_codes, A.J);
    A.part_bits = std::min(std::max(ix_->tuning.sweep_bits, kPartMinBits), kPartMaxBits);
    A.sweep_q = A.sweep_part ? std::max<uint32_t>(ix_->tuning.sweep_queries, MIH_WAVE) : kSweepQueries;
    // lookahead fills the waves of the round kernel
    A.look_max = lookahead_ ? std::min<uint32_t>(std::max<uint32_t>(ix_->tuning.lookahead, 1u), kLookMax) : 1u;
    A.look_items = A.look_max > 1 ? round_grid_ * (MIH_BLOCK / MIH_WAVE) : 0u;
    A.look_masks = (uint64_t)A.look_items * MIH_WAVE * A.J * kLookPasses;
    A.qb = qb_;
    A.t = t_;
    A.out_ids = out_ids_;
    A.out_dists = out_dists_;
    A.active = active_;
    A.active_tmp = active_tmp_;
    A.next_t = next_t_;
    A.new_slots = new_slots_;
    A.done_list = done_list_;
    A.ovf_list = ovf_list_;
    A.groups = groups_;
    A.ctrl = ctrl_;
    A.work = work_;
    A.work_sweep = work_ + 1;
    A.stats = stats_;
    // huge buckets are shared out in pieces among the waves of the round
    // kernel (not where distinct codes are counted: a piece's walk does not)
    A.spill = spill_;
    A.spill_flag = spill_flag_;
    A.spill_tail = spill_cnt_;          // its own 128-byte line
    A.spill_next = spill_cnt_ + 16;     // and this one
    A.spill_cap = kSpillCap;
    A.spill_min = count_unique_ ? 0u : ix_->tuning.spill_codes;
}

uint64_t Engine::submit(const uint64_t *queries, uint32_t nq, const uint32_t *k,
                        const uint64_t *row_off, uint32_t *out_ids, uint32_t *out_dists,
                        uint32_t max_t, uint32_t budget)
{
    const uint64_t ticket = next_ticket_++;
    Req r;
    r.queries = queries;
    r.nq = nq;
    r.k.assign(k, k + nq);
    r.row_off.assign(row_off, row_off + nq);
    r.out_ids = out_ids;
    r.out_dists = out_dists;
    r.max_t = max_t;
    r.budget = budget;
    reqs_.emplace(ticket, std::move(r));
    pending_.push_back(ticket);
    return ticket;
}

uint64_t Engine::submit_rnn(const uint64_t *queries, uint32_t nq, const uint32_t *radius)
{
    const uint64_t ticket = next_ticket_++;
    Req r;
    r.queries = queries;
    r.nq = nq;
    r.k.assign(nq, kRnnK);
    r.row_off.assign(nq, 0);
    r.out_ids = r.out_dists = nullptr;
    r.radius.assign(radius, radius + nq);
    r.rnn.reset(new RnnCollector(nq));
    reqs_.emplace(ticket, std::move(r));
    pending_.push_back(ticket);
    return ticket;
}

bool Engine::take_rnn(uint64_t ticket, RnnOut &out)
{
    auto it = rnn_out_.find(ticket);
    if (it == rnn_out_.end()) return false;
    out = it->second;
    rnn_out_.erase(it);
    return true;
}

uint32_t Engine::pending_queries() const
{
    uint32_t p = 0;
    for (uint64_t t : pending_) {
        auto it = reqs_.find(t);
        if (it != reqs_.end()) p += it->second.nq - it->second.next;
    }
    return p;
}

hipError_t Engine::admit()
{
    std::vector<AdmitRec> recs;
    const uint32_t W = ix_->W;
    // queries that overflowed come back first; they keep their slot
    while (!reruns_.empty()) {
        Rerun rr = reruns_.front();
        uint64_t off;
        if (rr.cap > pool_.size() && pool_.free_total() == pool_.size() && recs.empty()) {
            // the exact capacity exceeds the pool: grow it while it is unused
            (void)hipStreamSynchronize(s_);
            uint64_t *np = nullptr;
            const uint64_t ns = std::max<uint64_t>(rr.cap, pool_.size() * 2);
            hipError_t e = hipMalloc((void **)&np, ns * 8);
            if (e != hipSuccess) return e;
            (void)hipFree(pool_mem_);
            pool_mem_ = np;
            qb_.buf = np;
            pool_.reset(ns);
            graph_tuning_version_ = ~0u;   // kernel arguments changed
        }
        if (!pool_.alloc(rr.cap, off)) break;
        SlotInfo &si = slot_info_[rr.slot];
        const Req &r = reqs_.at(si.ticket);
        si.buf_off = off;
        si.buf_len = rr.cap;
        AdmitRec a;
        a.slot = rr.slot;
        a.k = r.k[si.query];
        a.cap = rr.cap;
        a.tau0 = rr.tau0;
        a.max_t = r.max_t;
        a.budget = r.budget;
        a.buf_off = off;
        a.query = (uint64_t)(uintptr_t)(qb_.queries + (uint64_t)rr.slot * W);
        a.out_ids = r.rnn ? 0 : (uint64_t)(uintptr_t)(r.out_ids + r.row_off[si.query]);
        a.out_dists = r.rnn ? 0 : (uint64_t)(uintptr_t)(r.out_dists + r.row_off[si.query]);
        recs.push_back(a);
        reruns_.pop_front();
    }
    while (reruns_.empty() && !pending_.empty()) {
        const uint64_t ticket = pending_.front();
        Req &r = reqs_.at(ticket);
        bool stalled = false;
        while (r.next < r.nq) {
            const uint32_t i = r.next;
            const uint32_t k = r.k[i];
            if (k == 0) {   // nothing to search and nothing to write
                r.next++;
                r.done++;
                continue;
            }
            uint64_t off;
            const uint32_t cap = r.rnn ? kRnnCapacity : search_capacity(k, ix_->tuning.buffer_mult);
            if (free_slots_.empty() || !pool_.alloc(cap, off)) { stalled = true; break; }
            const uint32_t slot = free_slots_.back();
            free_slots_.pop_back();
            slot_info_[slot] = SlotInfo{ticket, i, off, cap};
            AdmitRec a;
            a.slot = slot;
            a.k = k;
            a.cap = cap;
            a.max_t = r.max_t;
            a.budget = r.budget;
            // an r-neighbour query starts (and stays) at its radius
            a.tau0 = r.rnn ? std::min(r.radius[i], ix_->bits) : ix_->bits;
            a.buf_off = off;
            a.query = (uint64_t)(uintptr_t)(r.queries + (uint64_t)i * W);
            a.out_ids = r.rnn ? 0 : (uint64_t)(uintptr_t)(r.out_ids + r.row_off[i]);
            a.out_dists = r.rnn ? 0 : (uint64_t)(uintptr_t)(r.out_dists + r.row_off[i]);
            recs.push_back(a);
            r.next++;
            in_flight_++;
        }
        if (stalled) break;
        pending_.pop_front();
    }
    if (recs.empty()) return hipSuccess;
    hipError_t e = sync_copy(admit_dev_, recs.data(), sizeof(AdmitRec) * recs.size(),
                             hipMemcpyHostToDevice, s_);
    if (e != hipSuccess) return e;
    MihArgs A;
    fill_args(A);
    return mih_admit(A, admit_dev_, (uint32_t)recs.size(), s_);
}

hipError_t Engine::capture_graph()
{
    if (graph_exec_) { (void)hipGraphExecDestroy(graph_exec_); graph_exec_ = nullptr; }
    if (graph_) { (void)hipGraphDestroy(graph_); graph_ = nullptr; }
    MihArgs A;
    fill_args(A);
    uint32_t per_cu = (uint32_t)mih_round_occupancy(A.W, A.tm, A.inline_codes, A.J, A.spill_min ? 3 : 0, 0);
    if (ix_->tuning.blocks_per_cu && ix_->tuning.blocks_per_cu < per_cu) per_cu = ix_->tuning.blocks_per_cu;
    round_grid_ = cu_count() * per_cu;
    uint32_t per_cu_sweep =
        (uint32_t)mih_round_occupancy(A.W, A.tm, A.inline_codes, A.J, A.sweep_part ? 2 : 1, A.part_bits);
    if (ix_->tuning.blocks_per_cu && ix_->tuning.blocks_per_cu < per_cu_sweep)
        per_cu_sweep = ix_->tuning.blocks_per_cu;
    sweep_grid_ = cu_count() * per_cu_sweep;
    fill_args(A);   // again, now that the round's grid is known
    graph_lookahead_ = lookahead_;
    if (!use_graph_) {
        graph_tuning_version_ = ix_->tuning_version;
        graph_count_unique_ = count_unique_;
        return hipSuccess;
    }
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e1 = mih_regroup(A, cs);
        if (e1 == hipSuccess && A.sweep_shift) e1 = mih_sweep(A, sweep_grid_, cs);
        if (e1 == hipSuccess) e1 = mih_round(A, round_grid_, cs);
        if (e1 == hipSuccess) e1 = mih_advance(A, S_, cs);
        if (e1 == hipSuccess) e1 = finish_round(A, cs);
        e = hipStreamEndCapture(cs, &graph_);
        if (e1 != hipSuccess) e = e1;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&graph_exec_, graph_, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        // fall back to direct launches
        (void)hipGetLastError();
        if (graph_) { (void)hipGraphDestroy(graph_); graph_ = nullptr; }
        graph_exec_ = nullptr;
        use_graph_ = false;
    }
    graph_tuning_version_ = ix_->tuning_version;
    graph_count_unique_ = count_unique_;
    return hipSuccess;
}

// End of a round, on the device: the top-k rows of the finished queries,
// then the control block and the done list to pinned host memory.
hipError_t Engine::finish_round(const MihArgs &A, hipStream_t s)
{
    const uint32_t grid = std::min<uint32_t>(S_, cu_count() * 4);
    hipError_t e = finalize_done(qb_, done_list_, &ctrl_->n_done, out_ids_, out_dists_, grid, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ctrl_host_, ctrl_, sizeof(Control), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(done_host_, done_list_, 4ull * S_, hipMemcpyDeviceToHost, s);
    (void)A;
    return e;
}

hipError_t Engine::run_round()
{
    hipError_t e;
    if (graph_tuning_version_ != ix_->tuning_version || (use_graph_ && !graph_exec_) ||
        graph_count_unique_ != count_unique_ || graph_lookahead_ != lookahead_) {
        if ((e = capture_graph()) != hipSuccess) return e;
    }
    if (use_graph_ && graph_exec_) {
        // the events bracket the whole replay; the regroup and advance
        // kernels around the search kernel take microseconds
        if ((e = hipEventRecord(ev_a_, s_)) != hipSuccess) return e;
        if ((e = hipGraphLaunch(graph_exec_, s_)) != hipSuccess) return e;
        if ((e = hipEventRecord(ev_b_, s_)) != hipSuccess) return e;
    } else {
        MihArgs A;
        fill_args(A);
        if ((e = mih_regroup(A, s_)) != hipSuccess) return e;
        if ((e = hipEventRecord(ev_a_, s_)) != hipSuccess) return e;
        if (A.sweep_shift && (e = mih_sweep(A, sweep_grid_, s_)) != hipSuccess) return e;
        if ((e = mih_round(A, round_grid_, s_)) != hipSuccess) return e;
        if ((e = hipEventRecord(ev_b_, s_)) != hipSuccess) return e;
        if ((e = mih_advance(A, S_, s_)) != hipSuccess) return e;
        if ((e = finish_round(A, s_)) != hipSuccess) return e;
    }
    if ((e = hipStreamSynchronize(s_)) != hipSuccess) return e;
    float ms = 0;
    if (hipEventElapsedTime(&ms, ev_a_, ev_b_) == hipSuccess) stats_host_.search_kernel_ms += ms;
    else (void)hipGetLastError();
    stats_host_.search_launches++;
    stats_host_.rounds++;
    return hipSuccess;
}

hipError_t Engine::step(std::vector<uint64_t> &completed)
{
    hipError_t e = admit();
    if (e != hipSuccess) return e;
    // requests that needed no search (every k = 0, or no queries) are complete already
    for (auto it = reqs_.begin(); it != reqs_.end();) {
        if (it->second.next == it->second.nq && it->second.done == it->second.nq) {
            const uint64_t ticket = it->first;
            if ((e = complete(ticket, it->second, completed)) != hipSuccess) return e;
            it = reqs_.erase(it);
        } else {
            ++it;
        }
    }
    if (in_flight_ == 0) return hipSuccess;
    if ((e = run_round()) != hipSuccess) return e;
    // the round already wrote the top-k rows of its finished kNN queries and
    // copied the done list; r-neighbour hits are collected here
    const uint32_t n_done = ctrl_host_->n_done, n_ovf = ctrl_host_->n_ovf;
    std::vector<uint32_t> done(done_host_, done_host_ + n_done), ovf(n_ovf);
    if (n_done) {
        std::vector<uint32_t> rnn;
        for (uint32_t q : done) {
            auto it = reqs_.find(slot_info_[q].ticket);
            if (it != reqs_.end() && it->second.rnn) rnn.push_back(q);
        }
        if (!rnn.empty() && (e = collect_rnn(rnn)) != hipSuccess) return e;
    }
    if (n_ovf) {
        if ((e = sync_copy(ovf.data(), ovf_list_, 4ull * n_ovf, hipMemcpyDeviceToHost, s_)) != hipSuccess)
            return e;
        if ((e = exact_bounds(qb_, ovf_list_, n_ovf, bound_tau_, bound_cap_, s_)) != hipSuccess) return e;
        std::vector<uint32_t> tau(n_ovf), cap(n_ovf);
        if ((e = sync_copy(tau.data(), bound_tau_, 4ull * n_ovf, hipMemcpyDeviceToHost, s_)) != hipSuccess)
            return e;
        if ((e = sync_copy(cap.data(), bound_cap_, 4ull * n_ovf, hipMemcpyDeviceToHost, s_)) != hipSuccess)
            return e;
        for (uint32_t i = 0; i < n_ovf; ++i) {
            SlotInfo &si = slot_info_[ovf[i]];
            pool_.release(si.buf_off, si.buf_len);
            si.buf_len = 0;
            reruns_.push_back(Rerun{ovf[i], tau[i], std::max<uint32_t>(cap[i], 1u)});
            stats_host_.reruns++;
        }
    }
    if ((e = hipStreamSynchronize(s_)) != hipSuccess) return e;
    for (uint32_t q : done) {
        SlotInfo &si = slot_info_[q];
        auto it = reqs_.find(si.ticket);
        pool_.release(si.buf_off, si.buf_len);
        si.buf_len = 0;
        free_slots_.push_back(q);
        in_flight_--;
        if (it == reqs_.end()) continue;
        Req &r = it->second;
        r.done++;
        if (r.done == r.nq && r.next == r.nq) {
            if ((e = complete(it->first, r, completed)) != hipSuccess) return e;
            reqs_.erase(it);
        }
    }
    return hipSuccess;
}

// Moves the hits of finished r-neighbour queries out of their candidate
// buffers into their requests' collectors.
hipError_t Engine::collect_rnn(const std::vector<uint32_t> &slots)
{
    const uint32_t n = (uint32_t)slots.size();
    hipError_t e = sync_copy(tmp_list_, slots.data(), 4ull * n, hipMemcpyHostToDevice, s_);
    if (e == hipSuccess) e = gather_counts(qb_.count, tmp_list_, n, tmp_cnt_, s_);
    std::vector<uint32_t> cnt(n);
    if (e == hipSuccess) e = sync_copy(cnt.data(), tmp_cnt_, 4ull * n, hipMemcpyDeviceToHost, s_);
    if (e != hipSuccess) return e;
    // one add per request
    std::unordered_map<uint64_t, std::vector<uint32_t>> by_req;
    for (uint32_t i = 0; i < n; ++i) by_req[slot_info_[slots[i]].ticket].push_back(i);
    for (auto &kv : by_req) {
        Req &r = reqs_.at(kv.first);
        std::vector<uint32_t> query, count;
        std::vector<uint64_t> src;
        for (uint32_t i : kv.second) {
            const SlotInfo &si = slot_info_[slots[i]];
            query.push_back(si.query);
            src.push_back(si.buf_off);
            count.push_back(cnt[i]);
        }
        if ((e = r.rnn->add(qb_.buf, query, src, count, s_)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t Engine::complete(uint64_t ticket, Req &r, std::vector<uint64_t> &completed)
{
    if (r.rnn) {
        RnnOut out;
        hipError_t e = r.rnn->finish(ix_->bits, s_, out);
        if (e != hipSuccess) return e;
        rnn_out_[ticket] = out;
        r.rnn.reset();
    }
    completed.push_back(ticket);
    return hipSuccess;
}

hipError_t Engine::reset_stats()
{
    stats_host_ = EngineStats();
    return fill_u64((uint64_t *)stats_, kStatSlots, 0ull, s_);
}

hipError_t Engine::read_stats(EngineStats &out)
{
    unsigned long long st[kStatSlots] = {};
    hipError_t e = sync_copy(st, stats_, sizeof(st), hipMemcpyDeviceToHost, s_);
    if (e != hipSuccess) return e;
    out = stats_host_;
    out.probes = st[0];
    out.candidates = st[1];
    out.steps = st[2];
    out.appended = st[3];
    // the wall clock's rate (kHz) turns ticks into milliseconds
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
        out.tail_ms = (double)st[kStatTail] / khz;
    (void)hipGetLastError();
    return hipSuccess;
}

}  // namespace mih
