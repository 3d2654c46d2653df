// Launch interface of the multi-index search kernels (mih_query.hip).
#pragma once

#include "mih_common.h"

namespace mih {

// Table layouts as the search kernel sees them.
enum { TM_DIRECT = 0, TM_SORTED = 1, TM_GROUPED = 2, TM_HEADS = 3 };

// Most steps one round may run ahead for a group of queries.
constexpr uint32_t kLookMax = MIH_LOOKAHEAD_MAX;
// Shell masks a round may grow to by lookahead, in passes of every wave.
constexpr uint32_t kLookPasses = 4;

// Active queries that share the same next step form a group; its work items
// are the chunks of that step's shell for each of its queries, numbered
// from item_start, query-major.  When the round would leave waves idle, a
// group also takes its next steps (up to kLookMax in all): the items of
// query i of the group are then the chunks of steps t, t + 1, ..., in order.
// A group whose step has many more probes than its table has buckets per
// cache line runs in the sweep kernel instead (ipq = 0 there): its items
// are (key partition of 2^sweep_bits values, chunk of kSweepQueries queries).
struct Group {
    uint32_t t;           // first step to process
    uint32_t count;       // queries in the group
    uint32_t ipq;         // work items per query: step_items[steps], 0 when swept
    uint32_t steps;       // steps t .. t + steps - 1 run in this round
    uint32_t step_items[kLookMax + 1];   // items per query before step t + u
    uint32_t slot_start;  // first position of the group in the active list
    uint64_t item_start;  // first work item of the group
    uint32_t sweep_bits;  // swept: L, the key bits enumerated inside a partition; else 0
    uint32_t sweep_qc;    // swept: query chunks per partition
    uint64_t sweep_start; // first sweep item of the group (in each XCD's share)
    uint32_t final;       // 1: the round finishes step t of its queries (the last
                          // portion of a step cut by the work quantum, or all of it)
    uint32_t pad;
};

// Queries per sweep work item (one per lane), the smallest table that is
// swept, and the number of XCDs the partitions are dealt to.
constexpr uint32_t kSweepQueries = 64;   // at most one per lane
constexpr uint32_t kSweepMinBits = 20;
constexpr uint32_t kSweepXcds = 8;
constexpr uint32_t kSweepBatch = 4;   // consecutive sweep items claimed at once
// Device statistics slots of the engine: 0 probes, 1 candidates, 2 steps,
// 3 appended; from kStatRoundEnd, kTailPairs pairs (first wave end as a
// complement, last wave end) of the round kernel in the current round, a
// workgroup using pair blockIdx mod kTailPairs so that the atomics spread
// over many addresses; from kStatSweepEnd the same for the sweep kernels;
// kStatTail the sum of the rounds' tails in wall-clock ticks.
constexpr uint32_t kTailPairs = 64;
constexpr uint32_t kStatRoundEnd = 4, kStatSweepEnd = kStatRoundEnd + 2 * kTailPairs,
                   kStatTail = kStatSweepEnd + 2 * kTailPairs, kStatSlots = kStatTail + 1;
static_assert(kSweepQueries <= MIH_WAVE, "one lane per query of a sweep item");
// Partition kernel: the largest partition (key bits) whose occupancy bits
// are staged in LDS (2^18 bits = 32 KiB).
constexpr uint32_t kPartMaxBits = 18;
constexpr uint32_t kPartMinBits = 10;

// Device-resident control block of a search engine.
struct Control {
    uint32_t n_active;    // queries in the active list of the current round
    uint32_t n_groups;
    uint64_t total_items;
    uint32_t n_new;       // queries admitted since the last regroup
    uint32_t n_done;      // queries finished by the last advance
    uint32_t n_ovf;       // queries finished with an overflowed buffer
    uint32_t seq;         // rounds run (the spill flags of this round hold 2 seq, 2 seq + 1)
    uint64_t sweep_items; // items of the sweep kernel per XCD in the current round
};

// A piece of a huge bucket offered to every wave of the round kernel:
// table positions [pos, pos + len) of step t's table, for query slot.
struct SpillRec {
    uint32_t slot, t, pos, len;
};
constexpr uint32_t kSpillPiece = 1024;      // codes per piece
constexpr uint32_t kSpillCap = 1u << 20;    // pieces one round can offer

// One admitted query: its slot and the state it starts from.
struct AdmitRec {
    uint32_t slot, k, cap, tau0;
    uint32_t max_t;       // stop after this step at the latest (~0: no limit)
    uint32_t budget;      // stop once this many distinct codes were met (0: no limit)
    uint64_t buf_off;     // first buffer entry of the slot
    uint64_t query;       // device address of the query's words
    uint64_t out_ids;     // device address of the query's output row
    uint64_t out_dists;
};

struct MihArgs {
    const TableDev *tables;   // [m]
    const uint64_t *codes;    // database codes (read in INDIRECT mode)
    uint64_t n;
    uint32_t W, m, bits;
    uint32_t t_all;           // after this step every code has been found
    uint32_t tm;              // table layout: TM_DIRECT, TM_SORTED or TM_GROUPED
    uint32_t inline_codes;    // INLINE codes
    uint32_t chunk;           // masks per work item (multiple of 64 J)
    uint32_t J;               // masks per lane per iteration: 4, 8 or 16
    uint32_t occ_filter;      // DIRECT: test the occupancy bitmap before the offsets
    uint32_t sweep_shift;     // sweep a group when its probes reach 2^s >> sweep_shift (0: never)
    uint32_t sweep_bits;      // key bits enumerated inside one sweep partition
    uint32_t sweep_part;      // swept groups run in the partition kernel (occupancy tables)
    uint32_t part_bits;       // partition kernel: key bits of a partition (<= kPartMaxBits)
    uint32_t sweep_q;         // queries per sweep work item
    uint32_t look_items;      // a round may take further steps of its groups
                              // while its items stay within this (0: never)
    uint32_t quantum_items;   // most work items of one query per round (0: a whole
                              // step); a step with more continues in the next round
    uint32_t *cursor;         // [slots] items of the current step already run
    uint32_t look_max;        // most steps of a group per round (<= kLookMax)
    uint64_t look_masks;      // ... and while its shell masks stay within this
    QueryBatch qb;            // per-slot state (qb.queries is slot storage)
    uint32_t *t;              // [slots] current step of each query
    uint32_t *max_t;          // [slots] last step allowed (approximate search), or ~0
    uint32_t *budget;         // [slots] distinct codes after which to stop, or 0
    uint32_t *uniq;           // [slots] distinct codes met so far (when count_unique)
    uint32_t count_unique;    // some admitted query has a budget: count distinct codes
    uint64_t *out_ids;        // [slots] output row of each query
    uint64_t *out_dists;      // [slots]
    uint32_t *active;         // [slots] active list, grouped by step
    uint32_t *active_tmp;     // [slots] scratch of the regroup
    uint32_t *next_t;         // [slots] next step per active entry, or ~0
    uint32_t *new_slots;      // [slots] queries admitted since the last regroup
    uint32_t *done_list;      // [slots]
    uint32_t *ovf_list;       // [slots]
    Group *groups;            // [t_all + 1]
    Control *ctrl;
    unsigned long long *work; // work-item counter
    unsigned long long *work_sweep; // [kSweepXcds] work-item counters of the sweep kernel
    unsigned long long *stats;// [kStatSlots] counters (probes, candidates, ...)
    // Buckets of more than spill_min codes (0: never) are cut into pieces of
    // kSpillPiece codes that any wave of the round kernel may take: piece i
    // is offered once spill_flag[i] = 2 seq (the round's sequence number)
    // and taken by whoever turns it into 2 seq + 1.
    SpillRec *spill;                  // [spill_cap]
    uint32_t *spill_flag;             // [spill_cap]
    unsigned long long *spill_tail;   // pieces reserved this round
    unsigned long long *spill_next;   // next piece offered to helping waves
    uint32_t spill_cap;
    uint32_t spill_min;
};

hipError_t mih_round(const MihArgs &A, uint32_t grid, hipStream_t s);
// The swept groups of the round (returns at once when there are none).
hipError_t mih_sweep(const MihArgs &A, uint32_t grid, hipStream_t s);
// Workgroups per CU of a kernel (which: 0 round, 1 sweep, 2 partition,
// 3 round with huge buckets shared in pieces).
int mih_round_occupancy(uint32_t W, uint32_t tm, bool inline_codes, uint32_t J, int which,
                        uint32_t part_bits);
// One launch for a small batch of exact queries: `groups` workgroups per
// query run every step and the last to leave writes the top-k rows.
struct SmallArgs {
    uint32_t nq;
    uint32_t blocks;          // workgroups of the launch
    const uint32_t *first;    // [nq + 1] first workgroup of each query (query q has
                              // first[q + 1] - first[q] >= 1 workgroups)
    const uint32_t *query_of; // [blocks] the query of each workgroup
    const uint64_t *row_off;  // [nq] output row of each query
    uint32_t *out_ids, *out_dists;
    uint32_t *stop;           // [nq] ~0, then the step after which the query stopped
    uint32_t *exits;          // [nq] 0: workgroups that have left
    uint32_t *step_cnt;       // [nq][t_all + 1] 0: workgroups done with each step
    uint32_t *ovf_list;       // queries whose buffer overflowed (no rows written)
    uint32_t *ovf_count;      // 0 on entry
};
// A.qb describes the batch (queries [nq][W], k, cap, buf_off; tau = bits,
// count = 0 and hist = 0 on entry); A.stats (4 counters) zero on entry.
hipError_t mih_small(const MihArgs &A, const SmallArgs &S, hipStream_t s);
// Workgroups per CU of the one-launch kernel.
int mih_small_occupancy(uint32_t W, uint32_t tm, bool inline_codes, uint32_t J);
// Whether the partition kernel exists for this layout.
bool mih_part_kernel_ok(uint32_t W, uint32_t tm, bool inline_codes, uint32_t J);
bool mih_probes_per_lane_ok(uint32_t J);
// Start of a round: merge survivors and new queries into the active list.
hipError_t mih_regroup(const MihArgs &A, hipStream_t s);
// End of a round: termination tests; max_slots bounds the active list.
hipError_t mih_advance(const MihArgs &A, uint32_t max_slots, hipStream_t s);
// Admission of n queries described by rec (device memory).
hipError_t mih_admit(const MihArgs &A, const AdmitRec *rec, uint32_t n, hipStream_t s);

}  // namespace mih
