// Launch interface of the multi-index search kernels (mih_query.hip).
#pragma once

#include "mih_common.h"

namespace mih {

// Active queries that share the same next step form a group; its work items
// are the chunks of that step's shell for each of its queries, numbered
// from item_start, query-major.
struct Group {
    uint32_t t;           // step to process
    uint32_t count;       // queries in the group
    uint32_t ipq;         // work items per query: ceil(C(s_a, r') / chunk)
    uint32_t slot_start;  // first slot of the group in the active list
    uint64_t item_start;  // first work item of the group
};

struct Control {
    uint32_t n_active;
    uint32_t n_groups;
    uint64_t total_items;
};

struct MihArgs {
    const TableDev *tables;   // [m]
    const uint64_t *codes;    // database codes (read in INDIRECT mode)
    uint64_t n;
    uint32_t W, m, bits;
    uint32_t t_all;           // after this step every code has been found
    uint32_t sorted;          // SORTED tables
    uint32_t inline_codes;    // INLINE codes
    uint32_t chunk;           // masks per work item (multiple of 64 J)
    uint32_t J;               // masks per lane per iteration: 4, 8 or 16
    QueryBatch qb;
    uint32_t *t;              // [nq] current step of each query
    const uint32_t *active;   // [n_active] query of each slot, grouped by step
    const Group *groups;
    const Control *ctrl;
    unsigned long long *work; // work-item counter
    unsigned long long *stats;// [2] probes, candidates
};

hipError_t mih_round(const MihArgs &A, uint32_t grid, hipStream_t s);
int mih_round_occupancy(uint32_t W, bool sorted, bool inline_codes, uint32_t J);
bool mih_probes_per_lane_ok(uint32_t J);
// Termination tests and regrouping after a round.  nq bounds the number of
// active slots.  A.ctrl and ctrl_out may be the same; new_active must differ
// from A.active.
hipError_t mih_advance(const MihArgs &A, uint32_t nq, uint32_t *next_t, uint32_t *new_active,
                       Group *groups, Control *ctrl_out, hipStream_t s);

}  // namespace mih
