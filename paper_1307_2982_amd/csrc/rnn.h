// Results of r-neighbour search (Alg. 2): every code within Hamming distance
// r of a query, a variable number per query.
//
// A query's search leaves its hits, packed as (d << 32 | id), unordered in its
// candidate buffer.  When a query finishes, its entries are moved into the
// arena of its request (a device array that grows by doubling), so the
// buffer can serve the next query at once.  When the whole request is done,
// each query's entries are sorted into ascending (distance, id) order and
// written to the request's output rows.
#pragma once

#include <vector>

#include "mih_common.h"

namespace mih {

// Largest per-query result sorted inside one workgroup's LDS; longer lists
// go through the device radix sort.
constexpr uint32_t kRnnLdsSort = 4096;

// Device buffers of a finished r-neighbour request.
struct RnnOut {
    uint64_t *offsets = nullptr;   // [nq + 1]: rows of query i at [offsets[i], offsets[i+1])
    uint32_t *ids = nullptr;       // [total]
    uint32_t *dists = nullptr;     // [total]
    uint64_t total = 0;
    uint32_t nq = 0;
};
void free_rnn_out(RnnOut &o);

class RnnCollector {
public:
    explicit RnnCollector(uint32_t nq) : start_(nq, 0), count_(nq, 0) {}
    ~RnnCollector();
    RnnCollector(const RnnCollector &) = delete;
    RnnCollector &operator=(const RnnCollector &) = delete;

    // Moves count[i] entries at src + src_off[i] (entry offsets) into the
    // arena as the entries of query query[i].  Synchronises the stream.
    hipError_t add(const uint64_t *src, const std::vector<uint32_t> &query,
                   const std::vector<uint64_t> &src_off, const std::vector<uint32_t> &count,
                   hipStream_t s);
    // Sorts every query's entries by (distance, id) and writes them into
    // newly allocated output buffers (owned by `out` afterwards).  `bits` is
    // the code length (distances are at most bits).
    hipError_t finish(uint32_t bits, hipStream_t s, RnnOut &out);

private:
    hipError_t reserve(uint64_t entries, hipStream_t s);
    hipError_t moves_room(uint64_t n);

    std::vector<uint64_t> start_;   // arena offset of each query's entries
    std::vector<uint32_t> count_;
    uint64_t *arena_ = nullptr;
    uint64_t cap_ = 0, used_ = 0;
    RnnMove *moves_ = nullptr;
    uint64_t moves_cap_ = 0;
};

// out[i] = count[list[i]] for i < n.
hipError_t gather_counts(const uint32_t *count, const uint32_t *list, uint32_t n, uint32_t *out,
                         hipStream_t s);

}  // namespace mih
