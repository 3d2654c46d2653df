// Shared definitions of the MI355X multi-index hashing library: device
// helpers, the layouts that kernels and the host runtime agree on, and the
// host-side launch wrappers implemented in the .hip files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mih.h"

#define MIH_WAVE 64
#define MIH_BLOCK 256
#define MIH_BINOM_N 33   // C(n, r) for 0 <= n, r <= 32

// ---------------------------------------------------------------- device math

__device__ __forceinline__ uint32_t popc64(uint64_t x) { return (uint32_t)__popcll(x); }

// Hamming distance of two codes of W words (one xor and one popcount per 64
// bits, Section 6).
template <int W>
__device__ __forceinline__ uint32_t hamming(const uint64_t (&a)[W], const uint64_t (&b)[W])
{
    uint32_t d = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) d += popc64(a[w] ^ b[w]);
    return d;
}

// Bits [start, start + len) of a code, first bit least significant
// (len <= 32; the run may straddle two words).
template <int W>
__device__ __forceinline__ uint32_t substring(const uint64_t (&c)[W], uint32_t start, uint32_t len)
{
    uint32_t w0 = start >> 6, sh = start & 63;
    uint64_t v = 0;
#pragma unroll
    for (int w = 0; w < W; ++w)
        if ((uint32_t)w == w0) v = c[w] >> sh;
    if (sh + len > 64) {
#pragma unroll
        for (int w = 0; w < W; ++w)
            if ((uint32_t)w == w0 + 1) v |= c[w] << (64 - sh);
    }
    uint64_t mask = (len >= 64) ? ~0ull : ((1ull << len) - 1);
    return (uint32_t)(v & mask);
}

template <int W>
__device__ __forceinline__ void load_code(const uint64_t *__restrict__ p, uint64_t (&c)[W])
{
#pragma unroll
    for (int w = 0; w < W; ++w) c[w] = p[w];
}

// Relaxed device-scope load that bypasses the per-CU cache, for counters that
// other workgroups update with atomics.
__device__ __forceinline__ uint32_t load_relaxed(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long load_relaxed(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t x)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int off = 1; off < MIH_WAVE; off <<= 1) {
        uint32_t y = __shfl_up(x, off, MIH_WAVE);
        if (lane >= (uint32_t)off) x += y;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_broadcast_last(uint32_t x)
{
    return __shfl(x, MIH_WAVE - 1, MIH_WAVE);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x)
{
    return wave_broadcast_last(wave_inclusive_sum(x));
}

// Number of lanes below this one whose bit is set in `mask`.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Keeps the compiler from moving LDS accesses across this point and waits for
// this wave's outstanding LDS operations (lanes of one wave then see each
// other's LDS writes).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ----------------------------------------------------------- query state

// Per-call state of a batch of queries (structure of arrays, device memory).
// Each query keeps a buffer of packed candidates (d << 32 | id), a histogram
// of the distances of the kept candidates, and the current distance bound
// tau: a candidate is kept only if d <= tau.  tau only decreases and never
// drops below the true k-th distance, because it is derived from counts of
// real, distinct codes.
struct QueryBatch {
    const uint64_t *queries;   // [nq][W]
    const uint32_t *k;         // [nq]
    uint32_t *tau;             // [nq]
    uint32_t *count;           // [nq] candidates offered (may exceed cap)
    const uint32_t *cap;       // [nq]
    const uint64_t *buf_off;   // [nq]
    uint64_t *buf;             // packed candidates
    uint32_t *hist;            // [nq][bits + 1]
    uint32_t nq;
    uint32_t bits;
};

// Keep candidate (d, id) for query q: one atomic per wave reserves the slots
// (ballot + mbcnt), one atomic per kept candidate counts its distance.
__device__ __forceinline__ void append_candidates(const QueryBatch &qb, uint32_t q, bool keep,
                                                  uint32_t d, uint32_t id)
{
    uint64_t ballot = __ballot(keep);
    if (!ballot) return;
    uint32_t total = (uint32_t)__popcll(ballot);
    uint32_t leader = (uint32_t)__ffsll((long long)ballot) - 1;
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(&qb.count[q], total);
    base = __shfl(base, leader, MIH_WAVE);
    if (keep) {
        uint32_t slot = base + lanes_below(ballot);
        if (slot < qb.cap[q])
            qb.buf[qb.buf_off[q] + slot] = ((uint64_t)d << 32) | id;
        atomicAdd(&qb.hist[(uint64_t)q * (qb.bits + 1) + d], 1u);
    }
}

// Recompute tau for query q from its histogram (wave-cooperative): the
// smallest D whose cumulative count reaches k.  Any snapshot of the counters
// gives a valid bound; at a quiescent point it is exact.  Returns the new
// bound (the old one if k is not reached).
__device__ __forceinline__ uint32_t tighten_tau(const QueryBatch &qb, uint32_t q, uint32_t tau)
{
    const uint32_t nb = qb.bits + 1;
    const uint32_t per = (nb + MIH_WAVE - 1) / MIH_WAVE;   // <= 5
    const uint32_t lane = lane_id();
    const uint32_t *h = qb.hist + (uint64_t)q * nb;
    const uint32_t k = qb.k[q];
    uint32_t v[5];
    uint32_t local = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        uint32_t e = lane * per + i;
        v[i] = (i < (int)per && e < nb) ? load_relaxed(h + e) : 0u;
        local += v[i];
    }
    uint32_t incl = wave_inclusive_sum(local);
    uint32_t run = incl - local;
    uint32_t first = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        run += v[i];
        uint32_t e = lane * per + i;
        if (first == 0xFFFFFFFFu && i < (int)per && e < nb && run >= k && k > 0) first = e;
    }
    uint64_t has = __ballot(first != 0xFFFFFFFFu);
    if (!has) return tau;
    uint32_t src = (uint32_t)__ffsll((long long)has) - 1;
    uint32_t D = __shfl(first, src, MIH_WAVE);
    if (D < tau) {
        if (lane == 0) atomicMin(&qb.tau[q], D);
        tau = D;
    }
    return tau;
}

// Ascending sort of P (a power of two, at most 4096) packed entries in LDS by
// one workgroup of any size (bitonic network); every thread of the block must
// call it.
__device__ __forceinline__ void block_bitonic_sort(uint64_t *v, uint32_t P)
{
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = tid; i < P / 2; i += nt) {
                const uint32_t lo = 2 * stride * (i / stride) + (i % stride);
                const uint32_t hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t x = v[lo], y = v[hi];
                if ((x > y) == up) { v[lo] = y; v[hi] = x; }
            }
            __syncthreads();
        }
    }
}

// HEADS tables: a bucket's offset beside its first code (16 bytes, so that
// the entries of v and v + 1 usually share a line).
struct BucketHead {
    uint64_t code;    // the bucket's first code in table order (0 if empty)
    uint32_t start;   // offset of the bucket: codes with a smaller value
    uint32_t count;   // codes in the bucket
};

// `count` packed entries moved from entry offset src to entry offset dst.
struct RnnMove {
    uint64_t src, dst;
    uint32_t count, pad;
};

// ----------------------------------------------------------- index layout

struct TableDev {
    uint64_t mask[4];        // the code bits of this substring (words 0..W-1)
    uint8_t order[32];       // permuted: key bit k is code bit order[k]
    uint32_t permuted;       // 0: key bits are code bits [start, start + len)
    uint32_t pad0;
    const uint32_t *off;     // DIRECT: [2^len + 1]
    const uint32_t *occ;     // DIRECT: [2^len / 32 (at least 1)] bit v: bucket v non-empty
    const BucketHead *head;  // HEADS: [2^len + 1]
    const uint64_t *grp;     // GROUPED: [2^len / 32 (at least 1)]: bits 0..31 occupancy of
                             // buckets 32g..32g+31, bits 32..63 position of the group's first code
    const uint32_t *keys;    // SORTED: [n]
    const uint32_t *dir;     // SORTED: [2^dir_bits + 1]
    const uint32_t *ids;     // [n]
    const uint64_t *codes;   // INLINE: [n][W]
    uint32_t len, start, dir_bits, pad;
};

// Word idx of a code held in registers (W <= 4, idx < W).
template <int W>
__device__ __forceinline__ uint64_t code_word(const uint64_t (&c)[W], uint32_t idx)
{
    uint64_t v = c[0];
#pragma unroll
    for (int w = 1; w < W; ++w)
        if ((uint32_t)w == idx) v = c[w];
    return v;
}

// Key of a code in table T: its substring bits, contiguous or in the table's
// bit order (substring optimisation, Section 5.5).
template <int W>
__device__ __forceinline__ uint32_t table_key(const uint64_t (&c)[W], const TableDev &T)
{
    if (!T.permuted) return substring<W>(c, T.start, T.len);
    uint32_t key = 0;
    for (uint32_t k = 0; k < T.len; ++k) {
        const uint32_t b = T.order[k];
        key |= (uint32_t)((code_word<W>(c, b >> 6) >> (b & 63)) & 1u) << k;
    }
    return key;
}

// Hamming distance of two codes restricted to table T's substring, from
// their xor.
template <int W>
__device__ __forceinline__ uint32_t table_dist(const uint64_t (&x)[W], const TableDev &T)
{
    uint32_t d = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) d += __popcll(x[w] & T.mask[w]);
    return d;
}

// ----------------------------------------------------------- host wrappers

namespace mih {

// scan.hip
hipError_t fill_u32(uint32_t *p, uint64_t n, uint32_t value, hipStream_t s);
hipError_t fill_u64(uint64_t *p, uint64_t n, uint64_t value, hipStream_t s);
// Exclusive prefix sum of n uint32 values (in == out allowed).  tmp must hold
// scan_tmp_words(n) uint32.
uint64_t scan_tmp_words(uint64_t n);
hipError_t exclusive_sum_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *tmp,
                             hipStream_t s);
// Inclusive suffix minimum: out[i] = min(in[i..n)).
hipError_t suffix_min_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *tmp,
                          hipStream_t s);
// dst[i] = rows[list[i]] for rows of W words.
hipError_t gather_rows(const uint64_t *rows, const uint32_t *list, uint32_t nlist, uint32_t W,
                       uint64_t *dst, hipStream_t s);

// build.hip
// keys[i] = key of code i in table T (T's bit layout fields only), ids[i] = i.
hipError_t extract_keys(const uint64_t *codes, uint64_t n, uint32_t W, const TableDev &T,
                        uint32_t *keys, uint32_t *ids, hipStream_t s);
uint64_t radix_tmp_words(uint64_t n);
// Stable sort of (keys, ids) by the low `key_bits` bits of keys, ping-ponging
// between (keys, ids) and (keys2, ids2); on return (keys, ids) name the
// buffers that hold the result.  tmp must hold radix_tmp_words(n) uint32.
hipError_t radix_sort_pairs(uint32_t *&keys, uint32_t *&ids, uint32_t *&keys2, uint32_t *&ids2,
                            uint64_t n, uint32_t key_bits, uint32_t *tmp, hipStream_t s);
// off[v] = number of sorted keys whose (key >> shift) is below v, for
// v in [0, nbuckets]; tmp as for suffix_min_u32(nbuckets + 1).
hipError_t bucket_offsets(const uint32_t *sorted_keys, uint64_t n, uint32_t shift,
                          uint32_t *off, uint64_t nbuckets, uint32_t *tmp, hipStream_t s);
hipError_t gather_codes(const uint64_t *codes, const uint32_t *ids, uint64_t n, uint32_t W,
                        uint64_t *out, hipStream_t s);
// occ[v / 32] bit v % 32 = [off[v + 1] > off[v]] for v < nbuckets.
hipError_t occupancy_bits(const uint32_t *off, uint64_t nbuckets, uint32_t *occ, hipStream_t s);
// head[v] = {first code of bucket v (codes in table order, 64-bit), off[v]}
// for v <= nbuckets.
hipError_t bucket_heads(const uint32_t *off, uint64_t nbuckets, const uint64_t *codes,
                        BucketHead *head, hipStream_t s);
// grp[g] = (off[32 g] << 32) | occupancy bits of buckets 32g..32g+31.
hipError_t group_records(const uint32_t *off, uint64_t nbuckets, uint64_t *grp, hipStream_t s);

// linscan.hip
struct LinscanArgs {
    const uint64_t *codes;
    uint64_t n;
    QueryBatch qb;               // qb.tau holds linscan_pad(nq) entries
    const uint64_t *queries_padded;   // [linscan_pad(nq)][W], zero tail
    uint32_t W;
};
// Rows of the padded query and bound arrays that the scan reads.
inline uint32_t linscan_pad(uint32_t nq) { return (nq + 15) / 16 * 16; }
hipError_t linscan_init(const LinscanArgs &a, uint64_t sample, const uint32_t *tau0,
                        hipStream_t s);
hipError_t linscan_run(const LinscanArgs &a, uint32_t num_cus, hipStream_t s);

// api.hip: linscan_knn with every device buffer carved from the region
// [base, base + size) (256-byte aligned); allocates no device memory.
// MIH_ERR_CAPACITY when one query's pass or exact re-run does not fit.
mih_status linscan_check_args(const uint64_t *codes, uint64_t n, uint32_t bits,
                              const uint64_t *queries, uint32_t nq, uint32_t k,
                              const uint32_t *k_per_query, const uint32_t *out_ids,
                              const uint32_t *out_dists);
mih_status linscan_knn_in_region(const uint64_t *codes, uint64_t n, uint32_t bits,
                                 const uint64_t *queries, uint32_t nq, uint32_t k,
                                 const uint32_t *k_per_query, uint32_t *out_ids,
                                 uint32_t *out_dists, hipStream_t s, char *base, uint64_t size);

// topk.hip
struct FinalArgs {
    QueryBatch qb;
    const uint64_t *row_off;   // [nq]
    uint32_t *out_ids;
    uint32_t *out_dists;
    uint32_t *overflow_list;   // [nq] queries whose buffer overflowed
    uint32_t *overflow_count;  // device scalar
};
hipError_t find_overflow(const FinalArgs &a, hipStream_t s);
hipError_t finalize_topk(const FinalArgs &a, hipStream_t s);
// Finalize the listed queries; out_ids[q] / out_dists[q] are the device
// addresses of query q's output rows.
hipError_t finalize_list(const QueryBatch &qb, const uint32_t *list, uint32_t nlist,
                         const uint64_t *out_ids, const uint64_t *out_dists, hipStream_t s);
// Top-k rows of the first *count queries of list (count in device memory),
// skipping r-neighbour queries; grid workgroups share them.
hipError_t finalize_done(const QueryBatch &qb, const uint32_t *list, const uint32_t *count,
                         const uint64_t *out_ids, const uint64_t *out_dists, uint32_t grid,
                         hipStream_t s);
// For re-runs: per listed query, exact tau and the capacity it needs.
hipError_t exact_bounds(const QueryBatch &qb, const uint32_t *list, uint32_t nlist,
                        uint32_t *tau_out, uint32_t *cap_out, hipStream_t s);

}  // namespace mih
