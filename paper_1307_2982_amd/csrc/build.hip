// Table construction (Algorithm 1) on the device.
//
// For each substring j the build produces the ids of all codes ordered by
// (substring value, id): a stable LSD radix sort of (value, id) pairs whose
// ids start in ascending order.  A bucket (all codes sharing a substring
// value, Section 2) is then a contiguous run of that order, located either
// through direct offsets (off[v] = number of codes whose value is below v,
// one entry per possible value as in the direct-address tables of Section 6)
// or through the sorted values and a prefix directory.
#include "mih_common.h"

namespace {

constexpr uint32_t kItems = 16;
constexpr uint32_t kTile = MIH_BLOCK * kItems;

template <int W>
__global__ __launch_bounds__(MIH_BLOCK) void extract_keys_kernel(const uint64_t *__restrict__ codes,
                                                                 uint64_t n, TableDev T, uint32_t *keys,
                                                                 uint32_t *ids)
{
    uint64_t i = (uint64_t)blockIdx.x * MIH_BLOCK + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * MIH_BLOCK;
    for (; i < n; i += stride) {
        uint64_t c[W];
        load_code<W>(codes + i * W, c);
        keys[i] = table_key<W>(c, T);
        ids[i] = (uint32_t)i;
    }
}

__global__ __launch_bounds__(MIH_BLOCK) void rs_upsweep(const uint32_t *__restrict__ keys, uint64_t n,
                                                        uint32_t shift, uint32_t mask,
                                                        uint32_t *__restrict__ counts, uint32_t nblocks)
{
    __shared__ uint32_t h[256];
    const uint32_t tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    for (uint32_t j = 0; j < kItems; ++j) {
        uint64_t p = base + j * MIH_BLOCK + tid;
        if (p < n) atomicAdd(&h[(keys[p] >> shift) & mask], 1u);
    }
    __syncthreads();
    counts[(uint64_t)tid * nblocks + blockIdx.x] = h[tid];
}

// Scatter one tile in stable order: element p goes to the start of its digit
// for this tile plus the number of earlier elements of the tile with the same
// digit.  Elements are taken in rounds of 256 in index order; within a wave
// the rank among equal digits comes from eight ballots.
__global__ __launch_bounds__(MIH_BLOCK) void rs_downsweep(const uint32_t *__restrict__ keys,
                                                          const uint32_t *__restrict__ ids,
                                                          uint32_t *__restrict__ okeys,
                                                          uint32_t *__restrict__ oids, uint64_t n,
                                                          uint32_t shift, uint32_t mask,
                                                          const uint32_t *__restrict__ offsets,
                                                          uint32_t nblocks)
{
    __shared__ uint32_t base_off[256];
    __shared__ uint32_t wcount[4][256];
    const uint32_t tid = threadIdx.x, wave = tid >> 6;
    base_off[tid] = offsets[(uint64_t)tid * nblocks + blockIdx.x];
    for (int w = 0; w < 4; ++w) wcount[w][tid] = 0;
    __syncthreads();
    const uint64_t tile = (uint64_t)blockIdx.x * kTile;
    const uint64_t below = (1ull << lane_id()) - 1;
    for (uint32_t j = 0; j < kItems; ++j) {
        const uint64_t p = tile + j * MIH_BLOCK + tid;
        const bool valid = p < n;
        uint32_t key = valid ? keys[p] : 0u;
        uint32_t id = valid ? ids[p] : 0u;
        uint32_t d = (key >> shift) & mask;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        uint32_t rank = (uint32_t)__popcll(peers & below);
        if (valid && rank == 0) wcount[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = base_off[d] + rank;
            for (uint32_t w = 0; w < wave; ++w) pos += wcount[w][d];
            okeys[pos] = key;
            oids[pos] = id;
        }
        __syncthreads();
        base_off[tid] += wcount[0][tid] + wcount[1][tid] + wcount[2][tid] + wcount[3][tid];
        for (int w = 0; w < 4; ++w) wcount[w][tid] = 0;
        __syncthreads();
    }
}

// Bucket starts: off[v] = i for the first i whose value is v; empty buckets
// keep the fill value and are completed by a suffix minimum.
__global__ __launch_bounds__(MIH_BLOCK) void mark_bucket_starts(const uint32_t *__restrict__ keys,
                                                                uint64_t n, uint32_t shift,
                                                                uint32_t *off, uint64_t nbuckets)
{
    uint64_t i = (uint64_t)blockIdx.x * MIH_BLOCK + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * MIH_BLOCK;
    if (i == 0) off[nbuckets] = (uint32_t)n;
    for (; i < n; i += stride) {
        uint32_t v = keys[i] >> shift;
        if (i == 0 || (keys[i - 1] >> shift) != v) off[v] = (uint32_t)i;
    }
}

// Bit v of occ = [bucket v is non-empty] = [off[v+1] > off[v]].
__global__ __launch_bounds__(MIH_BLOCK) void occupancy_kernel(const uint32_t *__restrict__ off,
                                                              uint64_t nbuckets, uint32_t *occ)
{
    const uint64_t nwords = (nbuckets + 31) / 32;
    uint64_t w = (uint64_t)blockIdx.x * MIH_BLOCK + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * MIH_BLOCK;
    for (; w < nwords; w += stride) {
        uint32_t word = 0;
        const uint64_t v0 = w * 32;
        uint32_t prev = off[v0];
        for (uint32_t b = 0; b < 32 && v0 + b < nbuckets; ++b) {
            const uint32_t nxt = off[v0 + b + 1];
            if (nxt > prev) word |= 1u << b;
            prev = nxt;
        }
        occ[w] = word;
    }
}

// Record g of a GROUPED table: the occupancy bits of buckets 32g..32g+31
// and, in the high half, the position of the group's first code.
__global__ __launch_bounds__(MIH_BLOCK) void group_records_kernel(const uint32_t *__restrict__ off,
                                                                  uint64_t nbuckets, uint64_t *grp)
{
    const uint64_t ngroups = (nbuckets + 31) / 32;
    uint64_t g = (uint64_t)blockIdx.x * MIH_BLOCK + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * MIH_BLOCK;
    for (; g < ngroups; g += stride) {
        uint32_t word = 0;
        const uint64_t v0 = g * 32;
        const uint32_t first = off[v0];
        uint32_t prev = first;
        for (uint32_t b = 0; b < 32 && v0 + b < nbuckets; ++b) {
            const uint32_t nxt = off[v0 + b + 1];
            if (nxt > prev) word |= 1u << b;
            prev = nxt;
        }
        grp[g] = ((uint64_t)first << 32) | word;
    }
}

__global__ __launch_bounds__(MIH_BLOCK) void bucket_heads_kernel(const uint32_t *__restrict__ off,
                                                                 uint64_t nbuckets,
                                                                 const uint64_t *__restrict__ codes,
                                                                 BucketHead *head)
{
    uint64_t v = (uint64_t)blockIdx.x * MIH_BLOCK + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * MIH_BLOCK;
    for (; v <= nbuckets; v += stride) {
        const uint32_t b0 = off[v];
        const uint32_t c = v < nbuckets ? off[v + 1] - b0 : 0u;
        BucketHead h;
        h.code = c ? codes[b0] : 0ull;
        h.start = b0;
        h.count = c;
        head[v] = h;
    }
}

template <int W>
__global__ __launch_bounds__(MIH_BLOCK) void gather_codes_kernel(const uint64_t *__restrict__ codes,
                                                                 const uint32_t *__restrict__ ids,
                                                                 uint64_t n, uint64_t *__restrict__ out)
{
    uint64_t i = (uint64_t)blockIdx.x * MIH_BLOCK + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * MIH_BLOCK;
    for (; i < n; i += stride) {
        const uint64_t *src = codes + (uint64_t)ids[i] * W;
#pragma unroll
        for (int w = 0; w < W; ++w) out[i * W + w] = src[w];
    }
}

uint32_t grid_for(uint64_t n)
{
    uint64_t b = (n + MIH_BLOCK - 1) / MIH_BLOCK;
    if (b < 1) b = 1;
    if (b > 65536ull * 4) b = 65536ull * 4;
    return (uint32_t)b;
}

}  // namespace

namespace mih {

hipError_t extract_keys(const uint64_t *codes, uint64_t n, uint32_t W, const TableDev &T,
                        uint32_t *keys, uint32_t *ids, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const uint32_t g = grid_for(n);
    switch (W) {
    case 1: extract_keys_kernel<1><<<g, MIH_BLOCK, 0, s>>>(codes, n, T, keys, ids); break;
    case 2: extract_keys_kernel<2><<<g, MIH_BLOCK, 0, s>>>(codes, n, T, keys, ids); break;
    case 3: extract_keys_kernel<3><<<g, MIH_BLOCK, 0, s>>>(codes, n, T, keys, ids); break;
    case 4: extract_keys_kernel<4><<<g, MIH_BLOCK, 0, s>>>(codes, n, T, keys, ids); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

uint64_t radix_tmp_words(uint64_t n)
{
    uint64_t nb = (n + kTile - 1) / kTile;
    if (nb == 0) nb = 1;
    return 256 * nb + scan_tmp_words(256 * nb);
}

hipError_t radix_sort_pairs(uint32_t *&keys, uint32_t *&ids, uint32_t *&keys2, uint32_t *&ids2,
                            uint64_t n, uint32_t key_bits, uint32_t *tmp, hipStream_t s)
{
    if (n <= 1 || key_bits == 0) return hipSuccess;
    const uint64_t nb = (n + kTile - 1) / kTile;
    if (nb > 0xFFFFFFFFull / 256) return hipErrorInvalidValue;
    uint32_t *counts = tmp;
    uint32_t *scan_tmp = tmp + 256 * nb;
    for (uint32_t shift = 0; shift < key_bits; shift += 8) {
        uint32_t bits = key_bits - shift < 8 ? key_bits - shift : 8;
        uint32_t mask = (1u << bits) - 1;
        rs_upsweep<<<(uint32_t)nb, MIH_BLOCK, 0, s>>>(keys, n, shift, mask, counts, (uint32_t)nb);
        hipError_t e = exclusive_sum_u32(counts, counts, 256 * nb, scan_tmp, s);
        if (e != hipSuccess) return e;
        rs_downsweep<<<(uint32_t)nb, MIH_BLOCK, 0, s>>>(keys, ids, keys2, ids2, n, shift, mask,
                                                         counts, (uint32_t)nb);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint32_t *t = keys; keys = keys2; keys2 = t;
        t = ids; ids = ids2; ids2 = t;
    }
    return hipSuccess;
}

hipError_t bucket_offsets(const uint32_t *sorted_keys, uint64_t n, uint32_t shift, uint32_t *off,
                          uint64_t nbuckets, uint32_t *tmp, hipStream_t s)
{
    hipError_t e = fill_u32(off, nbuckets + 1, 0xFFFFFFFFu, s);
    if (e != hipSuccess) return e;
    mark_bucket_starts<<<grid_for(n), MIH_BLOCK, 0, s>>>(sorted_keys, n, shift, off, nbuckets);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return suffix_min_u32(off, off, nbuckets + 1, tmp, s);
}

hipError_t occupancy_bits(const uint32_t *off, uint64_t nbuckets, uint32_t *occ, hipStream_t s)
{
    occupancy_kernel<<<grid_for((nbuckets + 31) / 32), MIH_BLOCK, 0, s>>>(off, nbuckets, occ);
    return hipGetLastError();
}

hipError_t bucket_heads(const uint32_t *off, uint64_t nbuckets, const uint64_t *codes, BucketHead *head,
                        hipStream_t s)
{
    bucket_heads_kernel<<<grid_for(nbuckets + 1), MIH_BLOCK, 0, s>>>(off, nbuckets, codes, head);
    return hipGetLastError();
}

hipError_t group_records(const uint32_t *off, uint64_t nbuckets, uint64_t *grp, hipStream_t s)
{
    group_records_kernel<<<grid_for((nbuckets + 31) / 32), MIH_BLOCK, 0, s>>>(off, nbuckets, grp);
    return hipGetLastError();
}

hipError_t gather_codes(const uint64_t *codes, const uint32_t *ids, uint64_t n, uint32_t W,
                        uint64_t *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const uint32_t g = grid_for(n);
    switch (W) {
    case 1: gather_codes_kernel<1><<<g, MIH_BLOCK, 0, s>>>(codes, ids, n, out); break;
    case 2: gather_codes_kernel<2><<<g, MIH_BLOCK, 0, s>>>(codes, ids, n, out); break;
    case 3: gather_codes_kernel<3><<<g, MIH_BLOCK, 0, s>>>(codes, ids, n, out); break;
    case 4: gather_codes_kernel<4><<<g, MIH_BLOCK, 0, s>>>(codes, ids, n, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mih
