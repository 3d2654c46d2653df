// Exact top-k from a query's candidate buffer.
//
// The buffer holds every code whose distance is at most the final bound
// (plus, for multi-index search, some farther codes kept before the bound
// fell), and the histogram counts the kept distances.  The k-th distance D is
// the smallest distance whose cumulative count reaches min(k, kept); every
// kept code closer than D is in the result, and among the codes at distance D
// the ones with the lowest ids fill the remaining places (found by a radix
// select on the id when there are more of them than places).  The selected
// entries, packed as (d << 32 | id), are sorted in LDS so that the output is
// in ascending (distance, id) order.
#include "mih_common.h"

namespace {

__device__ __forceinline__ void kth_distance(const QueryBatch &qb, uint32_t q, uint32_t &kk,
                                             uint32_t &D, uint32_t &below, uint32_t &at_D)
{
    const uint32_t nb = qb.bits + 1;
    const uint32_t *h = qb.hist + (uint64_t)q * nb;
    uint64_t total = 0;
    for (uint32_t d = 0; d < nb; ++d) total += h[d];
    const uint32_t k = qb.k[q];
    kk = total < k ? (uint32_t)total : k;
    D = 0; below = 0; at_D = 0;
    if (kk == 0) return;
    uint32_t cum = 0;
    for (uint32_t d = 0; d < nb; ++d) {
        if (cum + h[d] >= kk) { D = d; below = cum; at_D = h[d]; return; }
        cum += h[d];
    }
}

// One workgroup finalizes query q into oid[0..k), odist[0..k).
__device__ void finalize_one(const QueryBatch &qb, uint32_t q, uint32_t *oid, uint32_t *odist)
{
    __shared__ uint64_t sel[MIH_K_MAX];
    __shared__ uint32_t digit_hist[256];
    __shared__ uint32_t s_kk, s_D, s_below, s_at_D, s_prefix, s_pmask, s_remaining, s_count;
    const uint32_t tid = threadIdx.x;
    const uint32_t k = qb.k[q];
    if (k == 0) return;
    if (tid == 0) {
        uint32_t kk, D, below, at_D;
        kth_distance(qb, q, kk, D, below, at_D);
        s_kk = kk; s_D = D; s_below = below; s_at_D = at_D;
        s_prefix = 0; s_pmask = 0; s_remaining = kk - below; s_count = 0;
    }
    __syncthreads();
    const uint32_t kk = s_kk, D = s_D;
    const uint32_t cnt = qb.count[q], cap = qb.cap[q];
    const uint32_t nbuf = cnt < cap ? cnt : cap;
    const uint64_t *buf = qb.buf + qb.buf_off[q];

    uint32_t id_cut = 0xFFFFFFFFu;
    if (kk > 0 && s_at_D > kk - s_below) {
        // radix select: the (kk - below)-th smallest id among entries at D
        for (int shift = 24; shift >= 0; shift -= 8) {
            digit_hist[tid] = 0;
            __syncthreads();
            const uint32_t prefix = s_prefix, pmask = s_pmask;
            for (uint32_t e = tid; e < nbuf; e += MIH_BLOCK) {
                uint64_t v = buf[e];
                uint32_t d = (uint32_t)(v >> 32), id = (uint32_t)v;
                if (d == D && (id & pmask) == prefix) atomicAdd(&digit_hist[(id >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (tid == 0) {
                uint32_t rem = s_remaining, cum = 0, dg = 0;
                for (dg = 0; dg < 256; ++dg) {
                    if (cum + digit_hist[dg] >= rem) break;
                    cum += digit_hist[dg];
                }
                s_remaining = rem - cum;
                s_prefix = prefix | (dg << shift);
                s_pmask = pmask | (255u << shift);
            }
            __syncthreads();
        }
        id_cut = s_prefix;
    }

    for (uint32_t e = tid; e < nbuf; e += MIH_BLOCK) {
        uint64_t v = buf[e];
        uint32_t d = (uint32_t)(v >> 32), id = (uint32_t)v;
        if (kk > 0 && (d < D || (d == D && id <= id_cut))) {
            uint32_t p = atomicAdd(&s_count, 1u);
            if (p < MIH_K_MAX) sel[p] = v;
        }
    }
    __syncthreads();
    uint32_t P = 1;
    while (P < kk) P <<= 1;
    for (uint32_t i = kk + tid; i < P; i += MIH_BLOCK) sel[i] = ~0ull;
    __syncthreads();
    block_bitonic_sort(sel, P);
    for (uint32_t r = tid; r < k; r += MIH_BLOCK) {
        if (r < kk) {
            oid[r] = (uint32_t)sel[r];
            odist[r] = (uint32_t)(sel[r] >> 32);
        } else {
            oid[r] = MIH_SENTINEL;
            odist[r] = MIH_SENTINEL;
        }
    }
}

__global__ __launch_bounds__(MIH_BLOCK) void finalize_kernel(mih::FinalArgs a)
{
    const uint32_t q = blockIdx.x;
    const uint64_t off = a.row_off[q];
    finalize_one(a.qb, q, a.out_ids + off, a.out_dists + off);
}

// Queries of a list, each with its own output row (device addresses).
__global__ __launch_bounds__(MIH_BLOCK) void finalize_list_kernel(QueryBatch qb, const uint32_t *list,
                                                                  const uint64_t *out_ids,
                                                                  const uint64_t *out_dists)
{
    const uint32_t q = list[blockIdx.x];
    finalize_one(qb, q, reinterpret_cast<uint32_t *>(out_ids[q]),
                 reinterpret_cast<uint32_t *>(out_dists[q]));
}

// The queries a round finished (count read on the device, so that the launch
// can sit in a captured graph): each workgroup takes every gridDim-th one.
// r-neighbour queries (k = 0xFFFFFFFF) have no top-k rows and are skipped.
__global__ __launch_bounds__(MIH_BLOCK) void finalize_done_kernel(QueryBatch qb, const uint32_t *list,
                                                                  const uint32_t *count,
                                                                  const uint64_t *out_ids,
                                                                  const uint64_t *out_dists)
{
    const uint32_t n = *count;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const uint32_t q = list[i];
        if (qb.k[q] == 0xFFFFFFFFu) continue;
        finalize_one(qb, q, reinterpret_cast<uint32_t *>(out_ids[q]),
                     reinterpret_cast<uint32_t *>(out_dists[q]));
        __syncthreads();   // finalize_one's shared state is reused by the next query
    }
}

__global__ __launch_bounds__(MIH_BLOCK) void find_overflow_kernel(QueryBatch qb, uint32_t *list,
                                                                  uint32_t *count)
{
    uint32_t q = blockIdx.x * MIH_BLOCK + threadIdx.x;
    if (q >= qb.nq) return;
    // a query with k = 0 has no output, whatever its buffer holds
    if (qb.k[q] > 0 && qb.count[q] > qb.cap[q]) list[atomicAdd(count, 1u)] = q;
}

__global__ __launch_bounds__(MIH_BLOCK) void exact_bounds_kernel(QueryBatch qb, const uint32_t *list,
                                                                 uint32_t nlist, uint32_t *tau_out,
                                                                 uint32_t *cap_out)
{
    uint32_t i = blockIdx.x * MIH_BLOCK + threadIdx.x;
    if (i >= nlist) return;
    uint32_t q = list[i];
    uint32_t kk, D, below, at_D;
    kth_distance(qb, q, kk, D, below, at_D);
    tau_out[i] = kk ? D : qb.bits;
    cap_out[i] = kk ? below + at_D : 0;
}

}  // namespace

namespace mih {

hipError_t find_overflow(const FinalArgs &a, hipStream_t s)
{
    if (a.qb.nq == 0) return hipSuccess;
    hipError_t e = fill_u32(a.overflow_count, 1, 0u, s);
    if (e != hipSuccess) return e;
    find_overflow_kernel<<<(a.qb.nq + MIH_BLOCK - 1) / MIH_BLOCK, MIH_BLOCK, 0, s>>>(
        a.qb, a.overflow_list, a.overflow_count);
    return hipGetLastError();
}

hipError_t finalize_topk(const FinalArgs &a, hipStream_t s)
{
    if (a.qb.nq == 0) return hipSuccess;
    finalize_kernel<<<a.qb.nq, MIH_BLOCK, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t finalize_list(const QueryBatch &qb, const uint32_t *list, uint32_t nlist,
                         const uint64_t *out_ids, const uint64_t *out_dists, hipStream_t s)
{
    if (nlist == 0) return hipSuccess;
    finalize_list_kernel<<<nlist, MIH_BLOCK, 0, s>>>(qb, list, out_ids, out_dists);
    return hipGetLastError();
}

hipError_t finalize_done(const QueryBatch &qb, const uint32_t *list, const uint32_t *count,
                         const uint64_t *out_ids, const uint64_t *out_dists, uint32_t grid,
                         hipStream_t s)
{
    if (grid == 0) return hipSuccess;
    finalize_done_kernel<<<grid, MIH_BLOCK, 0, s>>>(qb, list, count, out_ids, out_dists);
    return hipGetLastError();
}

hipError_t exact_bounds(const QueryBatch &qb, const uint32_t *list, uint32_t nlist,
                        uint32_t *tau_out, uint32_t *cap_out, hipStream_t s)
{
    if (nlist == 0) return hipSuccess;
    exact_bounds_kernel<<<(nlist + MIH_BLOCK - 1) / MIH_BLOCK, MIH_BLOCK, 0, s>>>(qb, list, nlist,
                                                                                 tau_out, cap_out);
    return hipGetLastError();
}

}  // namespace mih
