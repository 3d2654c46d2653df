// Exact top-k kernels: the finished queries of a batch or of a device
// round, overflow detection and the exact bounds of re-runs.  The top-k of
// one query (k-th distance, radix select on the id, LDS sort) is in
// topk_dev.h.
#include "topk_dev.h"

namespace {

__global__ __launch_bounds__(MIH_BLOCK) void finalize_kernel(mih::FinalArgs a)
{
    __shared__ FinalizeLds L;
    const uint32_t q = blockIdx.x;
    const uint64_t off = a.row_off[q];
    finalize_one(a.qb, q, a.out_ids + off, a.out_dists + off, L);
}

// Queries of a list, each with its own output row (device addresses).
__global__ __launch_bounds__(MIH_BLOCK) void finalize_list_kernel(QueryBatch qb, const uint32_t *list,
                                                                  const uint64_t *out_ids,
                                                                  const uint64_t *out_dists)
{
    __shared__ FinalizeLds L;
    const uint32_t q = list[blockIdx.x];
    finalize_one(qb, q, reinterpret_cast<uint32_t *>(out_ids[q]),
                 reinterpret_cast<uint32_t *>(out_dists[q]), L);
}

// The queries a round finished (count read on the device, so that the launch
// can sit in a captured graph): each workgroup takes every gridDim-th one.
// r-neighbour queries (k = 0xFFFFFFFF) have no top-k rows and are skipped.
__global__ __launch_bounds__(MIH_BLOCK) void finalize_done_kernel(QueryBatch qb, const uint32_t *list,
                                                                  const uint32_t *count,
                                                                  const uint64_t *out_ids,
                                                                  const uint64_t *out_dists)
{
    __shared__ FinalizeLds L;
    const uint32_t n = *count;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const uint32_t q = list[i];
        if (qb.k[q] == 0xFFFFFFFFu) continue;
        finalize_one(qb, q, reinterpret_cast<uint32_t *>(out_ids[q]),
                     reinterpret_cast<uint32_t *>(out_dists[q]), L);
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
