// Exact kNN by linear scan: the distance of every database code to every
// query (the baseline of Section 5; one xor and one popcount per 64 bits,
// Section 6), batched for the GPU.
//
// Work layout.  Each workgroup owns a contiguous range of database codes and
// streams it once: a block of 256*R codes is loaded into registers (coalesced
// rows), then every query of the batch is compared against it, QB queries at
// a time held in scalar registers.  The codes are read from HBM once per call
// whatever the number of queries, so the kernel is bound by the vector ALU
// (xor and bit count).
//
// Keeping only candidates that can still be neighbours.  Per query a bound
// tau is kept in device memory: a code is offered to the query's buffer only
// if its distance is at most tau.  tau starts at the k-th smallest distance
// within a prefix sample of the database (an upper bound on the true k-th
// distance) and is lowered from the histogram of offered distances whenever
// a wave offers something.  The fast path folds the test into the bit count:
// t = d + (2^31 - 1 - tau) has its top bit clear exactly when d <= tau, and
// the minimum over all (code, query) pairs of a wave decides whether any pair
// needs the slow path.
#include "mih_common.h"

namespace {

template <int W, int QH>
__global__ __launch_bounds__(MIH_BLOCK) void sample_bound_kernel(const uint64_t *__restrict__ codes,
                                                                 uint64_t sample, QueryBatch qb)
{
    __shared__ uint32_t h[QH][257];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t nb = qb.bits + 1;
    const uint32_t q0 = blockIdx.x * QH;
    for (uint32_t i = tid; i < QH * 257; i += MIH_BLOCK) (&h[0][0])[i] = 0;
    uint64_t g[QH][W];
#pragma unroll
    for (int j = 0; j < QH; ++j) {
        uint32_t q = q0 + j < qb.nq ? q0 + j : qb.nq - 1;
#pragma unroll
        for (int w = 0; w < W; ++w) g[j][w] = qb.queries[(uint64_t)q * W + w];
    }
    __syncthreads();
    for (uint64_t i = tid; i < sample; i += MIH_BLOCK) {
        uint64_t c[W];
        load_code<W>(codes + i * W, c);
#pragma unroll
        for (int j = 0; j < QH; ++j) atomicAdd(&h[j][hamming<W>(c, g[j])], 1u);
    }
    __syncthreads();
    const uint32_t per = (nb + MIH_WAVE - 1) / MIH_WAVE;
    for (uint32_t j = wave; j < QH; j += MIH_BLOCK / MIH_WAVE) {
        uint32_t q = q0 + j;
        if (q >= qb.nq) break;
        uint32_t k = qb.k[q];
        uint32_t v[5], local = 0;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            uint32_t e = lane * per + i;
            v[i] = (i < (int)per && e < nb) ? h[j][e] : 0u;
            local += v[i];
        }
        uint32_t run = wave_inclusive_sum(local) - local;
        uint32_t first = 0xFFFFFFFFu;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            run += v[i];
            uint32_t e = lane * per + i;
            if (first == 0xFFFFFFFFu && i < (int)per && e < nb && k > 0 && run >= k) first = e;
        }
        uint64_t has = __ballot(first != 0xFFFFFFFFu);
        uint32_t D = qb.bits;
        if (has) D = __shfl(first, (uint32_t)__ffsll((long long)has) - 1, MIH_WAVE);
        if (lane == 0) qb.tau[q] = D;
    }
}

// Bit count of x plus acc in one v_bcnt_u32_b32.  Written out because the
// compiler otherwise regroups the additions and spends a separate add on the
// bound.  acc_s is a wave-uniform value (scalar operand), acc_v a vector one.
__device__ __forceinline__ uint32_t bcnt_acc_s(uint32_t x, uint32_t acc_s)
{
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "s"(acc_s));
    return r;
}

__device__ __forceinline__ uint32_t bcnt_acc_v(uint32_t x, uint32_t acc_v)
{
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc_v));
    return r;
}

// queries and qb.tau hold nbatches * QB rows; rows from qb.nq on are padding
// whose bound test is forced to fail.
template <int W, int QB, int R>
__global__ __launch_bounds__(MIH_BLOCK) void linscan_kernel(const uint64_t *__restrict__ codes,
                                                            const uint64_t *__restrict__ queries,
                                                            uint64_t n, QueryBatch qb,
                                                            uint64_t range_len, uint32_t nbatches)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63;
    const uint64_t begin = (uint64_t)blockIdx.x * range_len;
    const uint64_t end = begin + range_len < n ? begin + range_len : n;
    // different workgroups start at different query batches, so that each
    // query is being compared by few workgroups at a time and its bound
    // tightens before much of the database has been offered to it
    const uint32_t rot = blockIdx.x % nbatches;

    for (uint64_t base = begin; base < end; base += (uint64_t)MIH_BLOCK * R) {
        uint64_t c[R][W];
        bool valid[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            uint64_t idx = base + (uint64_t)r * MIH_BLOCK + tid;
            valid[r] = idx < end;
            uint64_t src = valid[r] ? idx : begin;
#pragma unroll
            for (int w = 0; w < W; ++w) c[r][w] = codes[src * W + w];
        }
        uint32_t b = rot;
        // the bounds of a batch come in one vector load (lane j holds query
        // q0 + j mod QB) issued one batch ahead
        const uint32_t lq = lane % (uint32_t)QB;
        uint32_t tv = load_relaxed(qb.tau + b * QB + lq);
        for (uint32_t bi = 0; bi < nbatches; ++bi) {
            const uint32_t q0 = b * QB;
            const uint32_t bn = b + 1 == nbatches ? 0u : b + 1;
            const uint32_t tv_next = load_relaxed(qb.tau + bn * QB + lq);
            const uint64_t *qp = queries + (uint64_t)q0 * W;
            uint64_t g[QB][W];
            uint32_t bias[QB];   // 2^31 - 1 - tau, or 2^31 for padding rows
#pragma unroll
            for (int j = 0; j < QB; ++j) {
#pragma unroll
                for (int w = 0; w < W; ++w) g[j][w] = qp[j * W + w];
                bias[j] = q0 + j < qb.nq ? 0x7FFFFFFFu - __builtin_amdgcn_readlane(tv, j) : 0x80000000u;
            }
            uint32_t mn = 0xFFFFFFFFu;
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int j = 0; j < QB; ++j) {
                    const uint64_t x0 = c[r][0] ^ g[j][0];
                    uint32_t t = bcnt_acc_s((uint32_t)x0, bias[j]);
                    t = bcnt_acc_v((uint32_t)(x0 >> 32), t);
#pragma unroll
                    for (int w = 1; w < W; ++w) {
                        const uint64_t x = c[r][w] ^ g[j][w];
                        t = bcnt_acc_v((uint32_t)x, t);
                        t = bcnt_acc_v((uint32_t)(x >> 32), t);
                    }
                    mn = mn < t ? mn : t;
                }
            if (__ballot(mn < 0x80000000u)) {
                // slow path: some pair of this wave is within its query's bound
#pragma unroll 1
                for (int j = 0; j < QB; ++j) {
                    const uint32_t q = q0 + j;
                    if (q >= qb.nq) break;
                    const uint32_t tau_j = 0x7FFFFFFFu - bias[j];
                    uint32_t d[R];
                    bool any = false;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        d[r] = hamming<W>(c[r], g[j]);
                        any |= valid[r] && d[r] <= tau_j;
                    }
                    // most queries of a batch that reached the slow path have no hit
                    if (!__ballot(any)) continue;
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        append_candidates(qb, q, valid[r] && d[r] <= tau_j, d[r],
                                          (uint32_t)(base + (uint64_t)r * MIH_BLOCK + tid));
                    tighten_tau(qb, q, tau_j);
                }
            }
            tv = tv_next;
            b = bn;
        }
    }
}

template <int W, int QB, int R>
hipError_t launch_scan(const mih::LinscanArgs &a, uint32_t num_cus, hipStream_t s)
{
    const uint64_t per_block = (uint64_t)MIH_BLOCK * R;
    const uint64_t blocks_needed = (a.n + per_block - 1) / per_block;
    uint64_t grid = (uint64_t)num_cus * 8;
    if (grid > blocks_needed) grid = blocks_needed;
    if (grid < 1) grid = 1;
    // range per workgroup, a whole number of register blocks
    uint64_t range = (blocks_needed + grid - 1) / grid * per_block;
    grid = (a.n + range - 1) / range;
    if (grid < 1) grid = 1;
    const uint32_t nbatches = (a.qb.nq + QB - 1) / QB;
    linscan_kernel<W, QB, R><<<(uint32_t)grid, MIH_BLOCK, 0, s>>>(a.codes, a.queries_padded, a.n,
                                                                  a.qb, range, nbatches);
    return hipGetLastError();
}

template <int W>
hipError_t launch_sample(const mih::LinscanArgs &a, uint64_t sample, hipStream_t s)
{
    constexpr int QH = 16;
    const uint32_t grid = (a.qb.nq + QH - 1) / QH;
    sample_bound_kernel<W, QH><<<grid, MIH_BLOCK, 0, s>>>(a.codes, sample, a.qb);
    return hipGetLastError();
}

}  // namespace

namespace mih {

hipError_t linscan_init(const LinscanArgs &a, uint64_t sample, const uint32_t *tau0, hipStream_t s)
{
    if (a.qb.nq == 0) return hipSuccess;
    hipError_t e = fill_u32(a.qb.count, a.qb.nq, 0u, s);
    if (e == hipSuccess) e = fill_u32(a.qb.hist, (uint64_t)a.qb.nq * (a.qb.bits + 1), 0u, s);
    if (e != hipSuccess) return e;
    if (tau0) return hipMemcpyAsync(a.qb.tau, tau0, sizeof(uint32_t) * a.qb.nq,
                                    hipMemcpyDeviceToDevice, s);
    if (sample == 0 || a.n == 0) return fill_u32(a.qb.tau, a.qb.nq, a.qb.bits, s);
    switch (a.W) {
    case 1: return launch_sample<1>(a, sample, s);
    case 2: return launch_sample<2>(a, sample, s);
    case 3: return launch_sample<3>(a, sample, s);
    case 4: return launch_sample<4>(a, sample, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t linscan_run(const LinscanArgs &a, uint32_t num_cus, hipStream_t s)
{
    if (a.qb.nq == 0 || a.n == 0) return hipSuccess;
    switch (a.W) {
    case 1: return launch_scan<1, 16, 8>(a, num_cus, s);
    case 2: return launch_scan<2, 8, 8>(a, num_cus, s);
    case 3: return launch_scan<3, 8, 4>(a, num_cus, s);
    case 4: return launch_scan<4, 4, 4>(a, num_cus, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mih
