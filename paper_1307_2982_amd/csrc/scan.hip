// Device-wide fills and scans over uint32 arrays of up to 2^33 elements:
// the exclusive prefix sum used by the radix sort and the suffix minimum that
// turns bucket starts into direct-address offsets.  Reduce-then-scan in three
// launches: per-tile totals, a single-workgroup scan of the totals, then each
// tile rescanned with its carried-in value.
#include "mih_common.h"

namespace {

constexpr uint32_t kItems = 16;
constexpr uint32_t kTile = MIH_BLOCK * kItems;   // 4096 elements per workgroup

struct SumOp {
    static __device__ __forceinline__ uint32_t identity() { return 0u; }
    static __device__ __forceinline__ uint32_t apply(uint32_t a, uint32_t b) { return a + b; }
};
struct MinOp {
    static __device__ __forceinline__ uint32_t identity() { return 0xFFFFFFFFu; }
    static __device__ __forceinline__ uint32_t apply(uint32_t a, uint32_t b) { return a < b ? a : b; }
};

template <class Op>
__device__ __forceinline__ uint32_t wave_inclusive(uint32_t x)
{
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int off = 1; off < MIH_WAVE; off <<= 1) {
        uint32_t y = __shfl_up(x, off, MIH_WAVE);
        if (lane >= (uint32_t)off) x = Op::apply(x, y);
    }
    return x;
}

// Exclusive scan of one value per thread over a 256-thread block; also
// returns the block total.
template <class Op>
__device__ __forceinline__ uint32_t block_exclusive(uint32_t x, uint32_t *lds4, uint32_t &total)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t incl = wave_inclusive<Op>(x);
    if (lane == 63) lds4[wave] = incl;
    __syncthreads();
    uint32_t before = Op::identity();
    for (uint32_t w = 0; w < wave; ++w) before = Op::apply(before, lds4[w]);
    total = Op::apply(Op::apply(Op::apply(lds4[0], lds4[1]), lds4[2]), lds4[3]);
    uint32_t excl_in_wave = __shfl_up(incl, 1, MIH_WAVE);
    if (lane == 0) excl_in_wave = Op::identity();
    __syncthreads();
    return Op::apply(before, excl_in_wave);
}

template <bool Rev>
__device__ __forceinline__ uint64_t phys(uint64_t p, uint64_t n) { return Rev ? n - 1 - p : p; }

template <class Op, bool Rev>
__global__ __launch_bounds__(MIH_BLOCK) void tile_reduce(const uint32_t *__restrict__ in, uint64_t n,
                                                         uint32_t *__restrict__ partial)
{
    __shared__ uint32_t lds4[4];
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    uint32_t acc = Op::identity();
    for (uint32_t j = 0; j < kItems; ++j) {
        uint64_t p = base + j * MIH_BLOCK + threadIdx.x;
        if (p < n) acc = Op::apply(acc, in[phys<Rev>(p, n)]);
    }
    uint32_t total;
    block_exclusive<Op>(acc, lds4, total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// One workgroup scans the per-tile totals in place (exclusive).
template <class Op>
__global__ __launch_bounds__(1024) void scan_partials(uint32_t *partial, uint64_t nb)
{
    __shared__ uint32_t lds[32];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t per = (nb + 1023) / 1024;
    const uint64_t lo = tid * per, hi = lo + per < nb ? lo + per : nb;
    uint32_t acc = Op::identity();
    for (uint64_t i = lo; i < hi; ++i) acc = Op::apply(acc, partial[i]);
    uint32_t incl = wave_inclusive<Op>(acc);
    if (lane == 63) lds[wave] = incl;
    __syncthreads();
    uint32_t before = Op::identity();
    for (uint32_t w = 0; w < wave; ++w) before = Op::apply(before, lds[w]);
    uint32_t excl = __shfl_up(incl, 1, MIH_WAVE);
    if (lane == 0) excl = Op::identity();
    uint32_t run = Op::apply(before, excl);
    for (uint64_t i = lo; i < hi; ++i) {
        uint32_t v = partial[i];
        partial[i] = run;
        run = Op::apply(run, v);
    }
}

// LDS position of tile element p: one pad word after every kItems words, so
// that threads reading kItems consecutive elements hit distinct banks.
__device__ __forceinline__ uint32_t pad(uint32_t p) { return p + p / kItems; }

template <class Op, bool Rev, bool Inclusive>
__global__ __launch_bounds__(MIH_BLOCK) void tile_scan(const uint32_t *__restrict__ in, uint32_t *out,
                                                       uint64_t n, const uint32_t *__restrict__ partial)
{
    __shared__ uint32_t tile[kTile + kTile / kItems];
    __shared__ uint32_t lds4[4];
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    const uint32_t tid = threadIdx.x;
    for (uint32_t j = 0; j < kItems; ++j) {
        uint64_t p = base + j * MIH_BLOCK + tid;
        tile[pad(j * MIH_BLOCK + tid)] = (p < n) ? in[phys<Rev>(p, n)] : Op::identity();
    }
    __syncthreads();
    uint32_t v[kItems];
    uint32_t acc = Op::identity();
#pragma unroll
    for (uint32_t j = 0; j < kItems; ++j) {
        v[j] = tile[pad(tid * kItems + j)];
        acc = Op::apply(acc, v[j]);
    }
    uint32_t total;
    uint32_t run = Op::apply(partial[blockIdx.x], block_exclusive<Op>(acc, lds4, total));
#pragma unroll
    for (uint32_t j = 0; j < kItems; ++j) {
        uint32_t next = Op::apply(run, v[j]);
        tile[pad(tid * kItems + j)] = Inclusive ? next : run;
        run = next;
    }
    __syncthreads();
    for (uint32_t j = 0; j < kItems; ++j) {
        uint64_t p = base + j * MIH_BLOCK + tid;
        if (p < n) out[phys<Rev>(p, n)] = tile[pad(j * MIH_BLOCK + tid)];
    }
}

template <class Op, bool Rev, bool Inclusive>
hipError_t scan_impl(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *tmp, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const uint64_t nb = (n + kTile - 1) / kTile;
    if (nb > 0x7FFFFFFFull) return hipErrorInvalidValue;
    tile_reduce<Op, Rev><<<(uint32_t)nb, MIH_BLOCK, 0, s>>>(in, n, tmp);
    scan_partials<Op><<<1, 1024, 0, s>>>(tmp, nb);
    tile_scan<Op, Rev, Inclusive><<<(uint32_t)nb, MIH_BLOCK, 0, s>>>(in, out, n, tmp);
    return hipGetLastError();
}

template <class T>
__global__ __launch_bounds__(MIH_BLOCK) void fill_kernel(T *p, uint64_t n, T value)
{
    uint64_t i = (uint64_t)blockIdx.x * MIH_BLOCK + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * MIH_BLOCK;
    for (; i < n; i += stride) p[i] = value;
}

template <class T>
hipError_t fill_impl(T *p, uint64_t n, T value, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + MIH_BLOCK - 1) / MIH_BLOCK;
    if (blocks > 65536ull * 8) blocks = 65536ull * 8;
    fill_kernel<T><<<(uint32_t)blocks, MIH_BLOCK, 0, s>>>(p, n, value);
    return hipGetLastError();
}

__global__ __launch_bounds__(MIH_BLOCK) void gather_rows_kernel(const uint64_t *__restrict__ rows,
                                                                const uint32_t *__restrict__ list,
                                                                uint32_t nlist, uint32_t W,
                                                                uint64_t *__restrict__ dst)
{
    uint64_t i = (uint64_t)blockIdx.x * MIH_BLOCK + threadIdx.x;
    if (i >= (uint64_t)nlist * W) return;
    uint64_t r = i / W, w = i % W;
    dst[i] = rows[(uint64_t)list[r] * W + w];
}

}  // namespace

namespace mih {

hipError_t gather_rows(const uint64_t *rows, const uint32_t *list, uint32_t nlist, uint32_t W,
                       uint64_t *dst, hipStream_t s)
{
    if (nlist == 0) return hipSuccess;
    uint64_t total = (uint64_t)nlist * W;
    gather_rows_kernel<<<(uint32_t)((total + MIH_BLOCK - 1) / MIH_BLOCK), MIH_BLOCK, 0, s>>>(
        rows, list, nlist, W, dst);
    return hipGetLastError();
}

hipError_t fill_u32(uint32_t *p, uint64_t n, uint32_t value, hipStream_t s)
{
    return fill_impl<uint32_t>(p, n, value, s);
}

hipError_t fill_u64(uint64_t *p, uint64_t n, uint64_t value, hipStream_t s)
{
    return fill_impl<uint64_t>(p, n, value, s);
}

uint64_t scan_tmp_words(uint64_t n) { return (n + kTile - 1) / kTile + 64; }

hipError_t exclusive_sum_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *tmp,
                             hipStream_t s)
{
    return scan_impl<SumOp, false, false>(in, out, n, tmp, s);
}

hipError_t suffix_min_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *tmp,
                          hipStream_t s)
{
    return scan_impl<MinOp, true, true>(in, out, n, tmp, s);
}

}  // namespace mih
