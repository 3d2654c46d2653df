// Measurement helper: the rate at which the device serves independent random
// reads of 64-byte lines, the kind of read that dominates the multi-index
// search (each probed bucket entry and each candidate code outside a run is
// such a read).  A bench reports the search kernel's fetched lines per
// second against this rate.
#include "mih_common.h"

namespace {

// SplitMix64 finaliser (Steele, Lea, Flood 2014), as an address hash.
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Each lane reads `per_lane` words, DEPTH at a time with all DEPTH loads in
// flight together, each from its own pseudo-random line of the array.
template <int DEPTH>
__global__ __launch_bounds__(MIH_BLOCK) void random_lines_kernel(const uint64_t *__restrict__ a, uint64_t lines,
                                                                 uint64_t per_lane, uint64_t *sink)
{
    const uint64_t tid = (uint64_t)blockIdx.x * MIH_BLOCK + threadIdx.x;
    uint64_t acc = 0;
    for (uint64_t i = 0; i < per_lane; i += DEPTH) {
        uint64_t v[DEPTH];
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) {
            const uint64_t h = mix64((tid << 24) + i + d);
            v[d] = a[(h % lines) * 8 + (h >> 61)];
        }
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) acc ^= v[d];
    }
    // keep the loads: one add per wave into the sink
    for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off, MIH_WAVE);
    if ((threadIdx.x & 63) == 0) atomicAdd(reinterpret_cast<unsigned long long *>(sink), (unsigned long long)acc);
}

}  // namespace

extern "C" mih_status mih_random_read_rate(const uint64_t *array, uint64_t words, uint64_t reads, uint32_t depth,
                                           uint64_t *sink, void *stream, double *ms)
{
    if (!array || !sink || !ms || words < 8 || reads == 0) return MIH_ERR_INVALID;
    if (depth != 1 && depth != 4 && depth != 8 && depth != 16) return MIH_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    const uint64_t threads = (uint64_t)cus * 8 * MIH_BLOCK;
    uint64_t per_lane = (reads + threads - 1) / threads;
    per_lane = (per_lane + depth - 1) / depth * depth;
    const uint64_t lines = words / 8;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipGetLastError();
        return MIH_ERR_DEVICE;
    }
    hipError_t e = hipEventRecord(e0, s);
    const dim3 grid((uint32_t)(threads / MIH_BLOCK)), block(MIH_BLOCK);
    if (e == hipSuccess) {
        switch (depth) {
        case 1: random_lines_kernel<1><<<grid, block, 0, s>>>(array, lines, per_lane, sink); break;
        case 4: random_lines_kernel<4><<<grid, block, 0, s>>>(array, lines, per_lane, sink); break;
        case 8: random_lines_kernel<8><<<grid, block, 0, s>>>(array, lines, per_lane, sink); break;
        default: random_lines_kernel<16><<<grid, block, 0, s>>>(array, lines, per_lane, sink); break;
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return MIH_ERR_DEVICE;
    }
    *ms = t;
    return MIH_OK;
}
