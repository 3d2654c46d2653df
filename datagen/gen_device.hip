// Seeded synthetic codes generated on the device, bit-identical to the host
// generators in gen.c (same SplitMix64 counters, same integer recipe).
//
// This module produces inputs only and holds none of the search method's
// arithmetic.  It exists because the 1e9-code clustered workload (128-D
// points and 256 hyperplanes: 3.3e13 multiply-adds) is far too slow to
// produce on the host.  The clustered codes are made in three passes per
// chunk of points: dg_dev_points writes the points x = 10 mu + 3 eps as fp64,
// the caller multiplies them by the hyperplanes with a plain fp64 matrix
// product, and dg_dev_pack turns the signs into code words.  Every product
// and partial sum is an integer below 2^53 in magnitude (|w| <= 6*65536,
// |x| <= 13*6*65536, 128 terms), so the fp64 arithmetic is exact in any
// summation order and equals the host's int64 result.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define DG_GAMMA 0x9E3779B97F4A7C15ULL
#define DG_DIM 128
#define DG_PER_POINT (1 + 3 * DG_DIM)

__device__ __forceinline__ uint64_t dg_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t dg_out(uint64_t seed, uint64_t c)
{
    return dg_mix64(seed + (c + 1) * DG_GAMMA);
}

__device__ __forceinline__ int64_t dg_gauss(uint64_t seed, uint64_t c)
{
    int64_t s = 0;
    for (int w = 0; w < 3; ++w) {
        uint64_t u = dg_out(seed, c + (uint64_t)w);
        s += (int64_t)(u & 0xFFFF) + (int64_t)((u >> 16) & 0xFFFF) + (int64_t)((u >> 32) & 0xFFFF) +
             (int64_t)(u >> 48);
    }
    return s - 6 * 65536;
}

__global__ void dg_uniform_kernel(uint64_t *out, uint64_t n, uint32_t words, uint64_t seed,
                                  uint64_t first_row)
{
    const uint64_t total = n * words;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = dg_out(seed, first_row * words + i);
}

// x[p][d] for points first_row + p, p < n; mu is [1000][128] (integers).
__global__ void dg_points_kernel(double *x, uint64_t n, uint64_t seed, uint64_t first_row,
                                 const int64_t *mu)
{
    const uint64_t total = n * DG_DIM;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t p = i / DG_DIM, d = i % DG_DIM;
        const uint64_t base = (first_row + p) * (uint64_t)DG_PER_POINT;
        const uint64_t comp = __umul64hi(dg_out(seed, base), 1000ull);
        x[i] = (double)(10 * mu[comp * DG_DIM + d] + 3 * dg_gauss(seed, base + 1 + 3 * d));
    }
}

// out[p][w] bit b = [dots[p][64 w + b] > 0] for p < n.
__global__ void dg_pack_kernel(uint64_t *out, const double *dots, uint64_t n, uint32_t bits)
{
    const uint32_t words = bits / 64;
    const uint64_t total = n * words;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t p = i / words, w = i % words;
        const double *row = dots + p * bits + w * 64;
        uint64_t word = 0;
        for (uint32_t b = 0; b < 64; ++b)
            if (row[b] > 0.0) word |= 1ull << b;
        out[i] = word;
    }
}

static uint32_t dg_blocks(uint64_t work)
{
    uint64_t b = (work + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (uint32_t)b;
}

extern "C" {

// Device buffer out [n][words] receives rows [first_row, first_row + n) of
// the uniform stream.  Returns a hipError_t value (0 on success).
int dg_dev_uniform(uint64_t *out, uint64_t n, uint32_t words, uint64_t seed, uint64_t first_row,
                   void *stream)
{
    if (n == 0) return 0;
    dg_uniform_kernel<<<dg_blocks(n * words), 256, 0, (hipStream_t)stream>>>(out, n, words, seed,
                                                                            first_row);
    return (int)hipGetLastError();
}

// Device x [n][128] (fp64) receives the points of rows [first_row, first_row+n)
// of the clustered stream; mu is the device copy of the mixture means.
int dg_dev_points(double *x, uint64_t n, uint64_t seed, uint64_t first_row, const int64_t *mu,
                  void *stream)
{
    if (n == 0) return 0;
    dg_points_kernel<<<dg_blocks(n * DG_DIM), 256, 0, (hipStream_t)stream>>>(x, n, seed, first_row, mu);
    return (int)hipGetLastError();
}

// Device out [n][bits/64] receives the sign bits of dots [n][bits].
int dg_dev_pack(uint64_t *out, const double *dots, uint64_t n, uint32_t bits, void *stream)
{
    if (n == 0) return 0;
    if (bits == 0 || bits % 64 || bits > 256) return (int)hipErrorInvalidValue;
    dg_pack_kernel<<<dg_blocks(n * (bits / 64)), 256, 0, (hipStream_t)stream>>>(out, dots, n, bits);
    return (int)hipGetLastError();
}

}  // extern "C"
