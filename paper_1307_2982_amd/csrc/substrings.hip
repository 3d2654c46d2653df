// Substring optimisation (Section 5.5): assign the code bits to substrings
// so that bits within one substring are as little correlated as possible.
//
// The correlations come from co-occurrence counts over a sample of codes,
// counts[i][j] = number of codes with bits i and j both set, which is the
// Gram matrix X^T X of the 0/1 sample matrix X (samples x bits).  That is a
// dense integer contraction, so it runs on the matrix cores: 8-bit operands
// (0 or 1) with 32-bit accumulation are exact.  The greedy assignment itself
// works on a bits x bits table on the host.
#include <algorithm>
#include <cmath>
#include <vector>

#include "mih_common.h"

namespace {

typedef int v16i __attribute__((ext_vector_type(16)));

constexpr uint32_t kSlice = 1u << 16;   // samples per wave

// One wave per (32 x 32 tile of the counts, slice of samples).  Each
// v_mfma_i32_32x32x16_i8 adds 16 samples: lane l holds, for row l % 32 of
// the tile, the bits of samples 8 (l / 32) .. 8 (l / 32) + 7 as 8 bytes of
// A (bits of the row's code bit) and of B (bits of the column's code bit).
template <int W>
__global__ __launch_bounds__(64) void cooc_kernel(const uint64_t *__restrict__ codes, uint64_t n,
                                                  uint32_t bits, uint32_t *counts)
{
    const uint32_t lane = threadIdx.x;
    const uint32_t tiles = bits / 32;
    const uint32_t ti = blockIdx.x / tiles, tj = blockIdx.x % tiles;
    const uint64_t n0 = (uint64_t)blockIdx.y * kSlice;
    const uint64_t n1 = n0 + kSlice < n ? n0 + kSlice : n;
    const uint32_t r = lane & 31, half = lane >> 5;
    const uint32_t bi = ti * 32 + r, bj = tj * 32 + r;
    v16i acc = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t base = n0; base < n1; base += 16) {
        uint64_t a = 0, b = 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint64_t sidx = base + half * 8 + e;
            if (sidx < n1) {
                const uint64_t *c = codes + sidx * W;
                a |= ((c[bi >> 6] >> (bi & 63)) & 1ull) << (8 * e);
                b |= ((c[bj >> 6] >> (bj & 63)) & 1ull) << (8 * e);
            }
        }
        acc = __builtin_amdgcn_mfma_i32_32x32x16_i8((long)a, (long)b, acc, 0, 0, 0);
    }
    // accumulator register k of lane l: row 8 (k / 4) + 4 (l / 32) + k % 4, column l % 32
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t i = ti * 32 + 8 * (k / 4) + 4 * half + (k % 4);
        const uint32_t j = tj * 32 + r;
        if (acc[k]) atomicAdd(&counts[(uint64_t)i * bits + j], (uint32_t)acc[k]);
    }
}

}  // namespace

extern "C" {

mih_status mih_bit_cooccurrence(const uint64_t *codes, uint64_t n, uint32_t bits, void *stream,
                                uint32_t *counts)
{
    if (!counts || bits == 0 || bits % 64 != 0 || bits > 256) return MIH_ERR_INVALID;
    if (n && (!codes || ((uintptr_t)codes & 7) != 0)) return MIH_ERR_INVALID;
    if (n > 0x7FFFFFFFull) return MIH_ERR_UNSUPPORTED;   // 32-bit counts
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint32_t> host((size_t)bits * bits, 0);
    uint32_t *dev = nullptr;
    if (hipMalloc((void **)&dev, (size_t)bits * bits * 4) != hipSuccess) {
        (void)hipGetLastError();
        return MIH_ERR_NOMEM;
    }
    hipError_t e = mih::fill_u32(dev, (uint64_t)bits * bits, 0u, s);
    if (e == hipSuccess && n) {
        const uint32_t tiles = bits / 32;
        const dim3 grid(tiles * tiles, (uint32_t)((n + kSlice - 1) / kSlice));
        switch (bits / 64) {
        case 1: cooc_kernel<1><<<grid, 64, 0, s>>>(codes, n, bits, dev); break;
        case 2: cooc_kernel<2><<<grid, 64, 0, s>>>(codes, n, bits, dev); break;
        case 3: cooc_kernel<3><<<grid, 64, 0, s>>>(codes, n, bits, dev); break;
        case 4: cooc_kernel<4><<<grid, 64, 0, s>>>(codes, n, bits, dev); break;
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(counts, dev, (size_t)bits * bits * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return MIH_ERR_DEVICE;
    }
    return MIH_OK;
}

mih_status mih_greedy_bit_order(const uint32_t *counts, uint64_t n, uint32_t bits, uint32_t m,
                                uint32_t first_bit, uint16_t *bit_order)
{
    if (!counts || !bit_order || bits == 0 || bits > 256 || m < 1 || m > bits || first_bit >= bits)
        return MIH_ERR_INVALID;
    // |Pearson correlation| of bits u and v over the sample; a constant bit
    // is uncorrelated with every bit
    std::vector<double> corr((size_t)bits * bits, 0.0);
    for (uint32_t u = 0; u < bits; ++u)
        for (uint32_t v = 0; v < bits; ++v) {
            const int64_t cu = counts[(size_t)u * bits + u], cv = counts[(size_t)v * bits + v];
            const int64_t cuv = counts[(size_t)u * bits + v];
            const int64_t N = (int64_t)n;
            const int64_t vu = cu * (N - cu), vv = cv * (N - cv);
            if (vu == 0 || vv == 0) continue;
            const int64_t num = N * cuv - cu * cv;
            const double c = (double)num / std::sqrt((double)vu * (double)vv);
            corr[(size_t)u * bits + v] = c < 0 ? -c : c;
        }
    std::vector<uint32_t> len(m), start(m);
    for (uint32_t j = 0, st = 0; j < m; ++j) {
        len[j] = bits / m + (j < bits % m ? 1u : 0u);
        start[j] = st;
        st += len[j];
    }
    std::vector<std::vector<uint32_t>> sub(m);
    std::vector<uint8_t> used(bits, 0);
    // a seed bit for the first substring; each next substring starts with
    // the unused bit most correlated with the previous substring's bit
    sub[0].push_back(first_bit);
    used[first_bit] = 1;
    for (uint32_t j = 1; j < m; ++j) {
        const uint32_t prev = sub[j - 1][0];
        uint32_t best = bits;
        for (uint32_t u = 0; u < bits; ++u)
            if (!used[u] && (best == bits || corr[(size_t)prev * bits + u] > corr[(size_t)prev * bits + best]))
                best = u;
        sub[j].push_back(best);
        used[best] = 1;
    }
    // then, substring by substring in turn, the unused bit whose largest
    // correlation with the substring's bits is smallest
    for (uint32_t assigned = m; assigned < bits;) {
        for (uint32_t j = 0; j < m && assigned < bits; ++j) {
            if (sub[j].size() >= len[j]) continue;
            uint32_t best = bits;
            double best_v = 0.0;
            for (uint32_t u = 0; u < bits; ++u) {
                if (used[u]) continue;
                double mx = 0.0;
                for (uint32_t v : sub[j]) mx = std::max(mx, corr[(size_t)u * bits + v]);
                if (best == bits || mx < best_v) { best = u; best_v = mx; }
            }
            sub[j].push_back(best);
            used[best] = 1;
            ++assigned;
        }
    }
    for (uint32_t j = 0; j < m; ++j)
        for (uint32_t k = 0; k < len[j]; ++k) bit_order[start[j] + k] = (uint16_t)sub[j][k];
    return MIH_OK;
}

}  // extern "C"
