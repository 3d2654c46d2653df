// Exact top-k of one query from its candidate buffer, by one workgroup
// (device code shared by the top-k kernels and the one-launch search of
// small batches).
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
#pragma once

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

// The LDS of one finalization (the caller's, so that a kernel can share it
// with the LDS of an earlier phase).
struct FinalizeLds {
    uint64_t sel[MIH_K_MAX];
    uint32_t digit_hist[256];
    uint32_t kk, D, below, at_D, prefix, pmask, remaining, count;
};

// One workgroup (any size) finalizes query q into oid[0..k), odist[0..k).
__device__ void finalize_one(const QueryBatch &qb, uint32_t q, uint32_t *oid, uint32_t *odist, FinalizeLds &L)
{
    uint64_t *sel = L.sel;
    uint32_t *digit_hist = L.digit_hist;
    uint32_t &s_kk = L.kk, &s_D = L.D, &s_below = L.below, &s_at_D = L.at_D, &s_prefix = L.prefix,
             &s_pmask = L.pmask, &s_remaining = L.remaining, &s_count = L.count;
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
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
            for (uint32_t i = tid; i < 256; i += nt) digit_hist[i] = 0;
            __syncthreads();
            const uint32_t prefix = s_prefix, pmask = s_pmask;
            for (uint32_t e = tid; e < nbuf; e += nt) {
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

    for (uint32_t e = tid; e < nbuf; e += nt) {
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
    for (uint32_t i = kk + tid; i < P; i += nt) sel[i] = ~0ull;
    __syncthreads();
    block_bitonic_sort(sel, P);   // any workgroup size
    for (uint32_t r = tid; r < k; r += nt) {
        if (r < kk) {
            oid[r] = (uint32_t)sel[r];
            odist[r] = (uint32_t)(sel[r] >> 32);
        } else {
            oid[r] = MIH_SENTINEL;
            odist[r] = MIH_SENTINEL;
        }
    }
}

}  // namespace
