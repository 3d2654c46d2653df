// Device code of one search step (Algorithm 3), shared by the round
// kernels and the one-launch search of small batches: mask enumeration,
// bucket lookups in every table mode, and the candidate walk with
// first-encounter de-duplication.
#pragma once

#include "mih_common.h"
#include "mih_query.h"

namespace {

// J: masks per lane per iteration (a tuning knob; 64 J buckets are staged
// per wave and iteration).
constexpr uint32_t kWaves = MIH_BLOCK / MIH_WAVE;
// Candidates per lane and pass of the candidate walk: more loads in flight
// per wave, against the registers that keep them (64-bit codes: 2 keeps the
// kernel at six waves per SIMD).
template <int W>
constexpr int walk_depth() { return W == 1 ? 2 : 4; }

__device__ __forceinline__ uint32_t binom_calc(uint32_t n, uint32_t r)
{
    if (r > n) return 0;
    uint64_t c = 1;
    for (uint32_t i = 1; i <= r; ++i) c = c * (n - r + i) / i;
    return (uint32_t)c;
}

// Colex unranking: the mask with `rho` set bits among s whose rank in
// increasing numeric order is `rank` (combinatorial number system).
__device__ __forceinline__ uint32_t unrank_mask(uint32_t rank, uint32_t rho, uint32_t s,
                                                const uint32_t (*binom)[MIH_BINOM_N])
{
    uint32_t mask = 0;
    int c = (int)s - 1;
    for (int i = (int)rho; i >= 1; --i) {
        while (c >= i && binom[c][i] > rank) --c;
        rank -= binom[c][i];
        mask |= 1u << c;
        --c;
    }
    return mask;
}

// Next larger integer with the same number of set bits (Gosper).
__device__ __forceinline__ uint32_t next_mask(uint32_t x)
{
    uint64_t v = x;
    uint64_t c = v & (~v + 1);
    uint64_t r = v + c;
    return (uint32_t)((((r ^ v) >> 2) >> __builtin_ctzll(c)) | r);
}

template <int W>
__device__ __forceinline__ uint64_t u64_uniform(uint64_t x)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Round tail: each wave (round kernel) or workgroup (sweep kernels) that
// took work records when it ran out of it, as the largest end time and the
// largest complement of an end time (so that zero-filled slots start both
// maxima), in the constant-rate wall clock, in the slot pair of its
// workgroup.  The advance kernel's first wave adds each launch's spread
// (last end minus first end over the pairs) to a running sum and clears the
// pairs for the next round.
__device__ __forceinline__ void record_end(unsigned long long *pairs)
{
    unsigned long long *slot = pairs + 2 * (blockIdx.x % mih::kTailPairs);
    const unsigned long long now = (unsigned long long)__builtin_amdgcn_s_memrealtime();
    atomicMax(slot, ~now);
    atomicMax(slot + 1, now);
}

// Called by one whole wave.
__device__ __forceinline__ void fold_tails(unsigned long long *stats)
{
    static_assert(mih::kTailPairs == MIH_WAVE, "one pair per lane");
    const uint32_t lane = lane_id();
    unsigned long long add = 0;
    for (uint32_t k = mih::kStatRoundEnd; k <= mih::kStatSweepEnd; k += 2 * mih::kTailPairs) {
        const unsigned long long first_c = stats[k + 2 * lane], last = stats[k + 2 * lane + 1];
        unsigned long long mx = last, mc = last ? first_c : 0ull;   // max end; max complement = min end
#pragma unroll
        for (int sh = 1; sh < MIH_WAVE; sh <<= 1) {
            const unsigned long long o1 = (unsigned long long)__shfl_xor((long long)mx, sh, MIH_WAVE);
            const unsigned long long o2 = (unsigned long long)__shfl_xor((long long)mc, sh, MIH_WAVE);
            mx = o1 > mx ? o1 : mx;
            mc = o2 > mc ? o2 : mc;
        }
        if (mx) add += mx - ~mc;
        stats[k + 2 * lane] = 0;
        stats[k + 2 * lane + 1] = 0;
    }
    if (lane == 0) stats[mih::kStatTail] += add;
}

struct WaveStats {
    uint64_t probes, candidates;
};

// Key of the code at table position pos (INLINE codes).  With contiguous
// substrings only the one or two words that hold bits [start, start + len)
// are read.
template <int W>
__device__ __forceinline__ uint32_t entry_key(const TableDev &T, uint64_t pos)
{
    const uint64_t *c = T.codes + pos * W;
    if (T.permuted) {
        uint64_t g[W];
#pragma unroll
        for (int w = 0; w < W; ++w) g[w] = c[w];
        return table_key<W>(g, T);
    }
    const uint32_t w = T.start >> 6, o = T.start & 63;
    uint64_t v = c[w] >> o;
    if (o + T.len > 64) v |= c[w + 1] << (64 - o);
    return (uint32_t)(v & ((T.len >= 32) ? 0xFFFFFFFFull : ((1ull << T.len) - 1)));
}

// First position in [p, n) whose substring value is at least `key`, given
// that the values from p on are sorted and that one of them is at least key
// or the range ends at n: doubling steps, then a binary search.
template <int W>
__device__ __forceinline__ uint32_t gallop_at_least(const TableDev &T, uint64_t n, uint64_t key,
                                                    uint32_t p)
{
    uint64_t lo = p, step = 1;
    while (lo + step <= n && entry_key<W>(T, lo + step - 1) < key) {
        lo += step;
        step <<= 1;
    }
    uint64_t hi = lo + step < n ? lo + step : n;   // the answer lies in [lo, hi]
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (entry_key<W>(T, mid) < key) lo = mid + 1; else hi = mid;
    }
    return (uint32_t)lo;
}

// GROUPED tables: the bucket `key`, known to be non-empty, inside the run of
// codes sorted by substring value, starting the search at `p`, a position
// no later than the bucket's first code.  Returns its first position and size.  The common case
// (a few codes per group) is settled by one window of four entries read
// together; longer runs fall back to doubling steps and a binary search.
// Positions at or past n compare as larger than every value.
template <int W>
__device__ __forceinline__ void group_scan(const TableDev &T, uint64_t n, uint32_t key, uint32_t p,
                                           uint32_t &lo, uint32_t &cnt)
{
    uint32_t lt = 0, eq = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t pos = (uint64_t)p + i;
        const uint64_t v = pos < n ? (uint64_t)entry_key<W>(T, pos) : (1ull << 32);
        lt += v < key ? 1u : 0u;
        eq += v == key ? 1u : 0u;
    }
    if (lt + eq < 4) {           // the window ends inside the bucket's successor
        lo = p + lt;
        cnt = eq;
        return;
    }
    lo = lt < 4 ? p + lt : gallop_at_least<W>(T, n, key, p + 4);
    if (lo >= n) {               // cannot happen for an occupied bucket; stay in bounds
        cnt = 0;
        return;
    }
    const uint32_t end = gallop_at_least<W>(T, n, (uint64_t)key + 1, lo + 1);
    cnt = end - lo;
}

// The query's words (wave-uniform) and its key in table a.
template <int W>
__device__ __forceinline__ uint32_t query_key(const mih::MihArgs &A, uint32_t q, uint32_t a, uint64_t (&g)[W])
{
#pragma unroll
    for (int w = 0; w < W; ++w) g[w] = u64_uniform<W>(A.qb.queries[(uint64_t)q * W + w]);
    return table_key<W>(g, A.tables[a]);
}

// The buckets of a lane's J consecutive masks of rank r0 .. r0 + nmy - 1
// (among the `nbits`-bit masks with `rho` set bits, xored into key_base):
// their table positions [lo, lo + cnt) and, for HEADS tables, their first
// codes.  Empty buckets (and masks past nmy) get cnt = 0.
template <int W, int TM, int J>
__device__ __forceinline__ void lookup_block(const mih::MihArgs &A, const TableDev &T, uint32_t key_base,
                                             uint32_t nbits, uint32_t rho, uint32_t r0, uint32_t nmy,
                                             const uint32_t (*binom)[MIH_BINOM_N], uint32_t (&lo)[J],
                                             uint32_t (&cnt)[J], uint64_t (&head_code)[J])
{
    uint32_t keys[J];
    uint32_t mask = nmy ? unrank_mask(r0, rho, nbits, binom) : 0u;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        keys[j] = key_base ^ mask;
        if ((uint32_t)j + 1 < nmy && rho > 0) mask = next_mask(mask);
    }
    // DIRECT tables with the occupancy filter: one bit per bucket says
    // whether it holds codes; only occupied buckets read their offsets.
    // GROUPED tables: the group record holds the same bits.
    uint32_t occ_bits = ~0u;
    uint32_t gbase[J];
    if (TM == mih::TM_GROUPED) {
        occ_bits = 0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            gbase[j] = 0;
            if ((uint32_t)j < nmy) {
                const uint64_t rec = T.grp[keys[j] >> 5];
                const uint32_t bit = keys[j] & 31, occ = (uint32_t)rec;
                if ((occ >> bit) & 1u) occ_bits |= 1u << j;
                // every occupied bucket below this one in the group holds
                // at least one code: the bucket starts no earlier than here
                gbase[j] = (uint32_t)(rec >> 32) + __popc(occ & ((1u << bit) - 1u));
            }
        }
    } else if ((TM == mih::TM_HEADS || TM == mih::TM_DIRECT) && A.occ_filter) {
        occ_bits = 0;
#pragma unroll
        for (int j = 0; j < J; ++j)
            if ((uint32_t)j < nmy && ((T.occ[keys[j] >> 5] >> (keys[j] & 31)) & 1u)) occ_bits |= 1u << j;
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        cnt[j] = 0;
        lo[j] = 0;
        if ((uint32_t)j < nmy && ((occ_bits >> j) & 1u)) {
            const uint32_t key = keys[j];
            if (TM == mih::TM_GROUPED) {
                group_scan<W>(T, A.n, key, gbase[j], lo[j], cnt[j]);
            } else if (TM == mih::TM_HEADS) {
                const BucketHead h = T.head[key];   // one 16-byte entry, one line
                lo[j] = h.start;
                cnt[j] = h.count;
                head_code[j] = h.code;
            } else if (TM == mih::TM_DIRECT) {
                const uint32_t b0 = T.off[key];
                const uint32_t b1 = T.off[(uint64_t)key + 1];
                lo[j] = b0;
                cnt[j] = b1 - b0;
            } else {
                const uint32_t cell = key >> (T.len - T.dir_bits);
                uint32_t x0 = T.dir[cell], x1 = T.dir[(uint64_t)cell + 1];
                // first position with keys >= key, then first with keys > key
                uint32_t l = x0, h = x1;
                while (l < h) {
                    uint32_t mid = l + ((h - l) >> 1);
                    if (T.keys[mid] < key) l = mid + 1; else h = mid;
                }
                uint32_t e = l;
                h = x1;
                while (e < h) {
                    uint32_t mid = e + ((h - e) >> 1);
                    if (T.keys[mid] <= key) e = mid + 1; else h = mid;
                }
                lo[j] = l;
                cnt[j] = e - l;
            }
        }
    }
}

// Part of step t of query q: the buckets key_base ^ mask for the masks of
// rank [rb, re) among the `nbits`-bit masks with `rho` set bits.  A whole
// step is key_base = the query's key, nbits = s_a, rho = t / m; one key
// partition of a step (the sweep kernel) fixes the high bits of the key and
// enumerates the rest.
// Buckets a wave lists for offering in pieces (round kernel), per wave.
constexpr uint32_t kSpillList = 64;

// Returns how many huge buckets (more than A.spill_min codes; never when
// spill_min is 0) it listed in big[] instead of walking them: the caller
// offers them in pieces (spill_bucket).  A full list leaves the rest to
// this wave's walk.
template <int W, int TM, bool INLINE, int J, bool SPILL = false>
__device__ uint32_t process_step(const mih::MihArgs &A, uint32_t q, uint32_t t, uint32_t key_base,
                                 uint32_t nbits, uint32_t rho, uint32_t rb, uint32_t re,
                                 const uint32_t (*binom)[MIH_BINOM_N], uint32_t *stage_pos,
                                 uint32_t *stage_cum, uint64_t *stage_code, WaveStats &ws,
                                 uint2 *big = nullptr)
{
    uint32_t nbig = 0;
    const uint32_t lane = lane_id();
    const uint32_t m = A.m;
    const uint32_t rp = t / m, a = t - rp * m;
    const TableDev T = A.tables[a];
    // codes in table order: every table of an INLINE index, the leading
    // tables of a MIXED one (whose kernels are the indirect ones)
    const bool tinl = INLINE || T.codes != nullptr;
    uint64_t g[W];
    (void)query_key<W>(A, q, a, g);
    uint32_t tau = __builtin_amdgcn_readfirstlane(load_relaxed(A.qb.tau + q));

    for (uint32_t base = rb; base < re; base += MIH_WAVE * J) {
        const uint32_t r0 = base + lane * J;
        const uint32_t nmy = r0 < re ? (re - r0 < (uint32_t)J ? re - r0 : (uint32_t)J) : 0u;
        uint32_t lo[J], cnt[J];
        uint64_t head_code[J];   // HEADS: the first code of each bucket
        lookup_block<W, TM, J>(A, T, key_base, nbits, rho, r0, nmy, binom, lo, cnt, head_code);
        // buckets of more than spill_min codes are listed, not staged
        if (SPILL) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const uint32_t slot = nbig + lanes_below(__ballot(cnt[j] > A.spill_min));
                const bool b = cnt[j] > A.spill_min && slot < kSpillList;
                if (b) {
                    big[slot] = make_uint2(lo[j], cnt[j]);
                    cnt[j] = 0;
                }
                nbig += (uint32_t)__popcll(__ballot(b));
            }
        }
        // stage the non-empty buckets of the wave with the running count of
        // candidates before each, then walk the candidates 64 at a time
        uint32_t ne = 0, tc = 0;
#pragma unroll
        for (int j = 0; j < J; ++j) { ne += cnt[j] ? 1u : 0u; tc += cnt[j]; }
        const uint32_t ne_incl = wave_inclusive_sum(ne);
        const uint32_t tc_incl = wave_inclusive_sum(tc);
        const uint32_t NE = __shfl(ne_incl, MIH_WAVE - 1, MIH_WAVE);
        const uint32_t TC = __shfl(tc_incl, MIH_WAVE - 1, MIH_WAVE);
        uint32_t p = ne_incl - ne, c = tc_incl - tc;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if (cnt[j]) {
                stage_pos[p] = lo[j];
                stage_cum[p] = c;
                if (TM == mih::TM_HEADS) stage_code[p] = head_code[j];
                ++p;
                c += cnt[j];
            }
        }
        wave_lds_sync();
        ws.probes += __shfl(wave_inclusive_sum(nmy), MIH_WAVE - 1, MIH_WAVE);
        ws.candidates += TC;

        constexpr int kWalk = walk_depth<W>();
        // the candidates are walked kWalk x 64 at a time: lane l takes
        // e0 + 64 u + l for u < kWalk, so every load instruction covers 64
        // consecutive table positions, and the kWalk loads of a lane are in
        // flight together
        for (uint32_t e0 = 0; e0 < TC; e0 += MIH_WAVE * kWalk) {
            const uint32_t nu = (TC - e0 + MIH_WAVE - 1) / MIH_WAVE;   // live slices (wave-uniform)
            uint32_t bl[kWalk], pos[kWalk], id[kWalk];
            bool live[kWalk];
            uint64_t code[kWalk][W];
            // staged bucket of each candidate: the last one whose running
            // count is <= e (branch-free halving, the searches interleaved)
#pragma unroll
            for (int u = 0; u < kWalk; ++u) bl[u] = 0;
            for (uint32_t len = NE; len > 1;) {
                const uint32_t half = len >> 1;
#pragma unroll
                for (int u = 0; u < kWalk; ++u)
                    if ((uint32_t)u < nu && stage_cum[bl[u] + half] <= e0 + u * MIH_WAVE + lane) bl[u] += half;
                len -= half;
            }
#pragma unroll
            for (int u = 0; u < kWalk; ++u) {
                const uint32_t e = e0 + u * MIH_WAVE + lane;
                live[u] = e < TC;
                pos[u] = live[u] ? stage_pos[bl[u]] + (e - stage_cum[bl[u]]) : 0u;
                id[u] = 0;
                if (!tinl && live[u]) id[u] = T.ids[pos[u]];
            }
#pragma unroll
            for (int u = 0; u < kWalk; ++u) {
                if (live[u]) {
                    if (TM == mih::TM_HEADS && e0 + u * MIH_WAVE + lane == stage_cum[bl[u]]) {
                        code[u][0] = stage_code[bl[u]];   // a bucket's first code came with its offsets
                    } else if (tinl) {
                        load_code<W>(T.codes + (uint64_t)pos[u] * W, code[u]);
                    } else {
                        load_code<W>(A.codes + (uint64_t)id[u] * W, code[u]);
                    }
                } else {
#pragma unroll
                    for (int w = 0; w < W; ++w) code[u][w] = g[w];
                }
            }
#pragma unroll
            for (int u = 0; u < kWalk; ++u) {
                if ((uint32_t)u >= nu) break;
                const uint32_t d = hamming<W>(code[u], g);
                // first encounter of the code (the de-duplication rule
                // above); every candidate is tested when distinct codes are
                // counted, else only those within tau
                bool first = live[u] && (A.count_unique || d <= tau);
                if (first) {
                    uint64_t x[W];
#pragma unroll
                    for (int w = 0; w < W; ++w) x[w] = code[u][w] ^ g[w];
                    for (uint32_t j = 0; j < m; ++j) {
                        if (j == a) continue;
                        const uint32_t dj = table_dist<W>(x, A.tables[j]);
                        if (j < a ? dj <= rp : dj < rp) { first = false; break; }
                    }
                }
                if (A.count_unique) {
                    const uint64_t fb = __ballot(first);
                    if (fb && lane == 0) atomicAdd(A.uniq + q, (uint32_t)__popcll(fb));
                }
                const bool keep = first && d <= tau;
                if (keep && tinl) id[u] = T.ids[pos[u]];
                append_candidates(A.qb, q, keep, d, id[u]);
                if (__ballot(keep)) tau = tighten_tau(A.qb, q, tau);
            }
        }
        wave_lds_sync();
        const uint32_t g_tau = __builtin_amdgcn_readfirstlane(load_relaxed(A.qb.tau + q));
        tau = g_tau < tau ? g_tau : tau;
    }
    return nbig;
}

// The codes at table positions [pos0, pos0 + len) of step t's table, all in
// one bucket of query q: verified, de-duplicated and appended as in
// process_step (the pieces of a spilled bucket).
template <int W, bool INLINE>
__device__ __forceinline__ void walk_range(const mih::MihArgs &A, uint32_t q, uint32_t t, uint32_t pos0,
                                           uint32_t len, WaveStats &ws)
{
    const uint32_t lane = lane_id();
    const uint32_t m = A.m;
    const uint32_t rp = t / m, a = t - rp * m;
    const TableDev &T = A.tables[a];
    const bool tinl = INLINE || T.codes != nullptr;
    uint64_t g[W];
    (void)query_key<W>(A, q, a, g);
    uint32_t tau = __builtin_amdgcn_readfirstlane(load_relaxed(A.qb.tau + q));
    ws.candidates += len;
    constexpr int kWalk = walk_depth<W>();
    for (uint32_t e0 = 0; e0 < len; e0 += MIH_WAVE * kWalk) {
        uint32_t id[kWalk];
        bool live[kWalk];
        uint64_t code[kWalk][W];
#pragma unroll
        for (int u = 0; u < kWalk; ++u) {
            const uint32_t e = e0 + u * MIH_WAVE + lane;
            live[u] = e < len;
            id[u] = (!tinl && live[u]) ? T.ids[pos0 + e] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kWalk; ++u) {
            const uint32_t pos = pos0 + e0 + u * MIH_WAVE + lane;
            if (live[u]) {
                if (tinl) load_code<W>(T.codes + (uint64_t)pos * W, code[u]);
                else load_code<W>(A.codes + (uint64_t)id[u] * W, code[u]);
            } else {
#pragma unroll
                for (int w = 0; w < W; ++w) code[u][w] = g[w];
            }
        }
#pragma unroll
        for (int u = 0; u < kWalk; ++u) {
            if (e0 + u * MIH_WAVE >= len) continue;   // wave-uniform
            const uint32_t d = hamming<W>(code[u], g);
            bool keep = live[u] && d <= tau;
            if (keep) {
                uint64_t x[W];
#pragma unroll
                for (int w = 0; w < W; ++w) x[w] = code[u][w] ^ g[w];
                for (uint32_t j = 0; j < m; ++j) {
                    if (j == a) continue;
                    const uint32_t dj = table_dist<W>(x, A.tables[j]);
                    if (j < a ? dj <= rp : dj < rp) { keep = false; break; }
                }
            }
            if (keep && tinl) id[u] = T.ids[pos0 + e0 + u * MIH_WAVE + lane];
            append_candidates(A.qb, q, keep, d, id[u]);
            if (__ballot(keep)) tau = tighten_tau(A.qb, q, tau);
        }
    }
}

// Offer the bucket [lo, lo + cnt) of query q's step t in pieces, then take
// every piece no other wave has taken.  With no room left in the round's
// list the wave walks the bucket itself.  Nothing here waits for another
// wave: a piece is walked by whichever wave turns its flag first.
template <int W, bool INLINE>
__device__ __forceinline__ void spill_bucket(const mih::MihArgs &A, uint32_t seq, uint32_t q, uint32_t t, uint32_t lo,
                             uint32_t cnt, WaveStats &ws)
{
    const uint32_t lane = lane_id();
    const uint32_t k = (cnt + mih::kSpillPiece - 1) / mih::kSpillPiece;
    unsigned long long e0 = 0;
    if (lane == 0) e0 = atomicAdd(A.spill_tail, (unsigned long long)k);
    e0 = u64_uniform<1>(__shfl(e0, 0, MIH_WAVE));
    if (e0 + k > A.spill_cap) {
        walk_range<W, INLINE>(A, q, t, lo, cnt, ws);
        return;
    }
    for (uint32_t i = lane; i < k; i += MIH_WAVE) {
        const uint32_t off = i * mih::kSpillPiece;
        A.spill[e0 + i] = mih::SpillRec{q, t, lo + off, cnt - off < mih::kSpillPiece ? cnt - off : mih::kSpillPiece};
    }
    __threadfence();   // the pieces before their flags
    for (uint32_t i = lane; i < k; i += MIH_WAVE)
        __hip_atomic_store(A.spill_flag + e0 + i, 2 * seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // take back what nobody has taken, 64 entries at a time
    for (uint32_t b = 0; b < k; b += MIH_WAVE) {
        const bool took = b + lane < k && atomicCAS(A.spill_flag + e0 + b + lane, 2 * seq, 2 * seq + 1) == 2 * seq;
        for (uint64_t won = __ballot(took); won; won &= won - 1) {
            const uint32_t l = (uint32_t)__ffsll((long long)won) - 1;
            const uint32_t off = (b + l) * mih::kSpillPiece;
            walk_range<W, INLINE>(A, q, t, lo + off, cnt - off < mih::kSpillPiece ? cnt - off : mih::kSpillPiece, ws);
        }
    }
}

// Take pieces that other waves offer: batches of 64 consecutive list
// entries through a counter, each lane testing one entry and taking it if
// it is still offered; the wave then walks what its lanes took.  A batch
// that reaches past the entries reserved so far ends the help (such entries,
// and any not yet flagged, are taken by the waves that offer them, which
// take every piece of their own that nobody has).
template <int W, bool INLINE>
__device__ __forceinline__ void help_spilled(const mih::MihArgs &A, uint32_t seq, WaveStats &ws)
{
    const uint32_t lane = lane_id();
    for (;;) {
        unsigned long long c0 = ~0ull, end = 0;
        if (lane == 0) {
            end = load_relaxed(A.spill_tail);
            end = end < A.spill_cap ? end : A.spill_cap;
            if (load_relaxed(A.spill_next) < end) c0 = atomicAdd(A.spill_next, (unsigned long long)MIH_WAVE);
        }
        c0 = u64_uniform<1>(__shfl(c0, 0, MIH_WAVE));
        end = u64_uniform<1>(__shfl(end, 0, MIH_WAVE));
        if (c0 >= end) return;
        const unsigned long long i = c0 + lane;
        bool took = false;
        if (i < end && __hip_atomic_load(A.spill_flag + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 2 * seq)
            took = atomicCAS(A.spill_flag + i, 2 * seq, 2 * seq + 1) == 2 * seq;
        uint64_t won = __ballot(took);
        if (!won) continue;
        __threadfence();   // the pieces were written before their flags
        for (; won; won &= won - 1) {
            const uint32_t l = (uint32_t)__ffsll((long long)won) - 1;
            const mih::SpillRec R = A.spill[c0 + l];
            walk_range<W, INLINE>(A, R.slot, R.t, R.pos, R.len, ws);
        }
    }
}

}  // namespace
