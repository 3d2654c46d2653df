// Multi-index kNN search (Algorithm 3) for a batch of queries on the device.
//
// Search order.  Query g advances through steps t = 0, 1, 2, ...; step t
// uses table a = t mod m and substring radius r' = floor(t/m) and looks up
// every bucket of table a whose value differs from g's substring in exactly
// r' bits (C(s_a, r') buckets, Eq. 1).  After steps 0..t every code within
// Hamming distance t of g has been found (Proposition 2), so the query is
// finished once the codes found within distance t number at least k; with
// the bound tau of the candidate buffer this is the test tau <= t.
//
// De-duplication without per-query state.  A code h with substring distances
// d_0..d_{m-1} is met at every step (r', a) with d_a = r'.  In Algorithm 3's
// order of increasing t = m r' + a its first encounter is t_h =
// min_j (m d_j + j).  A candidate met at step (r', a) is accepted only if no
// table j gives an earlier step: d_j > r' for j < a and d_j >= r' for j > a.
// This keeps exactly the codes the paper's per-query bitstring would keep
// (Section 6, duplicate candidates), with no bitstring to clear, and it does
// not depend on the order in which the device happens to run the steps.
//
// Scheduling.  All queries of a call advance in rounds; a round performs one
// step of every active query, or several when it would otherwise leave
// waves idle (lookahead, decided by the regroup kernel).  The buckets of a
// step are enumerated in colexicographic order of the flip masks and split
// into work items of `chunk` masks; a persistent kernel hands items to waves
// through an atomic counter.  A step that fits in one item is processed by one wave, which
// then carries on with the query's next steps while they remain that small
// (the wave alone owns the query, so it can test termination itself).
// Between rounds a small kernel tests termination, moves unfinished queries
// to their next non-empty step and regroups the active queries by step.
#include "mih_step.h"
#include "topk_dev.h"

namespace {

template <int W, int TM, bool INLINE, int J, bool SPILL>
__global__ __launch_bounds__(MIH_BLOCK) void mih_round_kernel(mih::MihArgs A)
{
    __shared__ uint32_t binom[MIH_BINOM_N][MIH_BINOM_N];
    __shared__ uint32_t stage_pos[kWaves][MIH_WAVE * J];
    __shared__ uint32_t stage_cum[kWaves][MIH_WAVE * J];
    __shared__ uint64_t stage_code[kWaves][TM == mih::TM_HEADS ? MIH_WAVE * J : 1];
    __shared__ uint2 big[kWaves][SPILL ? kSpillList : 1];   // huge buckets of the wave's last step
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (uint32_t i = tid; i < MIH_BINOM_N * MIH_BINOM_N; i += MIH_BLOCK)
        binom[i / MIH_BINOM_N][i % MIH_BINOM_N] = binom_calc(i / MIH_BINOM_N, i % MIH_BINOM_N);
    __syncthreads();

    const uint32_t n_groups = A.ctrl->n_groups;
    const uint64_t total = A.ctrl->total_items;
    const uint32_t chunk = A.chunk;
    const uint32_t seq = SPILL ? A.ctrl->seq : 0u;
    WaveStats ws = {0, 0};
    bool worked = false;
    for (;;) {
        // pieces of huge buckets that other waves offer come first
        if (SPILL) help_spilled<W, INLINE>(A, seq, ws);
        uint64_t item = 0;
        if (lane == 0) item = atomicAdd(A.work, 1ull);
        item = u64_uniform<1>(__shfl(item, 0, MIH_WAVE));
        if (item >= total) break;
        worked = true;
        // group of the item: the last group whose first item is <= item
        uint32_t gl = 0, gh = n_groups;
        while (gh - gl > 1) {
            uint32_t mid = (gl + gh) >> 1;
            if (A.groups[mid].item_start <= item) gl = mid; else gh = mid;
        }
        gl = __builtin_amdgcn_readfirstlane(gl);
        const mih::Group *G = A.groups + gl;
        const uint32_t ipq = G->ipq, steps = G->steps;
        const uint64_t rel = item - G->item_start;
        const uint32_t slot = G->slot_start + (uint32_t)(rel / ipq);
        uint32_t part = (uint32_t)(rel % ipq);
        // the step of the window that holds the item (steps without probes
        // hold no items and are passed over)
        uint32_t u = 0;
        while (u + 1 < steps && G->step_items[u + 1] <= part) ++u;
        part -= G->step_items[u];
        const uint32_t q = A.active[slot];
        uint32_t t = G->t + u;
        const uint32_t rp = t / A.m;
        const uint32_t M = binom[A.tables[t - rp * A.m].len][rp];
        // the window's first step resumes where the last round's portion ended
        if (u == 0 && A.quantum_items) part += A.cursor[q];
        const uint32_t rb = part * chunk;
        const uint32_t re = rb + chunk < M ? rb + chunk : M;
        uint64_t gq[W];
        const uint32_t a0 = t - rp * A.m;
        const uint32_t nbig = process_step<W, TM, INLINE, J, SPILL>(
            A, q, t, query_key<W>(A, q, a0, gq), A.tables[a0].len, rp, rb, re, binom, stage_pos[wave],
            stage_cum[wave], stage_code[wave], ws, big[wave]);
        // huge buckets: offered in pieces to the other waves, this wave
        // taking those they have not
        if (SPILL)
            for (uint32_t i = 0; i < nbig; ++i)
                spill_bucket<W, INLINE>(A, seq, q, t, big[wave][i].x, big[wave][i].y, ws);
        if (ipq != 1 || steps != 1 || !G->final) continue;
        // the whole step (or its last portion) belonged to this wave: keep
        // going while steps are small
        for (;;) {
            const uint32_t tau = tighten_tau(A.qb, q, __builtin_amdgcn_readfirstlane(load_relaxed(A.qb.tau + q)));
            if (tau <= t || t >= A.t_all || t >= A.max_t[q]) break;
            if (A.budget[q] && (uint32_t)__builtin_amdgcn_readfirstlane(load_relaxed(A.uniq + q)) >= A.budget[q])
                break;
            const uint32_t tn = t + 1;
            const uint32_t rpn = tn / A.m;
            const uint32_t Mn = binom[A.tables[tn - rpn * A.m].len][rpn];
            if (Mn > chunk) break;
            if (SPILL) help_spilled<W, INLINE>(A, seq, ws);   // others' huge buckets first
            if (Mn) {
                const uint32_t an = tn - rpn * A.m;
                const uint32_t nb = process_step<W, TM, INLINE, J, SPILL>(
                    A, q, tn, query_key<W>(A, q, an, gq), A.tables[an].len, rpn, 0, Mn, binom, stage_pos[wave],
                    stage_cum[wave], stage_code[wave], ws, big[wave]);
                if (SPILL)
                    for (uint32_t i = 0; i < nb; ++i)
                        spill_bucket<W, INLINE>(A, seq, q, tn, big[wave][i].x, big[wave][i].y, ws);
            }
            t = tn;
            if (lane == 0) {
                A.t[q] = t;
                A.cursor[q] = 0;
            }
        }
    }
    // out of work items: take what is offered now, then leave (waiting for
    // more would put device-scope polls of many waves on the path of the
    // atomics of the waves still searching)
    if (lane == 0 && worked) record_end(A.stats + mih::kStatRoundEnd);
    if (SPILL) help_spilled<W, INLINE>(A, seq, ws);
    if (lane == 0) {
        atomicAdd(&A.stats[0], (unsigned long long)ws.probes);
        atomicAdd(&A.stats[1], (unsigned long long)ws.candidates);
    }
}

// Per-wave LDS state of a sweep item: its queries and staged buckets.
template <int W, int J>
struct SweepLds {
    uint32_t qstart[mih::kSweepQueries + 1];   // exclusive prefix of the masks per query
    uint32_t qkey[mih::kSweepQueries];         // partition bits | low bits of the query's key
    uint32_t qrho[mih::kSweepQueries];         // set bits of the query's masks
    uint32_t qslot[mih::kSweepQueries];
    uint32_t qtau[mih::kSweepQueries];         // bound of the query (refreshed after appends)
    uint64_t qg[mih::kSweepQueries][W];        // the query's words
    uint32_t stage_pos[MIH_WAVE * J];
    uint32_t stage_cum[MIH_WAVE * J];
    uint32_t stage_q[MIH_WAVE * J];
};

// First lookup of a probe: DIRECT with the occupancy filter the bucket's
// occupancy word, DIRECT its two offsets, GROUPED the group record,
// SORTED the bounds of the directory cell.
template <int TM>
__device__ __forceinline__ void first_lookup(const TableDev &T, uint32_t occ_filter, uint32_t key,
                                             uint32_t &pa, uint32_t &pb)
{
    if (TM == mih::TM_GROUPED) {
        const uint64_t rec = T.grp[key >> 5];
        pa = (uint32_t)rec;
        pb = (uint32_t)(rec >> 32);
    } else if (TM == mih::TM_HEADS) {
        pa = T.occ[key >> 5];
        pb = 0;
    } else if (TM == mih::TM_DIRECT) {
        if (occ_filter) {
            pa = T.occ[key >> 5];
            pb = 0;
        } else {
            pa = T.off[key];
            pb = T.off[(uint64_t)key + 1];
        }
    } else {
        const uint32_t cell = key >> (T.len - T.dir_bits);
        pa = T.dir[cell];
        pb = T.dir[(uint64_t)cell + 1];
    }
}

// The bucket [lo, lo + cnt) of a probe from its first lookup.
template <int W, int TM>
__device__ __forceinline__ void second_lookup(const TableDev &T, uint64_t n, uint32_t occ_filter,
                                              uint32_t key, uint32_t pa, uint32_t pb, uint32_t &lo,
                                              uint32_t &cnt)
{
    lo = cnt = 0;
    if (TM == mih::TM_GROUPED) {
        const uint32_t bit = key & 31;
        if ((pa >> bit) & 1u) group_scan<W>(T, n, key, pb + __popc(pa & ((1u << bit) - 1u)), lo, cnt);
    } else if (TM == mih::TM_HEADS) {
        if ((pa >> (key & 31)) & 1u) {
            const BucketHead h = T.head[key];
            lo = h.start;
            cnt = h.count;
        }
    } else if (TM == mih::TM_DIRECT) {
        if (occ_filter) {
            if ((pa >> (key & 31)) & 1u) {
                const uint32_t b0 = T.off[key];
                lo = b0;
                cnt = T.off[(uint64_t)key + 1] - b0;
            }
        } else {
            lo = pa;
            cnt = pb - pa;
        }
    } else {
        uint32_t l = pa, h = pb;
        while (l < h) {
            const uint32_t mid = l + ((h - l) >> 1);
            if (T.keys[mid] < key) l = mid + 1; else h = mid;
        }
        uint32_t e = l;
        h = pb;
        while (e < h) {
            const uint32_t mid = e + ((h - e) >> 1);
            if (T.keys[mid] <= key) e = mid + 1; else h = mid;
        }
        lo = l;
        cnt = e - l;
    }
}

// One sweep item: partition h of the key space of table a (values whose
// high s - L bits equal h) for up to kSweepQueries queries of a group at
// step t.  A query meets partition h only through the L-bit masks with
// r' - popc((key_q >> L) ^ h) set bits; over all h these are exactly the
// C(s, r') buckets of the step (Vandermonde's identity).  The masks of all
// the item's queries form one flat list that the lanes share, J per lane
// per block, so that a query with a handful of masks in this partition does
// not leave the wave idle.  Candidates keep their query; appends use one
// atomic each, and the bound of each query with new candidates is
// tightened once per block.
template <int W, int TM, bool INLINE, int J>
__device__ void sweep_item(const mih::MihArgs &A, const mih::Group &G, uint32_t h, uint32_t c,
                           const uint32_t (*binom)[MIH_BINOM_N], SweepLds<W, J> &S, WaveStats &ws)
{
    const uint32_t lane = lane_id();
    const uint32_t t = G.t, rp = t / A.m, a = t - rp * A.m;
    const TableDev T = A.tables[a];
    const bool tinl = INLINE || T.codes != nullptr;   // this table's codes in table order
    const uint32_t L = G.sweep_bits;
    const uint32_t low = L >= 32 ? 0xFFFFFFFFu : ((1u << L) - 1u);
    const uint32_t i0 = c * mih::kSweepQueries;
    const uint32_t nq = G.count - i0 < mih::kSweepQueries ? G.count - i0 : mih::kSweepQueries;

    // lane i: query i of the chunk, its part of this partition
    uint32_t M = 0;
    if (lane < nq) {
        const uint32_t q = A.active[G.slot_start + i0 + lane];
        uint64_t g[W];
#pragma unroll
        for (int w = 0; w < W; ++w) g[w] = A.qb.queries[(uint64_t)q * W + w];
        const uint32_t key = table_key<W>(g, A.tables[a]);   // not the local copy (see part_queries)
        const uint32_t wgt = __popc((L >= 32 ? 0u : key >> L) ^ h);
        const uint32_t rho = wgt <= rp ? rp - wgt : 0xFFFFFFFFu;
        M = rho <= L ? binom[L][rho] : 0u;
        S.qkey[lane] = (uint32_t)((uint64_t)h << L) | (key & low);
        S.qrho[lane] = rho <= L ? rho : 0u;
        S.qslot[lane] = q;
        S.qtau[lane] = load_relaxed(A.qb.tau + q);
#pragma unroll
        for (int w = 0; w < W; ++w) S.qg[lane][w] = g[w];
    }
    const uint32_t incl = wave_inclusive_sum(M);
    if (lane < mih::kSweepQueries) S.qstart[lane] = incl - M;
    if (lane == mih::kSweepQueries - 1) S.qstart[mih::kSweepQueries] = incl;
    wave_lds_sync();
    const uint32_t total = S.qstart[mih::kSweepQueries];
    ws.probes += total;

    for (uint32_t base = 0; base < total; base += MIH_WAVE * J) {
        const uint32_t f0 = base + lane * J;
        const uint32_t nmy = f0 < total ? (total - f0 < (uint32_t)J ? total - f0 : (uint32_t)J) : 0u;
        uint32_t keys[J], qi[J], lo[J], cnt[J];
        uint32_t cur = 0, mask = 0;
        if (nmy) {
            // the query whose masks contain flat index f0: last start <= f0
            uint32_t l = 0, hh = mih::kSweepQueries;
            while (hh - l > 1) {
                const uint32_t mid = (l + hh) >> 1;
                if (S.qstart[mid] <= f0) l = mid; else hh = mid;
            }
            cur = l;
            mask = unrank_mask(f0 - S.qstart[cur], S.qrho[cur], L, binom);
        }
#pragma unroll
        for (int j = 0; j < J; ++j) {
            keys[j] = S.qkey[cur] ^ mask;
            qi[j] = cur;
            if ((uint32_t)j + 1 < nmy) {
                const uint32_t f = f0 + j + 1;
                if (f < S.qstart[cur + 1]) {
                    mask = next_mask(mask);
                } else {
                    while (S.qstart[cur + 1] <= f) ++cur;   // f < total, so this stops
                    mask = (1u << S.qrho[cur]) - 1u;        // the first mask of that query
                }
            }
        }
        uint32_t pa[J], pb[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            pa[j] = pb[j] = 0;
            if ((uint32_t)j < nmy) first_lookup<TM>(T, A.occ_filter, keys[j], pa[j], pb[j]);
        }
#pragma unroll
        for (int j = 0; j < J; ++j) {
            lo[j] = cnt[j] = 0;
            if ((uint32_t)j < nmy) second_lookup<W, TM>(T, A.n, A.occ_filter, keys[j], pa[j], pb[j], lo[j], cnt[j]);
        }
        // stage the non-empty buckets with their query
        uint32_t ne = 0, tc = 0;
#pragma unroll
        for (int j = 0; j < J; ++j) { ne += cnt[j] ? 1u : 0u; tc += cnt[j]; }
        const uint32_t ne_incl = wave_inclusive_sum(ne);
        const uint32_t tc_incl = wave_inclusive_sum(tc);
        const uint32_t NE = __shfl(ne_incl, MIH_WAVE - 1, MIH_WAVE);
        const uint32_t TC = __shfl(tc_incl, MIH_WAVE - 1, MIH_WAVE);
        uint32_t p = ne_incl - ne, cc = tc_incl - tc;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if (cnt[j]) {
                S.stage_pos[p] = lo[j];
                S.stage_cum[p] = cc;
                S.stage_q[p] = qi[j];
                ++p;
                cc += cnt[j];
            }
        }
        wave_lds_sync();
        ws.candidates += TC;

        uint64_t touched = 0;   // queries of the item that received candidates
        for (uint32_t e0 = 0; e0 < TC; e0 += MIH_WAVE) {
            const uint32_t e = e0 + lane;
            const bool live = e < TC;
            uint32_t bl = 0, bh = NE;
            while (bh - bl > 1) {
                const uint32_t mid = (bl + bh) >> 1;
                if (S.stage_cum[mid] <= e) bl = mid; else bh = mid;
            }
            bool keep = false;
            if (live) {
                const uint32_t pos = S.stage_pos[bl] + (e - S.stage_cum[bl]);
                const uint32_t k = S.stage_q[bl];
                uint64_t code[W], g[W];
                uint32_t id = 0;
#pragma unroll
                for (int w = 0; w < W; ++w) g[w] = S.qg[k][w];
                if (tinl) {
                    load_code<W>(T.codes + (uint64_t)pos * W, code);
                } else {
                    id = T.ids[pos];
                    load_code<W>(A.codes + (uint64_t)id * W, code);
                }
                const uint32_t d = hamming<W>(code, g);
                keep = d <= S.qtau[k];
                if (keep) {
                    uint64_t x[W];
#pragma unroll
                    for (int w = 0; w < W; ++w) x[w] = code[w] ^ g[w];
                    for (uint32_t j = 0; j < A.m; ++j) {
                        if (j == a) continue;
                        const uint32_t dj = table_dist<W>(x, A.tables[j]);
                        if (j < a ? dj <= rp : dj < rp) { keep = false; break; }
                    }
                }
                if (keep) {
                    if (tinl) id = T.ids[pos];
                    const uint32_t q = S.qslot[k];
                    const uint32_t slot = atomicAdd(&A.qb.count[q], 1u);
                    if (slot < A.qb.cap[q]) A.qb.buf[A.qb.buf_off[q] + slot] = ((uint64_t)d << 32) | id;
                    atomicAdd(&A.qb.hist[(uint64_t)q * (A.qb.bits + 1) + d], 1u);
                    touched |= 1ull << k;
                }
            }
        }
        // tighten the bound of every query with new candidates (wave-wide)
        uint64_t tq = touched;
#pragma unroll
        for (int sh = 1; sh < MIH_WAVE; sh <<= 1) tq |= (uint64_t)__shfl_xor((long long)tq, sh, MIH_WAVE);
        tq = u64_uniform<1>(tq);
        while (tq) {
            const uint32_t k = (uint32_t)__ffsll((long long)tq) - 1;
            tq &= tq - 1;
            const uint32_t nt = tighten_tau(A.qb, S.qslot[k], S.qtau[k]);
            if (lane == 0) S.qtau[k] = nt;
        }
        wave_lds_sync();
    }
}

// The steps of swept groups, partition-major over the key space of their
// table.  Partition h goes to XCD h mod 8 (workgroups are dispatched to the
// eight XCDs in turn), so that the items of one partition, which read the
// same occupancy words, offsets and codes, share that XCD's L2; a wave
// first drains its own XCD's items, then helps the others.
template <int W, int TM, bool INLINE, int J>
__global__ __launch_bounds__(MIH_BLOCK) void mih_sweep_kernel(mih::MihArgs A)
{
    __shared__ uint32_t binom[MIH_BINOM_N][MIH_BINOM_N];
    __shared__ SweepLds<W, J> lds[kWaves];
    const uint64_t per_xcd = A.ctrl->sweep_items;
    if (per_xcd == 0) return;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (uint32_t i = tid; i < MIH_BINOM_N * MIH_BINOM_N; i += MIH_BLOCK)
        binom[i / MIH_BINOM_N][i % MIH_BINOM_N] = binom_calc(i / MIH_BINOM_N, i % MIH_BINOM_N);
    __syncthreads();

    const uint32_t n_groups = A.ctrl->n_groups;
    const uint32_t home = blockIdx.x % mih::kSweepXcds;
    WaveStats ws = {0, 0};
    bool worked = false;
    for (uint32_t k = 0; k < mih::kSweepXcds; ++k) {
        const uint32_t x = (home + k) % mih::kSweepXcds;
        for (;;) {
            // kSweepBatch consecutive items per claim: fewer atomics on the
            // XCD's counter, and the items of a claim share a partition
            uint64_t first = 0;
            if (lane == 0) first = atomicAdd(A.work_sweep + x, (unsigned long long)mih::kSweepBatch);
            first = u64_uniform<1>(__shfl(first, 0, MIH_WAVE));
            if (first >= per_xcd) break;
            worked = true;
            const uint64_t last = first + mih::kSweepBatch < per_xcd ? first + mih::kSweepBatch : per_xcd;
            for (uint64_t item = first; item < last; ++item) {
                uint32_t gl = 0, gh = n_groups;
                while (gh - gl > 1) {
                    const uint32_t mid = (gl + gh) >> 1;
                    if (A.groups[mid].sweep_start <= item) gl = mid; else gh = mid;
                }
                const mih::Group G = A.groups[gl];
                if (G.sweep_qc == 0) continue;   // not a swept group (cannot own an item)
                const uint64_t rel = item - G.sweep_start;
                const uint32_t h = (uint32_t)(rel / G.sweep_qc) * mih::kSweepXcds + x;
                const uint32_t c = (uint32_t)(rel % G.sweep_qc);
                sweep_item<W, TM, INLINE, J>(A, G, h, c, binom, lds[wave], ws);
            }
        }
    }
    if (lane == 0) {
        atomicAdd(&A.stats[0], (unsigned long long)ws.probes);
        atomicAdd(&A.stats[1], (unsigned long long)ws.candidates);
        if (worked) record_end(A.stats + mih::kStatSweepEnd);
    }
}

// ------------------------------------------------------------------------
// Partition sweep of large steps on tables with an occupancy map (DIRECT
// with the occupancy filter, HEADS).
//
// A step of r' over a table of s bits probes C(s, r') buckets per query;
// for the large steps of a big batch that is more probes than the table has
// buckets, and probing query by query reads the same occupancy words over
// and over from HBM (one 64-byte line holds the bits of 512 buckets).  Here
// the key space is cut into partitions of 2^L values; a work item is one
// partition and a chunk of the group's queries, run by one workgroup: the
// partition's occupancy bits (2^L / 8 bytes) are staged in LDS once, then
// every query of the chunk enumerates the buckets of its step that fall in
// the partition (those whose high s - L bits differ from the query's in w
// places, with r' - w of the low L bits flipped; over all partitions these
// are exactly the C(s, r') buckets of the step, by Vandermonde's identity)
// and tests them against LDS.  Only occupied buckets are read from HBM.
// Partitions are dealt to the eight XCDs in turn (workgroups are dispatched
// to them in turn) and the chunks of one partition are consecutive items,
// so that the workgroups of an XCD work on few partitions at a time and
// share their bucket lines in that XCD's L2.
//
// A lane walks J consecutive masks of the flat list of the wave's 64
// queries and tests them against LDS; the occupied buckets go to a queue
// in LDS, and once it holds a full pass, every lane reads kPartDepth bucket
// entries at once (HEADS: offset, size and first code in one 16-byte read),
// so that the wave keeps 64 kPartDepth independent reads in flight.  Most
// buckets hold one code; the further codes of a bucket are read level by
// level, kPartDepth at a time.
constexpr uint32_t kPartDepth = 4;

template <int W, int J>
struct PartLds {
    // the queue holds what a pass leaves plus one block of masks
    static constexpr uint32_t kQueue = MIH_WAVE * (kPartDepth + J);
    uint32_t qstart[MIH_WAVE + 1];   // exclusive prefix of the masks per query
    uint32_t qkey[MIH_WAVE];         // partition bits | low bits of the query's key
    uint32_t qrho[MIH_WAVE];         // set bits of the query's masks in the partition
    uint32_t qslot[MIH_WAVE];
    uint32_t qtau[MIH_WAVE];         // bound of the query (refreshed after appends)
    uint64_t qg[MIH_WAVE][W];        // the query's words
    uint32_t queue[kQueue];          // occupied buckets: low key bits << 6 | wave query
    uint16_t pend[2 * MIH_WAVE];     // queries with masks in the partition (index in the work item)
};

// Verify candidate `code` (table position pos) of query k of the wave:
// full distance, the first-encounter rule, then append.  Returns whether
// it was kept.
template <int W, bool TINL, class S>
__device__ __forceinline__ bool part_verify(const mih::MihArgs &A, const TableDev &T, uint32_t a, uint32_t rp,
                                            const S &P, uint32_t k, const uint64_t (&code)[W], uint32_t pos,
                                            uint32_t id)
{
    uint64_t g[W];
#pragma unroll
    for (int w = 0; w < W; ++w) g[w] = P.qg[k][w];
    const uint32_t d = hamming<W>(code, g);
    if (d > P.qtau[k]) return false;
    uint64_t x[W];
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = code[w] ^ g[w];
    for (uint32_t j = 0; j < A.m; ++j) {
        if (j == a) continue;
        const uint32_t dj = table_dist<W>(x, A.tables[j]);
        if (j < a ? dj <= rp : dj < rp) return false;
    }
    if (TINL) id = T.ids[pos];
    const uint32_t q = P.qslot[k];
    const uint32_t slot = atomicAdd(&A.qb.count[q], 1u);
    if (slot < A.qb.cap[q]) A.qb.buf[A.qb.buf_off[q] + slot] = ((uint64_t)d << 32) | id;
    atomicAdd(&A.qb.hist[(uint64_t)q * (A.qb.bits + 1) + d], 1u);
    return true;
}

// One pass over queue entries [head, head + cnt), cnt <= 64 kPartDepth: the
// buckets' entries, then their candidates.  Returns the wave queries that
// received candidates.
template <int W, int TM, bool INLINE, int J>
__device__ uint64_t part_drain(const mih::MihArgs &A, const TableDev &T, uint32_t a, uint32_t rp, uint32_t h,
                               uint32_t L, PartLds<W, J> &S, uint32_t head, uint32_t cnt, WaveStats &ws)
{
    constexpr uint32_t D = kPartDepth, Q = PartLds<W, J>::kQueue;
    const uint32_t lane = lane_id();
    const bool tinl = INLINE || T.codes != nullptr;
    uint32_t lo[D], num[D], qi[D];
    uint64_t first[D];
#pragma unroll
    for (uint32_t d = 0; d < D; ++d) {
        const uint32_t e = lane + MIH_WAVE * d;
        lo[d] = num[d] = qi[d] = 0;
        first[d] = 0;
        if (e < cnt) {
            const uint32_t v = S.queue[(head + e) % Q];
            const uint32_t key = (h << L) | (v >> 6);
            qi[d] = v & 63u;
            if (TM == mih::TM_HEADS) {
                const BucketHead hd = T.head[key];
                lo[d] = hd.start;
                num[d] = hd.count;
                first[d] = hd.code;
            } else {
                const uint32_t b0 = T.off[key];
                lo[d] = b0;
                num[d] = T.off[(uint64_t)key + 1] - b0;
            }
        }
    }
    uint32_t tc = 0, most = 0;
#pragma unroll
    for (uint32_t d = 0; d < D; ++d) {
        tc += num[d];
        most = num[d] > most ? num[d] : most;
    }
    ws.candidates += wave_sum(tc);
    uint64_t touched = 0;
    // level c: the c-th code of each of the lane's buckets (HEADS: level 0
    // came with the entries)
    for (uint32_t c = 0; __ballot(c < most); ++c) {
        uint64_t code[D][W];
        uint32_t id[D];
#pragma unroll
        for (uint32_t d = 0; d < D; ++d) {
            id[d] = 0;
            if (c < num[d]) {
                const uint32_t pos = lo[d] + c;
                if (TM == mih::TM_HEADS && c == 0) {
                    code[d][0] = first[d];
                } else if (tinl) {
                    load_code<W>(T.codes + (uint64_t)pos * W, code[d]);
                } else {
                    id[d] = T.ids[pos];
                    load_code<W>(A.codes + (uint64_t)id[d] * W, code[d]);
                }
            }
        }
#pragma unroll
        for (uint32_t d = 0; d < D; ++d) {
            if (c < num[d] && (tinl ? part_verify<W, true>(A, T, a, rp, S, qi[d], code[d], lo[d] + c, id[d])
                                    : part_verify<W, false>(A, T, a, rp, S, qi[d], code[d], lo[d] + c, id[d])))
                touched |= 1ull << qi[d];
        }
    }
    return touched;
}

// Tighten the bound of every wave query in `touched` (any lane's bits).
template <int W, int J>
__device__ void part_tighten(const mih::MihArgs &A, PartLds<W, J> &S, uint64_t touched)
{
    uint64_t tq = touched;
#pragma unroll
    for (int sh = 1; sh < MIH_WAVE; sh <<= 1) tq |= (uint64_t)__shfl_xor((long long)tq, sh, MIH_WAVE);
    tq = u64_uniform<1>(tq);
    while (tq) {
        const uint32_t k = (uint32_t)__ffsll((long long)tq) - 1;
        tq &= tq - 1;
        const uint32_t nt = tighten_tau(A.qb, S.qslot[k], S.qtau[k]);
        if (lane_id() == 0) S.qtau[k] = nt;
    }
    wave_lds_sync();
}

// The queries S.pend[0 .. nq) (at most 64; indices among the active entries
// that start at slot_start: the work item's queries) against partition h of L key
// bits, whose occupancy bits are in `occ` (bit v of the partition: word
// v / 32).
template <int W, int TM, bool INLINE, int J>
__device__ void part_queries(const mih::MihArgs &A, uint32_t t, uint32_t slot_start, uint32_t L, uint32_t h,
                             uint32_t nq, const uint32_t *occ, const uint32_t (*binom)[MIH_BINOM_N],
                             PartLds<W, J> &S, WaveStats &ws)
{
    constexpr uint32_t D = kPartDepth, Q = PartLds<W, J>::kQueue;
    static_assert(Q >= MIH_WAVE * (kPartDepth + J), "queue holds a pass's rest and a block");
    const uint32_t lane = lane_id();
    const uint32_t rp = t / A.m, a = t - rp * A.m;
    const TableDev &T = A.tables[a];
    const uint32_t low = (1u << L) - 1u;

    uint32_t M = 0;
    if (lane < nq) {
        const uint32_t q = A.active[slot_start + S.pend[lane]];
        uint64_t g[W];
#pragma unroll
        for (int w = 0; w < W; ++w) g[w] = A.qb.queries[(uint64_t)q * W + w];
        const uint32_t key = table_key<W>(g, T);
        const uint32_t wgt = __popc((key >> L) ^ h);
        const uint32_t rho = wgt <= rp ? rp - wgt : 0xFFFFFFFFu;
        M = rho <= L ? binom[L][rho] : 0u;
        S.qkey[lane] = (h << L) | (key & low);
        S.qrho[lane] = rho <= L ? rho : 0u;
        S.qslot[lane] = q;
        S.qtau[lane] = load_relaxed(A.qb.tau + q);
#pragma unroll
        for (int w = 0; w < W; ++w) S.qg[lane][w] = g[w];
    }
    const uint32_t incl = wave_inclusive_sum(M);
    S.qstart[lane] = incl - M;
    if (lane == MIH_WAVE - 1) S.qstart[MIH_WAVE] = incl;
    wave_lds_sync();
    const uint32_t total = S.qstart[MIH_WAVE];
    ws.probes += total;

    // each lane walks one contiguous range of the flat list, so that it
    // unranks a mask once per sub-chunk and steps with Gosper's rule after
    // (32-bit: partitions have at most 18 key bits)
    const uint32_t per_lane = (total + MIH_WAVE - 1) / MIH_WAVE;
    const uint32_t f0 = lane * per_lane;
    const uint32_t f_end = f0 + per_lane < total ? f0 + per_lane : total;
    uint32_t cur = 0, mask = 0, qkey = 0, next_start = 0;
    if (f0 < f_end) {
        // the query whose masks hold flat index f0: the last start <= f0
        uint32_t l = 0, hh = MIH_WAVE;
        while (hh - l > 1) {
            const uint32_t mid = (l + hh) >> 1;
            if (S.qstart[mid] <= f0) l = mid; else hh = mid;
        }
        cur = l;
        mask = unrank_mask(f0 - S.qstart[cur], S.qrho[cur], L, binom);
        qkey = S.qkey[cur];
        next_start = S.qstart[cur + 1];
    }
    uint32_t head = 0, tail = 0;   // queue positions (slot = position mod Q)
    for (uint32_t b = 0; b < per_lane; b += J) {
        // the J keys of the block (registers; a query boundary reads the
        // next query's entries), then their J occupancy words together,
        // then the occupied ones to the queue
        uint32_t v[J], qc[J];
        bool valid[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const uint32_t f = f0 + b + j;
            valid[j] = f < f_end;
            v[j] = (qkey ^ mask) & low;
            qc[j] = cur;
            if (f + 1 < next_start) {
                // Gosper's next mask with the same number of set bits
                const uint32_t c = mask & (0u - mask);
                const uint32_t r = mask + c;
                mask = (((r ^ mask) >> 2) >> __builtin_ctz(c | (c == 0 ? 1u : 0u))) | r;
            } else if (f + 1 < f_end) {
                do { ++cur; } while (S.qstart[cur + 1] <= f + 1);   // f + 1 < total: this stops
                mask = (1u << S.qrho[cur]) - 1u;                   // the first mask of that query
                qkey = S.qkey[cur];
                next_start = S.qstart[cur + 1];
            }
        }
        uint32_t word[J];
#pragma unroll
        for (int j = 0; j < J; ++j) word[j] = valid[j] ? occ[v[j] >> 5] : 0u;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const bool hit = (word[j] >> (v[j] & 31)) & 1u;
            const uint64_t bal = __ballot(hit);
            if (hit) S.queue[(tail + lanes_below(bal)) % Q] = (v[j] << 6) | qc[j];
            tail += (uint32_t)__popcll(bal);
        }
        if (tail - head >= MIH_WAVE * D) {
            wave_lds_sync();
            uint64_t touched = 0;
            for (; tail - head >= MIH_WAVE * D; head += MIH_WAVE * D)
                touched |= part_drain<W, TM, INLINE, J>(A, T, a, rp, h, L, S, head, MIH_WAVE * D, ws);
            part_tighten<W, J>(A, S, touched);   // ends with a wave sync: the slots read may be reused
        }
    }
    if (tail != head) {
        wave_lds_sync();
        const uint64_t touched = part_drain<W, TM, INLINE, J>(A, T, a, rp, h, L, S, head, tail - head, ws);
        part_tighten<W, J>(A, S, touched);
    }
}

template <int W, int TM, bool INLINE, int J>
__global__ __launch_bounds__(MIH_BLOCK) void mih_part_kernel(mih::MihArgs A)
{
    __shared__ uint32_t binom[MIH_BINOM_N][MIH_BINOM_N];
    __shared__ PartLds<W, J> pq[kWaves];
    extern __shared__ uint32_t occ[];   // (1 << part_bits) / 32 words
    __shared__ unsigned long long s_item;
    const uint64_t per_xcd = A.ctrl->sweep_items;
    if (per_xcd == 0) return;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (uint32_t i = tid; i < MIH_BINOM_N * MIH_BINOM_N; i += MIH_BLOCK)
        binom[i / MIH_BINOM_N][i % MIH_BINOM_N] = binom_calc(i / MIH_BINOM_N, i % MIH_BINOM_N);

    const uint32_t n_groups = A.ctrl->n_groups;
    const uint32_t home = blockIdx.x % mih::kSweepXcds;
    uint32_t staged_h = 0xFFFFFFFFu, staged_g = 0xFFFFFFFFu;   // partition whose bits are in occ
    WaveStats ws = {0, 0};
    bool worked = false;
    for (uint32_t k = 0; k < mih::kSweepXcds; ++k) {
        const uint32_t x = (home + k) % mih::kSweepXcds;
        for (;;) {
            __syncthreads();   // the previous item is done with occ and s_item
            if (tid == 0) s_item = atomicAdd(A.work_sweep + x, 1ull);
            __syncthreads();
            const uint64_t item = s_item;
            if (item >= per_xcd) break;
            worked = true;
            uint32_t gl = 0, gh = n_groups;
            while (gh - gl > 1) {
                const uint32_t mid = (gl + gh) >> 1;
                if (A.groups[mid].sweep_start <= item) gl = mid; else gh = mid;
            }
            // the fields of the group that the item needs (kept in registers)
            const mih::Group *Gp = A.groups + gl;
            const uint32_t qc = Gp->sweep_qc, gt = Gp->t, gcount = Gp->count, gslot = Gp->slot_start;
            const uint32_t L = Gp->sweep_bits;
            if (qc == 0) continue;   // not a swept group (cannot own an item)
            const uint64_t rel = item - Gp->sweep_start;
            const uint32_t h = (uint32_t)(rel / qc) * mih::kSweepXcds + x;
            const uint32_t c = (uint32_t)(rel % qc);
            if (h != staged_h || gl != staged_g) {
                const uint32_t a = gt % A.m;
                const uint32_t nw = (1u << L) >> 5;
                const uint32_t *src = A.tables[a].occ + ((uint64_t)h << (L - 5));
                for (uint32_t i = tid; i < nw; i += MIH_BLOCK) occ[i] = src[i];
                staged_h = h;
                staged_g = gl;
                __syncthreads();
            }
            // A query meets the partition through C(L, r' - w) masks, w the
            // distance of its key's high bits to h: none when w > r' or
            // r' - w > L (most queries at small r').  Each wave gathers the
            // queries that meet it from its share of the item, and runs them
            // 64 at a time, so that the set-up of a pass is paid for 64
            // queries with masks.
            const uint32_t q0 = c * A.sweep_q;
            const uint32_t qn = gcount - q0 < A.sweep_q ? gcount - q0 : A.sweep_q;
            const uint32_t rp = gt / A.m;
            const TableDev &T = A.tables[gt - rp * A.m];
            PartLds<W, J> &P = pq[wave];
            uint32_t npend = 0;
            for (uint32_t s0 = wave * MIH_WAVE; s0 < qn; s0 += kWaves * MIH_WAVE) {
                bool meets = false;
                if (s0 + lane < qn) {
                    const uint32_t q = A.active[gslot + q0 + s0 + lane];
                    uint64_t g[W];
#pragma unroll
                    for (int w = 0; w < W; ++w) g[w] = A.qb.queries[(uint64_t)q * W + w];
                    const uint32_t wgt = __popc((table_key<W>(g, T) >> L) ^ h);
                    meets = wgt <= rp && rp - wgt <= L;
                }
                const uint64_t bal = __ballot(meets);
                if (meets) P.pend[npend + lanes_below(bal)] = (uint16_t)(s0 + lane);   // < sweep_q <= 4096
                npend += (uint32_t)__popcll(bal);
                if (npend >= MIH_WAVE) {
                    wave_lds_sync();
                    part_queries<W, TM, INLINE, J>(A, gt, gslot + q0, L, h, MIH_WAVE, occ, binom, P, ws);
                    npend -= MIH_WAVE;
                    if (lane < npend) P.pend[lane] = P.pend[MIH_WAVE + lane];
                    wave_lds_sync();
                }
            }
            if (npend) {
                wave_lds_sync();
                part_queries<W, TM, INLINE, J>(A, gt, gslot + q0, L, h, npend, occ, binom, P, ws);
            }
        }
    }
    if (lane == 0) {
        atomicAdd(&A.stats[0], (unsigned long long)ws.probes);
        atomicAdd(&A.stats[1], (unsigned long long)ws.candidates);
        if (worked && wave == 0) record_end(A.stats + mih::kStatSweepEnd);
    }
}


// After a round: termination test for the step each active query just
// finished, and the next non-empty step for the others (a shell is empty
// when r' exceeds the substring length).  Finished queries go to the done
// list, or to the overflow list when their candidate buffer overflowed.
__global__ __launch_bounds__(MIH_BLOCK) void mih_advance_kernel(mih::MihArgs A)
{
    const uint32_t i = blockIdx.x * MIH_BLOCK + threadIdx.x;
    if (i < MIH_WAVE) fold_tails(A.stats);   // the first wave
    if (i >= A.ctrl->n_active) return;
    const uint32_t q = A.active[i];
    const uint32_t nb = A.qb.bits + 1;
    const uint32_t *h = A.qb.hist + (uint64_t)q * nb;
    const uint32_t k = A.qb.k[q];
    uint32_t D = 0xFFFFFFFFu, cum = 0;
    for (uint32_t d = 0; d < nb; ++d) {
        cum += h[d];
        if (cum >= k) { D = d; break; }
    }
    // the bound: the k-th distance found so far, or the query's own radius
    // (r-neighbour queries, exact re-runs) when that is smaller
    uint32_t tau = A.qb.tau[q];
    if (D < tau) { A.qb.tau[q] = D; tau = D; }
    uint32_t t = A.t[q];
    uint32_t out = 0xFFFFFFFFu;
    if (A.quantum_items) {
        // a step cut by the work quantum: its next portion in the next round
        // (the step is not complete, so no termination test yet)
        const uint32_t rp = t / A.m;
        uint32_t M = 0;
        if (rp <= A.tables[t - rp * A.m].len) {
            const uint32_t s = A.tables[t - rp * A.m].len;
            uint64_t c = 1;
            for (uint32_t i = 1; i <= rp; ++i) c = c * (s - rp + i) / i;
            M = (uint32_t)c;
        }
        const uint32_t it = (M + A.chunk - 1) / A.chunk;
        if (A.cursor[q] + A.quantum_items < it) {
            A.cursor[q] += A.quantum_items;
            A.next_t[i] = t;
            return;
        }
        A.cursor[q] = 0;
    }
    // after step t every code within distance t has been found (Prop. 2);
    // an approximate query also stops at its step limit or candidate budget
    const uint32_t max_t = A.max_t[q], budget = A.budget[q];
    const bool spent = budget != 0 && A.uniq[q] >= budget;
    if (!(tau <= t || t >= A.t_all || t >= max_t || spent)) {
        for (uint32_t tn = t + 1; tn <= max_t; ++tn) {
            const uint32_t rp = tn / A.m;
            if (rp <= A.tables[tn - rp * A.m].len) { out = tn; break; }   // C(s, r') > 0
            if (tau <= tn || tn >= A.t_all) break;
        }
    }
    A.next_t[i] = out;
    if (out != 0xFFFFFFFFu) {
        A.t[q] = out;
        return;
    }
    atomicAdd(&A.stats[2], (unsigned long long)t + 1);                  // steps
    atomicAdd(&A.stats[3], (unsigned long long)A.qb.count[q]);          // appended
    if (A.qb.count[q] > A.qb.cap[q]) {
        A.ovf_list[atomicAdd(&A.ctrl->n_ovf, 1u)] = q;
    } else {
        A.done_list[atomicAdd(&A.ctrl->n_done, 1u)] = q;
    }
}

// Start of a round (one workgroup): the queries that survived the last
// advance and the newly admitted ones (at step 0) form the active list,
// grouped by step; the work-item numbering follows the groups.
//
// Lookahead.  When the groups' steps make fewer items than the waves the
// round kernel runs (look_items), groups also take their following steps,
// lowest steps first, one step per group and pass, while the round stays
// within that many items and within look_masks shell masks (a few passes
// of every wave: past that, the extra steps would lengthen the round).  Taking a step early changes no result: a code is
// accepted only at its first step whatever the order the steps run in, the
// bound tau only ever shrinks to a value no smaller than the final k-th
// distance, and after the round every step up to the last one taken has run,
// which is all that the termination test (Proposition 2) needs.  A query of
// the group then resumes after its window's last step.
__global__ __launch_bounds__(1024) void mih_regroup_kernel(mih::MihArgs A)
{
    // Bins: two per step, 2 t for a portion of step t that the work quantum
    // leaves unfinished, 2 t + 1 for the portion that finishes it (or the
    // whole step).  [nbins] counts, [nbins] cursors, [nbins] window ends,
    // then per group (at most one per bin) its first step, query count,
    // items per query and steps taken: the serial part below works in LDS
    // only.
    extern __shared__ uint32_t bins[];
    __shared__ uint32_t binom[MIH_BINOM_N][MIH_BINOM_N];
    __shared__ uint32_t s_active, s_groups;
    __shared__ unsigned long long s_items, s_sweep;
    const uint32_t tid = threadIdx.x;
    const uint32_t nbins = 2 * (A.t_all + 1);
    mih::Control *ctrl = A.ctrl;
    const uint32_t n_old = ctrl->n_active;
    const uint32_t n_new = ctrl->n_new;
    const uint32_t Qi = A.quantum_items;
    uint32_t *last = bins + 2 * nbins;
    uint32_t *g_t = bins + 3 * nbins, *g_count = bins + 4 * nbins;
    uint32_t *g_ipq = bins + 5 * nbins, *g_steps = bins + 6 * nbins;
    for (uint32_t i = tid; i < 3 * nbins; i += 1024) bins[i] = 0;
    for (uint32_t i = tid; i < MIH_BINOM_N * MIH_BINOM_N; i += 1024)
        binom[i / MIH_BINOM_N][i % MIH_BINOM_N] = binom_calc(i / MIH_BINOM_N, i % MIH_BINOM_N);
    __syncthreads();
    // items of step t, and whether a query with `cur` of them done finishes
    // the step in this round
    auto items_of = [&](uint32_t t) {
        const uint32_t rp = t / A.m;
        const uint32_t M = binom[A.tables[t - rp * A.m].len][rp];
        return (M + A.chunk - 1) / A.chunk;
    };
    auto bin_of = [&](uint32_t t, uint32_t q) {
        const bool fin = Qi == 0 || A.cursor[q] + Qi >= items_of(t);
        return 2 * t + (fin ? 1u : 0u);
    };
    for (uint32_t i = tid; i < n_old; i += 1024) {
        const uint32_t nt = A.next_t[i];
        if (nt != 0xFFFFFFFFu) atomicAdd(&bins[bin_of(nt, A.active[i])], 1u);
    }
    for (uint32_t i = tid; i < n_new; i += 1024) atomicAdd(&bins[bin_of(0, A.new_slots[i])], 1u);
    __syncthreads();
    if (tid == 0) {
        uint32_t slot = 0, ng = 0;
        uint64_t items = 0, masks = 0;
        for (uint32_t b = 0; b < nbins; ++b) {
            uint32_t c = bins[b];
            bins[nbins + b] = slot;
            last[b] = b >> 1;
            if (!c) continue;
            const uint32_t t = b >> 1, fin = b & 1u;
            const uint32_t rp = t / A.m;
            const uint32_t s = A.tables[t - rp * A.m].len;
            const uint32_t M = binom[s][rp];
            const uint32_t it = (M + A.chunk - 1) / A.chunk;
            // many probes per bucket line: run the step partition by
            // partition (sweep kernel; no items of the round kernel); the
            // quantum cuts steps into portions of Qi items, the final one
            // holding what is left after the whole portions, and only steps
            // within one quantum are swept (a sweep runs a whole step)
            const bool sweep = A.sweep_shift != 0 && s >= mih::kSweepMinBits && (Qi == 0 || it <= Qi) &&
                               (uint64_t)c * M >= ((1ull << s) >> A.sweep_shift);
            uint32_t ipq = it;
            if (Qi) ipq = fin ? it - (it ? (it - 1) / Qi * Qi : 0u) : Qi;
            if (sweep) ipq = 0;
            g_t[ng] = t;
            g_count[ng] = c;
            g_ipq[ng] = ipq;
            g_steps[ng] = 1;
            A.groups[ng].step_items[0] = 0;
            A.groups[ng].step_items[1] = ipq;
            A.groups[ng].slot_start = slot;
            A.groups[ng].final = fin;
            ++ng;
            slot += c;
            items += (uint64_t)c * ipq;
            masks += (uint64_t)c * (sweep ? M : (uint64_t)ipq * A.chunk);
        }
        // lookahead: pass u offers step t + u to every group that finishes
        // its step and took all of its steps so far, while the round's items
        // and masks fit (and, under a quantum, while the step fits in one)
        for (uint32_t u = 1; u < A.look_max && items < A.look_items && masks < A.look_masks; ++u) {
            bool grew = false;
            for (uint32_t x = 0; x < ng; ++x) {
                if (g_ipq[x] == 0 || g_steps[x] != u || !A.groups[x].final) continue;
                const uint32_t tn = g_t[x] + u;
                if (tn > A.t_all) continue;
                const uint32_t rp = tn / A.m;
                const uint32_t M = binom[A.tables[tn - rp * A.m].len][rp];
                const uint32_t ni = (M + A.chunk - 1) / A.chunk;
                if (Qi && ni > Qi) continue;
                const uint64_t c = g_count[x];
                if (items + c * ni > A.look_items || masks + c * M > A.look_masks) continue;
                items += c * ni;
                masks += c * M;
                g_ipq[x] += ni;
                g_steps[x] = u + 1;
                A.groups[x].step_items[u + 1] = g_ipq[x];
                last[2 * g_t[x] + 1] = tn;
                grew = true;
            }
            if (!grew) break;
        }
        // the final groups and their item and sweep numbering
        items = 0;
        uint64_t sweep_items = 0;
        for (uint32_t x = 0; x < ng; ++x) {
            mih::Group &G = A.groups[x];
            G.t = g_t[x];
            G.count = g_count[x];
            G.ipq = g_ipq[x];
            G.steps = g_steps[x];
            G.item_start = items;
            G.sweep_start = sweep_items;
            items += (uint64_t)g_count[x] * g_ipq[x];
            G.sweep_bits = 0;
            G.sweep_qc = 0;
            if (g_ipq[x] == 0) {
                // at least kSweepXcds partitions: one share per XCD; the
                // partition kernel stages a partition's occupancy bits in LDS
                const uint32_t rp = g_t[x] / A.m;
                const uint32_t s = A.tables[g_t[x] - rp * A.m].len;
                const uint32_t Lmax = A.sweep_part ? A.part_bits : A.sweep_bits;
                const uint32_t L = Lmax < s - 3 ? Lmax : s - 3;
                const uint32_t qc = (g_count[x] + A.sweep_q - 1) / A.sweep_q;
                G.sweep_bits = L;
                G.sweep_qc = qc;
                sweep_items += ((1ull << (s - L)) / mih::kSweepXcds) * qc;   // per XCD
            }
        }
        s_active = slot;
        s_groups = ng;
        s_items = items;
        s_sweep = sweep_items;
    }
    __syncthreads();
    // a query whose group runs ahead resumes after the window's last step
    // (its cursor still counts the items of the window's first step, which
    // the round kernel needs; the window's later steps fit in one quantum,
    // so the advance kernel finds the last one finished whatever the cursor)
    for (uint32_t i = tid; i < n_old; i += 1024) {
        const uint32_t nt = A.next_t[i];
        if (nt != 0xFFFFFFFFu) {
            const uint32_t q = A.active[i];
            const uint32_t b = bin_of(nt, q);
            A.active_tmp[atomicAdd(&bins[nbins + b], 1u)] = q;
            if (last[b] != nt) A.t[q] = last[b];
        }
    }
    for (uint32_t i = tid; i < n_new; i += 1024) {
        const uint32_t q = A.new_slots[i];
        const uint32_t b = bin_of(0, q);
        A.active_tmp[atomicAdd(&bins[nbins + b], 1u)] = q;
        if (last[b] != 0) A.t[q] = last[b];
    }
    __syncthreads();
    const uint32_t total = s_active;
    for (uint32_t i = tid; i < total; i += 1024) A.active[i] = A.active_tmp[i];
    if (tid == 0) {
        ctrl->n_active = total;
        ctrl->n_groups = s_groups;
        ctrl->total_items = s_items;
        ctrl->sweep_items = s_sweep;
        ctrl->n_new = 0;
        ctrl->n_done = 0;
        ctrl->n_ovf = 0;
        *A.work = 0;
        for (uint32_t x = 0; x < mih::kSweepXcds; ++x) A.work_sweep[x] = 0;
        *A.spill_tail = 0;
        *A.spill_next = 0;
        A.ctrl->seq += 1;   // the pieces offered in earlier rounds no longer count
    }
}

// Admission: per-slot state of newly admitted queries (one thread each).
__global__ __launch_bounds__(MIH_BLOCK) void mih_admit_kernel(mih::MihArgs A, const mih::AdmitRec *rec,
                                                              uint32_t n)
{
    const uint32_t i = blockIdx.x * MIH_BLOCK + threadIdx.x;
    if (i == 0) A.ctrl->n_new = n;
    if (i >= n) return;
    const mih::AdmitRec r = rec[i];
    const uint32_t q = r.slot;
    const uint64_t *src = reinterpret_cast<const uint64_t *>(r.query);
    uint64_t *dst = const_cast<uint64_t *>(A.qb.queries) + (uint64_t)q * A.W;
    for (uint32_t w = 0; w < A.W; ++w) dst[w] = src[w];
    const_cast<uint32_t *>(A.qb.k)[q] = r.k;
    const_cast<uint32_t *>(A.qb.cap)[q] = r.cap;
    const_cast<uint64_t *>(A.qb.buf_off)[q] = r.buf_off;
    A.qb.tau[q] = r.tau0;
    A.qb.count[q] = 0;
    A.t[q] = 0;
    A.cursor[q] = 0;
    A.max_t[q] = r.max_t;
    A.budget[q] = r.budget;
    A.uniq[q] = 0;
    A.out_ids[q] = r.out_ids;
    A.out_dists[q] = r.out_dists;
    uint32_t *h = A.qb.hist + (uint64_t)q * (A.bits + 1);
    for (uint32_t d = 0; d <= A.bits; ++d) h[d] = 0;
    A.new_slots[i] = q;
}

// Which kernel: the round kernel, the sweep kernel, or the partition
// kernel (the sweep of tables with an occupancy map).
enum { K_ROUND = 0, K_SWEEP = 1, K_PART = 2, K_ROUND_SPILL = 3 };

// Kernel for (W, table mode, codes mode, J); J must be 4, 8 or 16.
template <int W, int TM, bool INLINE, int J>
const void *kernel_of(int which)
{
    if (which == K_PART) {
        if constexpr (TM == mih::TM_DIRECT || TM == mih::TM_HEADS)
            return reinterpret_cast<const void *>(&mih_part_kernel<W, TM, INLINE, J>);
        return nullptr;
    }
    return which == K_SWEEP ? reinterpret_cast<const void *>(&mih_sweep_kernel<W, TM, INLINE, J>)
           : which == K_ROUND_SPILL ? reinterpret_cast<const void *>(&mih_round_kernel<W, TM, INLINE, J, true>)
                                    : reinterpret_cast<const void *>(&mih_round_kernel<W, TM, INLINE, J, false>);
}

template <int W, int TM, bool INLINE>
const void *round_kernel_ptr(uint32_t J, int which)
{
    switch (J) {
    case 4: return kernel_of<W, TM, INLINE, 4>(which);
    case 8: return kernel_of<W, TM, INLINE, 8>(which);
    case 16: return kernel_of<W, TM, INLINE, 16>(which);
    default: return nullptr;
    }
}

template <int W>
const void *round_kernel_w(uint32_t tm, bool inline_codes, uint32_t J, int which)
{
    switch (tm) {
    case mih::TM_DIRECT:
        return inline_codes ? round_kernel_ptr<W, mih::TM_DIRECT, true>(J, which)
                            : round_kernel_ptr<W, mih::TM_DIRECT, false>(J, which);
    case mih::TM_SORTED:
        return inline_codes ? round_kernel_ptr<W, mih::TM_SORTED, true>(J, which)
                            : round_kernel_ptr<W, mih::TM_SORTED, false>(J, which);
    case mih::TM_GROUPED:   // the group scan reads the codes in table order
        return inline_codes ? round_kernel_ptr<W, mih::TM_GROUPED, true>(J, which) : nullptr;
    case mih::TM_HEADS:     // 64-bit codes in table order only
        if constexpr (W == 1) return inline_codes ? round_kernel_ptr<W, mih::TM_HEADS, true>(J, which) : nullptr;
        return nullptr;
    default: return nullptr;
    }
}

const void *round_kernel(uint32_t W, uint32_t tm, bool inline_codes, uint32_t J, int which = K_ROUND)
{
    switch (W) {
    case 1: return round_kernel_w<1>(tm, inline_codes, J, which);
    case 2: return round_kernel_w<2>(tm, inline_codes, J, which);
    case 3: return round_kernel_w<3>(tm, inline_codes, J, which);
    case 4: return round_kernel_w<4>(tm, inline_codes, J, which);
    default: return nullptr;
    }
}

// Dynamic LDS of the partition kernel: the occupancy bits of one partition.
size_t part_lds_bytes(uint32_t part_bits) { return ((size_t)1 << part_bits) / 8; }

}  // namespace

namespace mih {

bool mih_probes_per_lane_ok(uint32_t J) { return J == 4 || J == 8 || J == 16; }

hipError_t mih_round(const MihArgs &A, uint32_t grid, hipStream_t s)
{
    const void *k = round_kernel(A.W, A.tm, A.inline_codes, A.J, A.spill_min ? K_ROUND_SPILL : K_ROUND);
    if (!k) return hipErrorInvalidValue;
    void *args[] = {const_cast<MihArgs *>(&A)};
    return hipLaunchKernel(k, dim3(grid), dim3(MIH_BLOCK), args, 0, s);
}

hipError_t mih_sweep(const MihArgs &A, uint32_t grid, hipStream_t s)
{
    const void *k = round_kernel(A.W, A.tm, A.inline_codes, A.J, A.sweep_part ? K_PART : K_SWEEP);
    if (!k) return hipErrorInvalidValue;
    void *args[] = {const_cast<MihArgs *>(&A)};
    const size_t lds = A.sweep_part ? part_lds_bytes(A.part_bits) : 0;
    return hipLaunchKernel(k, dim3(grid), dim3(MIH_BLOCK), args, lds, s);
}

bool mih_part_kernel_ok(uint32_t W, uint32_t tm, bool inline_codes, uint32_t J)
{
    return round_kernel(W, tm, inline_codes, J, K_PART) != nullptr;
}

int mih_round_occupancy(uint32_t W, uint32_t tm, bool inline_codes, uint32_t J, int which,
                        uint32_t part_bits)
{
    const void *k = round_kernel(W, tm, inline_codes, J, which);
    const size_t lds = which == K_PART ? part_lds_bytes(part_bits) : 0;
    int blocks = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, MIH_BLOCK, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return blocks > 0 ? blocks : 1;
}

hipError_t mih_regroup(const MihArgs &A, hipStream_t s)
{
    const size_t lds = sizeof(uint32_t) * 7 * 2 * (A.t_all + 1);
    mih_regroup_kernel<<<1, 1024, lds, s>>>(A);
    return hipGetLastError();
}

hipError_t mih_advance(const MihArgs &A, uint32_t max_slots, hipStream_t s)
{
    if (max_slots == 0) return hipSuccess;
    mih_advance_kernel<<<(max_slots + MIH_BLOCK - 1) / MIH_BLOCK, MIH_BLOCK, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t mih_admit(const MihArgs &A, const AdmitRec *rec, uint32_t n, hipStream_t s)
{
    mih_admit_kernel<<<(n + MIH_BLOCK - 1) / MIH_BLOCK > 0 ? (n + MIH_BLOCK - 1) / MIH_BLOCK : 1,
                       MIH_BLOCK, 0, s>>>(A, rec, n);
    return hipGetLastError();
}

}  // namespace mih
