// The one-launch search of a small batch of queries (Algorithm 3 with every
// step run on the device, no host round trip between steps).
#include "mih_step.h"
#include "topk_dev.h"

namespace {

// One launch for a small batch: every query is taken by G workgroups (more
// for a query with more expected work), which run all its steps (Algorithm
// 3) on the device with no host round trip and no regroup between steps.  Steps go in windows: a window is one step, or
// consecutive steps whose masks together fill at most one pass of the
// query's waves.  Each workgroup takes its share of every window
// (contiguous ranges of masks, one per wave), in step order; the workgroup
// that finishes a window last (a counter per query and step) knows that
// steps 0 .. tw are complete, tests termination (Proposition 2) and, if the
// query is done, raises its stop flag.  The others do not wait for that test:
// they go on with the next window and leave at the next window boundary
// once the flag is up.  Steps they run ahead of the decision only add codes
// farther than the stop step, which is the engine's lookahead and changes
// no result.  A workgroup runs at most one window ahead of the completed
// ones (a bounded wait at each window; past the bound it goes on).  The
// workgroup that leaves last writes the top-k rows (or lists the query for
// an exact re-run when its candidate buffer overflowed).  This is for batches too
// small to fill the device with rounds, where the latency of the rounds,
// not the number of probes, sets the time.
template <int J>
constexpr uint32_t small_waves() { return J >= 16 ? 4 : (J >= 8 ? 8 : 16); }   // LDS staging per wave
// Most polls of a workgroup waiting for a step of its query to complete
// (each a device-scope load and a short sleep: a few milliseconds at most).
constexpr uint32_t kSmallPolls = 4096;

template <int W, int TM, bool INLINE, int J>
__global__ __launch_bounds__(small_waves<J>() * MIH_WAVE) void mih_small_kernel(
    mih::MihArgs A, mih::SmallArgs S)
{
    constexpr uint32_t kW = small_waves<J>(), kThreads = kW * MIH_WAVE;
    __shared__ uint32_t binom[MIH_BINOM_N][MIH_BINOM_N];
    // the staging of the search and the top-k of the last workgroup share LDS
    struct Stage {
        uint32_t pos[kW][MIH_WAVE * J];
        uint32_t cum[kW][MIH_WAVE * J];
        uint64_t code[kW][TM == mih::TM_HEADS ? MIH_WAVE * J : 1];
    };
    __shared__ union {
        Stage st;
        FinalizeLds fin;
    } U;
    uint32_t (&stage_pos)[kW][MIH_WAVE * J] = U.st.pos;
    uint32_t (&stage_cum)[kW][MIH_WAVE * J] = U.st.cum;
    auto &stage_code = U.st.code;
    __shared__ uint32_t s_flag;
    const uint32_t tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (uint32_t i = tid; i < MIH_BINOM_N * MIH_BINOM_N; i += kThreads)
        binom[i / MIH_BINOM_N][i % MIH_BINOM_N] = binom_calc(i / MIH_BINOM_N, i % MIH_BINOM_N);
    __syncthreads();
    WaveStats ws = {0, 0};
    const uint32_t q = S.query_of[blockIdx.x];
    const uint32_t g = blockIdx.x - S.first[q], G = S.first[q + 1] - S.first[q];
    if (A.qb.k[q] != 0) {
        uint32_t *step_cnt = S.step_cnt + (uint64_t)q * (A.t_all + 1);
        // masks of one pass of all the query's waves: small steps run
        // together in windows of at most one pass
        const uint32_t pass = MIH_WAVE * J, cap = G * kW * pass;
        auto masks_of = [&](uint32_t u) {
            const uint32_t r = u / A.m;
            return binom[A.tables[u - r * A.m].len][r];   // 0 when r' > s: the step covers radius u all the same
        };
        // expected candidates of a step (uniform codes: n / 2^s per bucket, at
        // least one): a window keeps them to a quarter of the query's buffer,
        // since the bound tau only falls once k codes have been found
        auto cands_of = [&](uint32_t u) {
            const uint32_t len = A.tables[u % A.m].len;
            const uint64_t per = len >= 64 ? 0 : A.n >> len;
            return (uint64_t)masks_of(u) * (per > 1 ? per : 1);
        };
        const uint64_t cand_cap = A.qb.cap[q] / 4;
        constexpr uint32_t kNone = 0xFFFFFFFFu;
        for (uint32_t t = 0, prev_tw = kNone, prev2_tw = kNone;;) {
            // the window t .. tw: every step up to a pass of masks in all (at
            // least step t), the same for every workgroup of the query
            uint32_t tw = t, total = masks_of(t);
            uint64_t cands = cands_of(t);
            while (tw < A.t_all && total + masks_of(tw + 1) <= cap && cands + cands_of(tw + 1) <= cand_cap) {
                ++tw;
                total += masks_of(tw);
                cands += cands_of(tw);
            }
            // A workgroup runs at most one window ahead of the completed
            // ones: before a window it waits, a bounded number of polls, for
            // the window before the previous one to complete (or the query to
            // stop), and before a window larger than one pass of the query's
            // waves for the previous one.  Without it, workgroups with no
            // share of the small early windows would run far ahead, into
            // steps past the stop, with the bound still loose.  Past the
            // bound a workgroup goes on, which is only speculation.
            const uint32_t need = total > cap ? prev_tw : prev2_tw;
            if (need != kNone) {
                if (tid == 0) {
                    for (uint32_t i = 0; i < kSmallPolls; ++i) {
                        if (load_relaxed(step_cnt + need) >= G || load_relaxed(S.stop + q) != kNone) break;
                        __builtin_amdgcn_s_sleep(8);
                    }
                }
                __syncthreads();
            }
            // the query's stop flag, seen at every window boundary
            if (tid == 0) s_flag = load_relaxed(S.stop + q);
            __syncthreads();
            const bool stopped = s_flag != kNone;
            __syncthreads();   // s_flag is rewritten below
            if (stopped) break;
            // contiguous ranges of whole passes over the window's masks, one per wave
            const uint32_t per = ((total + G * kW - 1) / (G * kW) + pass - 1) / pass * pass;
            const uint32_t rb = (g * kW + wave) * per;
            const uint32_t re = rb + per < total ? rb + per : total;
            uint32_t base = 0;
            for (uint32_t u = t; u <= tw && base < re; ++u) {
                const uint32_t M = masks_of(u);
                const uint32_t lo = rb > base ? rb - base : 0u, hi = re - base < M ? re - base : M;
                if (lo < hi) {
                    const uint32_t rp = u / A.m, a = u - rp * A.m;
                    uint64_t gq[W];
                    process_step<W, TM, INLINE, J>(A, q, u, query_key<W>(A, q, a, gq), A.tables[a].len, rp, lo, hi,
                                                   binom, stage_pos[wave], stage_cum[wave], stage_code[wave], ws);
                }
                base += M;
            }
            __syncthreads();   // this workgroup's share of the window is done
            if (tid == 0) {
                __threadfence();   // its candidates and counts before the step count
                s_flag = atomicAdd(step_cnt + tw, 1u) + 1 == G ? 1u : 0u;
                __threadfence();
            }
            __syncthreads();
            const bool last = s_flag != 0;
            __syncthreads();
            if (last) {
                // every workgroup has finished steps 0 .. tw: every code within
                // distance tw has been found.  Algorithm 3 stops after step
                // tau when tau <= tw (no earlier window reached tau), or
                // after the last step
                if (wave == 0) {
                    uint32_t tau = __builtin_amdgcn_readfirstlane(load_relaxed(A.qb.tau + q));
                    tau = tighten_tau(A.qb, q, tau);
                    uint32_t stop = 0xFFFFFFFFu;
                    if (tau <= tw) stop = tau > t ? tau : t;
                    else if (tw >= A.t_all) stop = tw;
                    if (lane == 0) s_flag = stop;
                }
                __syncthreads();
                const uint32_t stop = s_flag;
                if (stop != 0xFFFFFFFFu && tid == 0) atomicMin(S.stop + q, stop);
                __syncthreads();
                if (stop != 0xFFFFFFFFu) break;
            } else if (tw >= A.t_all) {
                break;   // the last step: its last finisher raises the flag
            }
            prev2_tw = prev_tw;
            prev_tw = tw;
            t = tw + 1;
        }
        // the workgroup that leaves last writes the rows
        if (tid == 0) {
            __threadfence();
            s_flag = atomicAdd(S.exits + q, 1u) + 1 == G ? 1u : 0u;
            __threadfence();
        }
        __syncthreads();
        if (s_flag) {
            const uint32_t cnt = load_relaxed(A.qb.count + q);
            if (tid == 0) {
                atomicAdd(&A.stats[2], (unsigned long long)load_relaxed(S.stop + q) + 1);   // steps
                atomicAdd(&A.stats[3], (unsigned long long)cnt);                            // appended
            }
            if (cnt > A.qb.cap[q]) {
                if (tid == 0) S.ovf_list[atomicAdd(S.ovf_count, 1u)] = q;
            } else {
                finalize_one(A.qb, q, S.out_ids + S.row_off[q], S.out_dists + S.row_off[q], U.fin);
            }
        }
    }
    if (lane == 0) {
        atomicAdd(&A.stats[0], (unsigned long long)ws.probes);
        atomicAdd(&A.stats[1], (unsigned long long)ws.candidates);
    }
}

template <int W, int TM, bool INLINE>
const void *small_kernel_j(uint32_t J)
{
    switch (J) {
    case 4: return reinterpret_cast<const void *>(&mih_small_kernel<W, TM, INLINE, 4>);
    case 8: return reinterpret_cast<const void *>(&mih_small_kernel<W, TM, INLINE, 8>);
    case 16: return reinterpret_cast<const void *>(&mih_small_kernel<W, TM, INLINE, 16>);
    default: return nullptr;
    }
}

template <int W>
const void *small_kernel_w(uint32_t tm, bool inline_codes, uint32_t J)
{
    switch (tm) {
    case mih::TM_DIRECT:
        return inline_codes ? small_kernel_j<W, mih::TM_DIRECT, true>(J) : small_kernel_j<W, mih::TM_DIRECT, false>(J);
    case mih::TM_SORTED:
        return inline_codes ? small_kernel_j<W, mih::TM_SORTED, true>(J) : small_kernel_j<W, mih::TM_SORTED, false>(J);
    case mih::TM_GROUPED:   // the group scan reads the codes in table order
        return inline_codes ? small_kernel_j<W, mih::TM_GROUPED, true>(J) : nullptr;
    case mih::TM_HEADS:     // 64-bit codes in table order only
        if constexpr (W == 1) return inline_codes ? small_kernel_j<W, mih::TM_HEADS, true>(J) : nullptr;
        return nullptr;
    default: return nullptr;
    }
}

const void *small_kernel(uint32_t W, uint32_t tm, bool inline_codes, uint32_t J)
{
    switch (W) {
    case 1: return small_kernel_w<1>(tm, inline_codes, J);
    case 2: return small_kernel_w<2>(tm, inline_codes, J);
    case 3: return small_kernel_w<3>(tm, inline_codes, J);
    case 4: return small_kernel_w<4>(tm, inline_codes, J);
    default: return nullptr;
    }
}

uint32_t small_block(uint32_t J) { return (J >= 16 ? 4u : (J >= 8 ? 8u : 16u)) * MIH_WAVE; }   // small_waves<J>()

}  // namespace

namespace mih {

hipError_t mih_small(const MihArgs &A, const SmallArgs &S, hipStream_t s)
{
    const void *k = small_kernel(A.W, A.tm, A.inline_codes, A.J);
    if (!k) return hipErrorInvalidValue;
    MihArgs a = A;
    SmallArgs b = S;
    void *args[] = {&a, &b};
    return hipLaunchKernel(k, dim3(S.blocks), dim3(small_block(A.J)), args, 0, s);
}

int mih_small_occupancy(uint32_t W, uint32_t tm, bool inline_codes, uint32_t J)
{
    const void *k = small_kernel(W, tm, inline_codes, J);
    int blocks = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, (int)small_block(J), 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return blocks > 0 ? blocks : 1;
}

}  // namespace mih
