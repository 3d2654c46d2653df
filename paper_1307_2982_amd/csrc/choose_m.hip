// Choosing the number of substrings m (Section 3.1 and Section 6, "Number
// of Substrings").
//
// The analytic side is the cost model of Eq. 6 for uniformly distributed
// codes: per table of s bits, the buckets within substring radius
// floor(s r / b) are looked up and each holds n / 2^s codes on average, and
// a lookup costs about as much as a candidate test.  With unequal substring
// lengths (b not divisible by m) the per-table terms are summed, which is
// Eq. 6 exactly when every table has s = b / m bits.  The radius r of a
// kNN query is modelled as the smallest r at which the expected number of
// uniform codes within distance r, n L(b, r) / 2^b, reaches k.
//
// The empirical side follows the paper's procedure: candidate values of m
// near b / log2 n (plus the model's own minimum) are each built and timed on
// a validation set of queries, and the fastest is selected.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include <hip/hip_runtime.h>

#include "mih.h"

namespace {

double binom(uint32_t n, uint32_t k)
{
    if (k > n) return 0.0;
    double r = 1.0;
    for (uint32_t i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

bool m_ok(uint32_t bits, uint32_t m)
{
    return m >= 1 && m <= MIH_M_MAX && m <= bits && (bits + m - 1) / m <= MIH_SUBSTRING_MAX;
}

}  // namespace

extern "C" {

double mih_model_cost(uint64_t n, uint32_t bits, uint32_t m, uint32_t r)
{
    if (bits == 0 || m == 0 || m > bits) return 0.0;
    const uint32_t base = bits / m, extra = bits % m;
    double total = 0.0;
    for (uint32_t j = 0; j < m; ++j) {
        const uint32_t s = base + (j < extra ? 1u : 0u);
        const uint32_t zmax = (uint32_t)(((uint64_t)s * r) / bits);
        double lookups = 0.0;
        for (uint32_t z = 0; z <= std::min(zmax, s); ++z) lookups += binom(s, z);
        total += (1.0 + (double)n / std::ldexp(1.0, (int)s)) * lookups;
    }
    return total;
}

uint32_t mih_model_radius(uint64_t n, uint32_t bits, uint32_t k)
{
    // expected codes within distance r: n L(bits, r) / 2^bits; the test
    // n L >= k 2^bits is made on the lower sum L while it is the smaller
    // part of 2^bits, and as (n - k) 2^bits >= n T on the upper tail
    // T = 2^bits - L beyond, so neither side loses its low-order terms
    if (k == 0) return 0;
    if ((uint64_t)k >= n) return bits;   // k = n needs every code; k > n cannot be met
    std::vector<double> tail(bits + 2, 0.0);   // tail[r] = sum_{z >= r} C(bits, z)
    for (uint32_t z = bits + 1; z-- > 0;) tail[z] = tail[z + 1] + binom(bits, z);
    double low = 0.0;
    for (uint32_t r = 0; r <= bits; ++r) {
        low += binom(bits, r);
        const double up = tail[r + 1];
        const bool ok = low <= up ? (double)n * std::ldexp(low, -(int)bits) >= (double)k
                                  : (double)(n - k) >= (double)n * std::ldexp(up, -(int)bits);
        if (ok) return r;
    }
    return bits;
}

mih_status mih_choose_m(const uint64_t *codes, uint64_t n, uint32_t bits, const uint64_t *queries,
                        uint32_t nq, uint32_t k, const uint32_t *candidates, uint32_t ncand,
                        const mih_build_opts *opts, void *stream, uint32_t *best_m,
                        mih_m_trial *trials, uint32_t *ntrials)
{
    if (!best_m || !ntrials) return MIH_ERR_INVALID;
    if (bits == 0 || bits % 64 != 0 || bits > 256) return MIH_ERR_INVALID;
    if (n < 2 || !codes || nq == 0 || !queries || k == 0 || k > MIH_K_MAX) return MIH_ERR_INVALID;
    if (ncand > MIH_M_TRIALS_MAX || (ncand && !candidates)) return MIH_ERR_INVALID;
    std::vector<uint32_t> cand;
    const uint32_t r = mih_model_radius(n, bits, k);
    if (ncand) {
        for (uint32_t i = 0; i < ncand; ++i)
            if (!m_ok(bits, candidates[i])) return MIH_ERR_INVALID;
        cand.assign(candidates, candidates + ncand);
    } else {
        // around the heuristic b / log2 n, plus the model's minimum
        const long c = std::lround((double)bits / std::log2((double)n));
        for (long m = c - 1; m <= c + 1; ++m)
            if (m >= 1 && m_ok(bits, (uint32_t)m)) cand.push_back((uint32_t)m);
        uint32_t arg = 0;
        double best = 0.0;
        for (uint32_t m = 1; m <= std::min<uint32_t>(bits, MIH_M_MAX); ++m) {
            if (!m_ok(bits, m)) continue;
            const double c6 = mih_model_cost(n, bits, m, r);
            if (arg == 0 || c6 < best) { arg = m; best = c6; }
        }
        if (arg) cand.push_back(arg);
        if (cand.empty()) return MIH_ERR_UNSUPPORTED;
    }
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    if (cand.size() > MIH_M_TRIALS_MAX) cand.resize(MIH_M_TRIALS_MAX);

    uint32_t *out = nullptr;
    if (hipMalloc((void **)&out, 2ull * nq * k * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return MIH_ERR_NOMEM;
    }
    uint32_t nt = 0, best = 0;
    double best_ms = 0.0;
    mih_status last_err = MIH_ERR_UNSUPPORTED;
    for (uint32_t m : cand) {
        mih_m_trial t;
        std::memset(&t, 0, sizeof(t));
        t.m = m;
        t.model_cost = mih_model_cost(n, bits, m, r);
        mih_index *ix = nullptr;
        t.status = mih_build(codes, n, bits, m, opts, stream, &ix);
        if (t.status == MIH_OK) {
            mih_index_info info;
            mih_index_get_info(ix, &info);
            t.build_ms = info.build_ms;
            t.device_bytes = info.device_bytes;
            // one call to warm the engine, one timed
            t.status = mih_knn(ix, queries, nq, k, nullptr, out, out + (uint64_t)nq * k, stream);
            mih_query_stats st;
            if (t.status == MIH_OK)
                t.status = mih_knn_ex(ix, queries, nq, k, nullptr, out, out + (uint64_t)nq * k, stream, &st);
            if (t.status == MIH_OK) t.search_ms = st.elapsed_ms;
            mih_free(ix);
        }
        if (t.status == MIH_OK && (best == 0 || t.search_ms < best_ms)) { best = m; best_ms = t.search_ms; }
        if (t.status != MIH_OK) last_err = t.status;
        if (trials) trials[nt] = t;
        ++nt;
    }
    (void)hipFree(out);
    *ntrials = nt;
    *best_m = best;
    return best ? MIH_OK : last_err;
}

}  // extern "C"
