// Collection and ordered output of r-neighbour results.
#include <algorithm>

#include "rnn.h"

namespace {

__global__ __launch_bounds__(MIH_BLOCK) void gather_counts_kernel(const uint32_t *count,
                                                                  const uint32_t *list, uint32_t n,
                                                                  uint32_t *out)
{
    const uint32_t i = blockIdx.x * MIH_BLOCK + threadIdx.x;
    if (i < n) out[i] = count[list[i]];
}

// One workgroup per move: dst[m.dst + e] = src[m.src + e] for e < m.count.
__global__ __launch_bounds__(MIH_BLOCK) void rnn_move_kernel(const uint64_t *__restrict__ src,
                                                             uint64_t *__restrict__ dst,
                                                             const RnnMove *moves)
{
    const RnnMove mv = moves[blockIdx.x];
    for (uint32_t e = threadIdx.x; e < mv.count; e += MIH_BLOCK) dst[mv.dst + e] = src[mv.src + e];
}

// One workgroup per query: its entries (arena offset m.src) sorted in LDS
// and split into ids and distances at output offset m.dst.  Longer lists are
// split unsorted and sorted afterwards by the radix sort.
__global__ __launch_bounds__(MIH_BLOCK) void rnn_emit_kernel(const uint64_t *__restrict__ arena,
                                                             const RnnMove *moves,
                                                             uint32_t *__restrict__ ids,
                                                             uint32_t *__restrict__ dists)
{
    __shared__ uint64_t v[mih::kRnnLdsSort];
    const RnnMove mv = moves[blockIdx.x];
    const uint32_t tid = threadIdx.x;
    const uint64_t *in = arena + mv.src;
    if (mv.count > mih::kRnnLdsSort) {
        for (uint32_t e = tid; e < mv.count; e += MIH_BLOCK) {
            const uint64_t x = in[e];
            ids[mv.dst + e] = (uint32_t)x;
            dists[mv.dst + e] = (uint32_t)(x >> 32);
        }
        return;
    }
    if (mv.count == 0) return;
    uint32_t P = 1;
    while (P < mv.count) P <<= 1;
    for (uint32_t e = tid; e < P; e += MIH_BLOCK) v[e] = e < mv.count ? in[e] : ~0ull;
    __syncthreads();
    block_bitonic_sort(v, P);
    for (uint32_t e = tid; e < mv.count; e += MIH_BLOCK) {
        ids[mv.dst + e] = (uint32_t)v[e];
        dists[mv.dst + e] = (uint32_t)(v[e] >> 32);
    }
}

uint32_t bits_for(uint32_t v)
{
    uint32_t b = 0;
    while (b < 32 && (v >> b) != 0) ++b;
    return b;
}

}  // namespace

namespace mih {

void free_rnn_out(RnnOut &o)
{
    if (o.offsets) (void)hipFree(o.offsets);
    if (o.ids) (void)hipFree(o.ids);
    if (o.dists) (void)hipFree(o.dists);
    o = RnnOut();
}

hipError_t gather_counts(const uint32_t *count, const uint32_t *list, uint32_t n, uint32_t *out,
                         hipStream_t s)
{
    if (n == 0) return hipSuccess;
    gather_counts_kernel<<<(n + MIH_BLOCK - 1) / MIH_BLOCK, MIH_BLOCK, 0, s>>>(count, list, n, out);
    return hipGetLastError();
}

RnnCollector::~RnnCollector()
{
    if (arena_) (void)hipFree(arena_);
    if (moves_) (void)hipFree(moves_);
}

hipError_t RnnCollector::reserve(uint64_t entries, hipStream_t s)
{
    if (entries <= cap_) return hipSuccess;
    const uint64_t ncap = std::max<uint64_t>({entries, 2 * cap_, 4096});
    uint64_t *na = nullptr;
    hipError_t e = hipMalloc((void **)&na, ncap * 8);
    if (e != hipSuccess) return e;
    if (used_) e = hipMemcpyAsync(na, arena_, used_ * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { (void)hipFree(na); return e; }
    if (arena_) (void)hipFree(arena_);
    arena_ = na;
    cap_ = ncap;
    return hipSuccess;
}

hipError_t RnnCollector::moves_room(uint64_t n)
{
    if (n <= moves_cap_) return hipSuccess;
    if (moves_) { (void)hipFree(moves_); moves_ = nullptr; moves_cap_ = 0; }
    const uint64_t nc = std::max<uint64_t>(n, 1024);
    hipError_t e = hipMalloc((void **)&moves_, nc * sizeof(RnnMove));
    if (e == hipSuccess) moves_cap_ = nc;
    return e;
}

hipError_t RnnCollector::add(const uint64_t *src, const std::vector<uint32_t> &query,
                             const std::vector<uint64_t> &src_off, const std::vector<uint32_t> &count,
                             hipStream_t s)
{
    const size_t n = query.size();
    if (n == 0) return hipSuccess;
    uint64_t need = used_;
    for (size_t i = 0; i < n; ++i) need += count[i];
    hipError_t e = reserve(need, s);
    if (e != hipSuccess) return e;
    std::vector<RnnMove> mv;
    mv.reserve(n);
    for (size_t i = 0; i < n; ++i) {
        start_[query[i]] = used_;
        count_[query[i]] = count[i];
        if (count[i]) mv.push_back(RnnMove{src_off[i], used_, count[i], 0});
        used_ += count[i];
    }
    if (mv.empty()) return hipSuccess;
    if ((e = moves_room(mv.size())) != hipSuccess) return e;
    e = hipMemcpyAsync(moves_, mv.data(), mv.size() * sizeof(RnnMove), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    rnn_move_kernel<<<(uint32_t)mv.size(), MIH_BLOCK, 0, s>>>(src, arena_, moves_);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipStreamSynchronize(s);   // the host vector and the source buffers are reused next
}

hipError_t RnnCollector::finish(uint32_t bits, hipStream_t s, RnnOut &out)
{
    const uint32_t nq = (uint32_t)count_.size();
    out = RnnOut();
    out.nq = nq;
    std::vector<uint64_t> off(nq + 1, 0);
    for (uint32_t i = 0; i < nq; ++i) off[i + 1] = off[i] + count_[i];
    const uint64_t total = off[nq];
    out.total = total;
    hipError_t e = hipMalloc((void **)&out.offsets, (nq + 1) * 8ull);
    if (e == hipSuccess) e = hipMalloc((void **)&out.ids, std::max<uint64_t>(total, 1) * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&out.dists, std::max<uint64_t>(total, 1) * 4);
    if (e == hipSuccess) e = hipMemcpyAsync(out.offsets, off.data(), (nq + 1) * 8ull, hipMemcpyHostToDevice, s);
    std::vector<RnnMove> mv;
    uint64_t longest = 0;
    for (uint32_t i = 0; i < nq; ++i) {
        if (count_[i] == 0) continue;
        mv.push_back(RnnMove{start_[i], off[i], count_[i], 0});
        if (count_[i] > kRnnLdsSort) longest = std::max<uint64_t>(longest, count_[i]);
    }
    if (e == hipSuccess && !mv.empty()) {
        if ((e = moves_room(mv.size())) == hipSuccess)
            e = hipMemcpyAsync(moves_, mv.data(), mv.size() * sizeof(RnnMove), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) {
            rnn_emit_kernel<<<(uint32_t)mv.size(), MIH_BLOCK, 0, s>>>(arena_, moves_, out.ids, out.dists);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // mv is read by the copy above
    if (e == hipSuccess && longest) {
        // long lists: stable sort by id, then stable sort by distance
        uint32_t *k2 = nullptr, *v2 = nullptr, *tmp = nullptr;
        e = hipMalloc((void **)&k2, longest * 4);
        if (e == hipSuccess) e = hipMalloc((void **)&v2, longest * 4);
        if (e == hipSuccess) e = hipMalloc((void **)&tmp, radix_tmp_words(longest) * 4);
        for (uint32_t i = 0; i < nq && e == hipSuccess; ++i) {
            if (count_[i] <= kRnnLdsSort) continue;
            const uint64_t c = count_[i];
            uint32_t *ids = out.ids + off[i], *ds = out.dists + off[i];
            uint32_t *a = ids, *b = ds, *a2 = k2, *b2 = v2;
            e = radix_sort_pairs(a, b, a2, b2, c, 32, tmp, s);
            // (a, b) = (ids, dists) sorted by id; now by distance, ids riding along
            uint32_t *x = b, *y = a, *x2 = b2, *y2 = a2;
            if (e == hipSuccess) e = radix_sort_pairs(x, y, x2, y2, c, bits_for(bits), tmp, s);
            if (e == hipSuccess && y != ids) e = hipMemcpyAsync(ids, y, c * 4, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess && x != ds) e = hipMemcpyAsync(ds, x, c * 4, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
        }
        if (k2) (void)hipFree(k2);
        if (v2) (void)hipFree(v2);
        if (tmp) (void)hipFree(tmp);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_rnn_out(out);
        return e;
    }
    if (arena_) (void)hipFree(arena_);
    arena_ = nullptr;
    cap_ = used_ = 0;
    return hipSuccess;
}

}  // namespace mih
