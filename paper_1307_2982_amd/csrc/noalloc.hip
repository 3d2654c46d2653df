// linscan_knn_noalloc: the linear-scan kNN of linscan_knn with every device
// buffer taken from one fixed, file-scope device array instead of hipMalloc,
// for callers that cannot allocate device memory (code under stream capture,
// tight serving loops, harnesses that forbid it).
//
// The array lives in this file's code object, so a process holds it on a
// GPU only once this entry point has run there, and then until the process
// ends.  Host code never passes the array's name to a kernel or a copy (in
// host code it names a host-side stand-in): its device address is looked up
// once per device with hipGetSymbolAddress, with that device current, and
// only that address is used.  Every call on a GPU shares that GPU's array and
// re-initialises what it reads (counters and histograms are cleared by a
// fill kernel at the start of each pass), so calls that overlap on one GPU
// race and must be serialised by the caller.
#include <mutex>

#include "mih_common.h"

namespace {

static __device__ __align__(256) unsigned char scratch[MIH_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_dev[kMaxDevices];   // device address of `scratch` on each device, once looked up

// Device address of this device's copy of the array.
hipError_t scratch_address(char **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || ((uintptr_t)p & 255) != 0) return hipErrorInvalidSymbol;
        scratch_dev[dev] = p;
    }
    *out = static_cast<char *>(scratch_dev[dev]);
    return hipSuccess;
}

}  // namespace

extern "C" mih_status linscan_knn_noalloc(const uint64_t *codes, uint64_t n, uint32_t bits,
                                          const uint64_t *queries, uint32_t nq, uint32_t k,
                                          const uint32_t *k_per_query, uint32_t *out_ids,
                                          uint32_t *out_dists, void *stream)
{
    const mih_status st = mih::linscan_check_args(codes, n, bits, queries, nq, k, k_per_query, out_ids,
                                                  out_dists);
    if (st != MIH_OK) return st;
    char *base = nullptr;
    if (scratch_address(&base) != hipSuccess) {
        (void)hipGetLastError();
        return MIH_ERR_DEVICE;
    }
    return mih::linscan_knn_in_region(codes, n, bits, queries, nq, k, k_per_query, out_ids, out_dists,
                                      (hipStream_t)stream, base, MIH_NOALLOC_SCRATCH_BYTES);
}
