// nsg_search_noalloc: nsg_search for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops).  Its one piece
// of scratch memory, the persistent grid's work counter, lives in a
// file-scope device array (one copy per device, kept until the process ends)
// instead of a library allocation; the kernels are nsg_search's.
#include "common.hpp"

#include <mutex>

// kScratchWords 32-bit words per device; the search uses word 0 (the work
// counter of the persistent grid), whatever the batch size.
constexpr int kScratchWords = 64;
static __device__ __align__(256) unsigned int scratch[kScratchWords];

namespace nsg {

constexpr int kMaxDevices = 64;
constexpr int64_t kNoallocPersistentMin = 4096;   // same batch-size rule as nsg_search

// Device address of this device's `scratch`, looked up once per device with
// that device current (each GPU holds its own copy at its own address; the
// array's name in host code is only a host-side stand-in).
static int scratch_ptr(unsigned int **out) {
    static std::mutex mu;
    static unsigned int *ptrs[kMaxDevices] = {};
    int dev = 0;
    NSG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(NSG_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(mu);
    if (!ptrs[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(NSG_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        ptrs[dev] = static_cast<unsigned int *>(p);
    }
    *out = ptrs[dev];
    return NSG_OK;
}

}  // namespace nsg

using namespace nsg;

extern "C" int nsg_search_noalloc(const nsg_index *idx, const float *queries, int64_t nq, int32_t k, int32_t L,
                                  uint32_t *out_ids, float *out_dist, void *stream) {
    clear_error();
    if (!idx) return fail(NSG_EINVAL, "index is NULL");
    if (nq < 0 || nq >= ((int64_t)1 << 31)) return fail(NSG_EINVAL, "nq=%lld out of range [0, 2^31)", (long long)nq);
    if (k < 1 || k > kMaxK) return fail(NSG_EINVAL, "k=%d out of range [1, %d]", k, kMaxK);
    if (L < 1 || L > kMaxL) return fail(NSG_EINVAL, "L=%d out of range [1, %d]", L, kMaxL);
    if (nq == 0) return NSG_OK;
    if (!queries || !out_ids || !out_dist) return fail(NSG_EINVAL, "NULL query or output pointer");
    SearchArgs a{};
    a.idx = idx;
    a.queries = queries;
    a.nq = nq;
    a.k_scalar = k;
    a.L_scalar = L;
    a.out_stride = k;
    a.out_ids = out_ids;
    a.out_dist = out_dist;
    a.learned = idx->stop.enabled && idx->stop.blob && L >= 16;
    a.L_cap = L;
    a.hash_bits = default_hash_bits(L);
    a.rerank = idx->storage != NSG_F32;
    a.persistent = nq >= kNoallocPersistentMin;
    if (a.persistent) {
        // the counter is cleared by a kernel at the start of every call
        int rc = scratch_ptr(&a.counter);
        if (rc) return rc;
    }
    a.start_override = NSG_SENT;
    a.self_offset = -1;
    a.stream = (hipStream_t)stream;
    return launch_search(a);
}
