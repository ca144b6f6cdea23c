// Approximate kNN graph by an inverted file, on the GPU.  The kNN graph is
// step (i) of the index build and the paper leaves it replaceable: nn-descent
// on the CPU for the million-scale sets, Faiss on the GPU for DEEP100M
// (Sec. 3.5, indexing complexity).  This is the inverted-file form, built on
// the library's own brute force (matrix cores):
//  1. cells: the nlist pivot points base[pivots[c]]; every point's nprobe
//     nearest pivots by (FP32 squared distance, c) (brute force of the points
//     against the pivots); a point's cell is its nearest pivot
//  2. the members of every cell in id order, and the points probing every
//     cell in id order (radix sort of (cell, id) keys)
//  3. cell by cell: the brute force of the probing points against the
//     members (K + 1 nearest, the point itself dropped), merged into each
//     probing point's running top K (one wave per point, a rank merge of two
//     sorted lists in LDS).  Cells have disjoint members, so a point meets
//     every candidate once, and the result is the exact top K by (FP32
//     squared distance, id) among the members of its probed cells.
#include "common.hpp"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

namespace nsg {
// the brute force on scratch the caller owns (defined beside
// nsg_knn_bruteforce): its scratch bytes for these operands, and the call
int bf_scratch_bytes(const float *base, int64_t n, const float *queries, int64_t nq, int d, int k, size_t *bytes);
int bf_with_scratch(const float *base, int64_t n, const float *queries, int64_t nq, int d, int k, int exclude_self,
                    uint32_t *out_ids, float *out_dist, void *scratch, size_t scratch_bytes, hipStream_t st);
}  // namespace nsg

namespace nsg {

// rows ids[b] of src[.][d] -> out[b][d] (one block per row)
__global__ void ivf_gather_kernel(const float *src, int d, const uint32_t *ids, float *out) {
    const int64_t b = blockIdx.x;
    const float *s = src + (int64_t)ids[b] * d;
    for (int j = threadIdx.x; j < d; j += blockDim.x) out[b * d + j] = s[j];
}

// (cell << 32 | i) for every point and (probed cell << 32 | i) for every probe
__global__ void ivf_keys_kernel(const uint32_t *probe, int64_t n, int nprobe, uint64_t *cell_keys,
                                uint64_t *probe_keys) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n * nprobe;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / nprobe;
        const uint64_t key = ((uint64_t)probe[t] << 32) | (uint64_t)i;
        probe_keys[t] = key;
        if (t % nprobe == 0) cell_keys[i] = key;
    }
}

// per-cell counts of sorted keys, and the ids (low halves) in key order
__global__ void ivf_split_kernel(const uint64_t *keys, int64_t m, int nlist, int64_t *count, uint32_t *ids) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[t];
        const uint32_t c = (uint32_t)(k >> 32);
        if (c < (uint32_t)nlist) atomicAdd(reinterpret_cast<unsigned long long *>(count + c), 1ull);
        ids[t] = (uint32_t)(k & 0xFFFFFFFFu);
    }
}

__global__ void ivf_fill_kernel(uint64_t *p, int64_t m, uint64_t v) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = v;
}

// One wave per probing point j of a cell: its K + 1 candidates (local member
// indices, sorted by distance then index, i.e. by (distance, global id) as
// members are in id order) mapped to global ids, itself dropped, merged with
// its running list lists[i][0 .. K) (sorted keys (distance bits << 32 | id),
// ~0 empty).  The two lists share no id (cells have disjoint members), so
// every key's output rank is its own index plus the count of smaller keys in
// the other list.
__global__ void __launch_bounds__(256) ivf_merge_kernel(const uint32_t *qids, int64_t nq, const uint32_t *member,
                                                        const uint32_t *cand, const float *cdist, int kc,
                                                        uint64_t *lists, int K) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * (blockDim.x >> 6) + w;
    const int stride = 2 * K + 2;
    uint64_t *a = reinterpret_cast<uint64_t *>(smem) + (size_t)w * stride;   // running list, K
    uint64_t *b = a + K;                                                      // candidates, <= K + 1
    if (j >= nq) return;
    const uint32_t i = qids[j];
    uint64_t *Li = lists + (int64_t)i * K;
    for (int t = lane; t < K; t += 64) a[t] = Li[t];
    // candidates without the point itself, in order (a ballot compaction)
    int nb = 0;
    for (int t0 = 0; t0 < kc; t0 += 64) {
        const int t = t0 + lane;
        uint64_t key = ~0ull;
        bool ok = false;
        if (t < kc) {
            const uint32_t loc = cand[j * kc + t];
            if (loc != NSG_SENT) {
                const uint32_t g = member[loc];
                if (g != i) {
                    key = ((uint64_t)__float_as_uint(cdist[j * kc + t]) << 32) | g;
                    ok = true;
                }
            }
        }
        const uint64_t m = __ballot(ok);
        if (ok) b[nb + __popcll(m & ((1ull << lane) - 1ull))] = key;
        nb += __popcll(m);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (nb == 0) return;
    // ranks: a[p] goes to p + #{b < a[p]}, b[q] to q + #{a < b[q]}
    uint64_t out_v[3];
    int out_r[3], cnt = 0;
    for (int p = lane; p < K; p += 64) {
        const uint64_t v = a[p];
        int lo = 0, hi = nb;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (b[mid] < v) lo = mid + 1; else hi = mid;
        }
        out_v[cnt] = v;
        out_r[cnt++] = p + lo;
    }
    uint64_t bv[3];
    int br[3], bc = 0;
    for (int q = lane; q < nb; q += 64) {
        const uint64_t v = b[q];
        int lo = 0, hi = K;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (a[mid] < v) lo = mid + 1; else hi = mid;
        }
        bv[bc] = v;
        br[bc++] = q + lo;
    }
    for (int t = 0; t < cnt; ++t)
        if (out_r[t] < K) Li[out_r[t]] = out_v[t];
    for (int t = 0; t < bc; ++t)
        if (br[t] < K) Li[br[t]] = bv[t];
}

__global__ void ivf_out_kernel(const uint64_t *lists, int64_t m, uint32_t *ids, float *dist) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t v = lists[t];
        const bool ok = v != ~0ull;
        ids[t] = ok ? (uint32_t)(v & 0xFFFFFFFFu) : NSG_SENT;
        dist[t] = ok ? __uint_as_float((uint32_t)(v >> 32)) : INFINITY;
    }
}

static unsigned grid_of(int64_t m) { return (unsigned)std::min<int64_t>((m + 255) / 256, 65535); }

}  // namespace nsg

using namespace nsg;

extern "C" int nsg_knn_ivf(const float *base, int64_t n, int32_t d, const uint32_t *pivots, int32_t nlist,
                           int32_t nprobe, int32_t K, uint32_t *out_ids, float *out_dist, void *stream) {
    clear_error();
    if (!base || !pivots || !out_ids || !out_dist) return fail(NSG_EINVAL, "NULL pointer");
    if (n < 2 || n >= ((int64_t)1 << 31)) return fail(NSG_EINVAL, "n out of range");
    if (d < 1 || d > 65536) return fail(NSG_EINVAL, "d out of range");
    if (nlist < 1 || nlist > n) return fail(NSG_EINVAL, "nlist=%d out of range [1, n]", nlist);
    if (nprobe < 1 || nprobe > nlist || nprobe > 160)
        return fail(NSG_EINVAL, "nprobe=%d out of range [1, min(nlist, 160)]", nprobe);
    if (K < 1 || K > 159) return fail(NSG_EINVAL, "K=%d out of range [1, 159]", K);
    hipStream_t st = (hipStream_t)stream;
    std::vector<uint32_t> hp((size_t)nlist);
    NSG_HIP(hipMemcpyAsync(hp.data(), pivots, 4 * (size_t)nlist, hipMemcpyDeviceToHost, st));
    NSG_HIP(hipStreamSynchronize(st));
    for (int c = 0; c < nlist; ++c)
        if ((int64_t)hp[c] >= n) return fail(NSG_EINVAL, "pivot %d is id %u >= n", c, hp[c]);

    std::vector<void *> bufs;
    struct Guard {
        std::vector<void *> &b;
        ~Guard() {
            for (void *p : b) hipFree(p);
        }
    } guard{bufs};
    auto dalloc = [&](void **p, size_t bytes) -> int {
        if (hipMalloc(p, bytes ? bytes : 16) != hipSuccess)
            return fail(NSG_ENOMEM, "ivf allocation of %zu bytes failed", bytes);
        bufs.push_back(*p);
        return NSG_OK;
    };
    const int64_t np = n * (int64_t)nprobe;
    if (np >= ((int64_t)1 << 31)) return fail(NSG_EUNSUPPORTED, "n * nprobe must be below 2^31");
    float *cent = nullptr, *pdist = nullptr;
    uint32_t *probe = nullptr, *member = nullptr, *qmember = nullptr;
    uint64_t *ck = nullptr, *cks = nullptr, *pk = nullptr, *pks = nullptr, *lists = nullptr;
    int64_t *counts = nullptr;
    int rc;
    if ((rc = dalloc((void **)&cent, sizeof(float) * (size_t)nlist * d)) ||
        (rc = dalloc((void **)&probe, sizeof(uint32_t) * (size_t)np)) ||
        (rc = dalloc((void **)&pdist, sizeof(float) * (size_t)np)) ||
        (rc = dalloc((void **)&ck, 8 * (size_t)n)) || (rc = dalloc((void **)&cks, 8 * (size_t)n)) ||
        (rc = dalloc((void **)&pk, 8 * (size_t)np)) || (rc = dalloc((void **)&pks, 8 * (size_t)np)) ||
        (rc = dalloc((void **)&member, 4 * (size_t)n)) || (rc = dalloc((void **)&qmember, 4 * (size_t)np)) ||
        (rc = dalloc((void **)&counts, 8 * 2 * (size_t)nlist)) ||
        (rc = dalloc((void **)&lists, 8 * (size_t)n * K)))
        return rc;
    // 1. cells and probes
    hipLaunchKernelGGL(ivf_gather_kernel, dim3((unsigned)nlist), dim3(256), 0, st, base, d, pivots, cent);
    NSG_HIP(hipGetLastError());
    if ((rc = nsg_knn_bruteforce(cent, nlist, base, n, d, nprobe, 0, probe, pdist, stream))) return rc;
    // 2. members and probing points of every cell, in id order
    hipLaunchKernelGGL(ivf_keys_kernel, dim3(grid_of(np)), dim3(256), 0, st, probe, n, nprobe, ck, pk);
    NSG_HIP(hipGetLastError());
    size_t tmp_bytes = 0, t1 = 0, t2 = 0;
    NSG_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, t1, ck, cks, (int)n, 0, 64, st));
    NSG_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, t2, pk, pks, (int)np, 0, 64, st));
    tmp_bytes = std::max(t1, t2);
    void *tmp = nullptr;
    if ((rc = dalloc(&tmp, tmp_bytes))) return rc;
    NSG_HIP(hipcub::DeviceRadixSort::SortKeys(tmp, t1, ck, cks, (int)n, 0, 64, st));
    NSG_HIP(hipcub::DeviceRadixSort::SortKeys(tmp, t2, pk, pks, (int)np, 0, 64, st));
    NSG_HIP(hipMemsetAsync(counts, 0, 8 * 2 * (size_t)nlist, st));
    hipLaunchKernelGGL(ivf_split_kernel, dim3(grid_of(n)), dim3(256), 0, st, cks, n, nlist, counts, member);
    hipLaunchKernelGGL(ivf_split_kernel, dim3(grid_of(np)), dim3(256), 0, st, pks, np, nlist, counts + nlist,
                       qmember);
    hipLaunchKernelGGL(ivf_fill_kernel, dim3(grid_of(n * K)), dim3(256), 0, st, lists, n * (int64_t)K, ~0ull);
    NSG_HIP(hipGetLastError());
    std::vector<int64_t> hc(2 * (size_t)nlist);
    NSG_HIP(hipMemcpyAsync(hc.data(), counts, 8 * hc.size(), hipMemcpyDeviceToHost, st));
    NSG_HIP(hipStreamSynchronize(st));
    int64_t mmax = 0, qmax = 0;
    for (int c = 0; c < nlist; ++c) {
        mmax = std::max(mmax, hc[c]);
        qmax = std::max(qmax, hc[nlist + c]);
    }
    // 3. cell by cell: probing points against members, merged into the lists.
    // Consecutive cells alternate between the caller's stream and a second
    // one, each with its own row, result and brute-force scratch buffers
    // (allocated once, for the largest cell), so that a cell's gathers and
    // brute force overlap the previous cell's; the merges, which update the
    // shared per-point lists, keep the cell order through events.
    const int kc = K + 1;
    float *bbuf[2] = {nullptr, nullptr}, *qbuf[2] = {nullptr, nullptr}, *cd[2] = {nullptr, nullptr};
    uint32_t *ci[2] = {nullptr, nullptr};
    void *ws[2] = {nullptr, nullptr};
    for (int h = 0; h < 2; ++h)
        if ((rc = dalloc((void **)&bbuf[h], sizeof(float) * (size_t)mmax * d)) ||
            (rc = dalloc((void **)&qbuf[h], sizeof(float) * (size_t)qmax * d)) ||
            (rc = dalloc((void **)&ci[h], sizeof(uint32_t) * (size_t)qmax * kc)) ||
            (rc = dalloc((void **)&cd[h], sizeof(float) * (size_t)qmax * kc)))
            return rc;
    size_t ws_bytes = 0;
    for (int c = 0; c < nlist; ++c) {
        const int64_t m = hc[c], q = hc[nlist + c];
        if (m == 0 || q == 0) continue;
        size_t b = 0;
        if ((rc = bf_scratch_bytes(bbuf[0], m, qbuf[0], q, d, kc, &b))) return rc;
        ws_bytes = std::max(ws_bytes, b);
    }
    for (int h = 0; h < 2; ++h)
        if ((rc = dalloc(&ws[h], ws_bytes))) return rc;
    struct Side {
        hipStream_t s2 = nullptr;
        hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
        ~Side() {
            if (s2) {
                hipStreamSynchronize(s2);
                hipStreamDestroy(s2);
            }
            for (hipEvent_t e : ev)
                if (e) hipEventDestroy(e);
        }
    } side;
    NSG_HIP(hipStreamCreateWithFlags(&side.s2, hipStreamNonBlocking));
    for (hipEvent_t &e : side.ev) NSG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // the second stream starts after the set-up above
    NSG_HIP(hipEventRecord(side.ev[2], st));
    NSG_HIP(hipStreamWaitEvent(side.s2, side.ev[2], 0));
    const int wpb = 4;
    const size_t lds = (size_t)wpb * (2 * K + 2) * 8;
    int64_t moff = 0, qoff = 0, done = 0;
    for (int c = 0; c < nlist; ++c) {
        const int64_t m = hc[c], q = hc[nlist + c];
        if (m > 0 && q > 0) {
            const int h = (int)(done & 1);
            hipStream_t s = h ? side.s2 : st;
            hipLaunchKernelGGL(ivf_gather_kernel, dim3((unsigned)m), dim3(128), 0, s, base, d, member + moff,
                               bbuf[h]);
            hipLaunchKernelGGL(ivf_gather_kernel, dim3((unsigned)q), dim3(128), 0, s, base, d, qmember + qoff,
                               qbuf[h]);
            NSG_HIP(hipGetLastError());
            if ((rc = bf_with_scratch(bbuf[h], m, qbuf[h], q, d, kc, 0, ci[h], cd[h], ws[h], ws_bytes, s)))
                return rc;
            // merges in cell order: after the previous cell's (other stream)
            if (done > 0) NSG_HIP(hipStreamWaitEvent(s, side.ev[h ^ 1], 0));
            hipLaunchKernelGGL(ivf_merge_kernel, dim3((unsigned)((q + wpb - 1) / wpb)), dim3(64 * wpb), lds, s,
                               qmember + qoff, q, member + moff, ci[h], cd[h], kc, lists, (int)K);
            NSG_HIP(hipGetLastError());
            NSG_HIP(hipEventRecord(side.ev[h], s));
            ++done;
        }
        moff += m;
        qoff += q;
    }
    // the caller's stream continues after the last merge
    if (done > 0) NSG_HIP(hipStreamWaitEvent(st, side.ev[(done - 1) & 1], 0));
    hipLaunchKernelGGL(ivf_out_kernel, dim3(grid_of(n * K)), dim3(256), 0, st, lists, n * (int64_t)K, out_ids,
                       out_dist);
    NSG_HIP(hipGetLastError());
    NSG_HIP(hipStreamSynchronize(st));
    return NSG_OK;
}
