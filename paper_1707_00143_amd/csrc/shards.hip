// Partitioned index: the point set split into subsets of consecutive rows,
// one NSG per subset, every query searched in every subset and the per-subset
// results merged (the paper's scheme for its largest sets: 16 sub-NSGs on
// DEEP100M, Sec. 4.2; 12 and 32 partitions on the Taobao sets, Sec. 4.3).
//
// On one GPU the subsets are one resident index whose graph rows hold global
// row ids (each subset's edges stay inside it), plus one navigating node per
// subset.  A search launch runs Algorithm 1 for every (query, subset) pair —
// one wavefront per pair, the same kernel as the single-graph search — into
// per-pair top-k lists; a merge kernel then ranks every listed key against
// the other lists (one wave per query) and writes the k smallest.
#include "wave.hpp"

#include <algorithm>
#include <vector>

struct nsg_shards {
    nsg_index *ix = nullptr;          // rows and graph (global ids)
    int32_t S = 0;
    std::vector<int64_t> offsets;     // host [S + 1]
    uint32_t *navs = nullptr;         // device [S], global ids
};

namespace nsg {

constexpr int kMaxShards = 64;
constexpr int kMaxShardKeys = 8192;   // S * k: one wave's merge keys fit 64 KB of LDS

// local -> global ids of one subset's rows; counts entries that are neither
// a local id of the subset nor the sentinel
__global__ void globalize_kernel(const uint32_t *g, int64_t rows, int R, uint32_t off, uint32_t size,
                                 uint32_t *out, unsigned long long *bad) {
    unsigned long long cnt = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows * R;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t u = g[i];
        if (u == NSG_SENT) {
            out[i] = NSG_SENT;
        } else if (u < size) {
            out[i] = u + off;
        } else {
            out[i] = NSG_SENT;
            ++cnt;
        }
    }
    if (cnt) atomicAdd(bad, cnt);
}

// number of keys in the sorted list a[0..n) below key
__device__ inline int count_below(const uint64_t *a, int n, uint64_t key) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// One wave per query: the S lists of k (distance, id) keys, each sorted, are
// staged in LDS; a listed key's rank in the union is its position in its own
// list plus the number of keys below it in every other list (keys are unique:
// the subsets are disjoint), so the keys of rank < k are written straight to
// their output slot.  Padding (SENT, +inf) fills the slots past the number of
// listed keys.
__global__ void __launch_bounds__(256) merge_shards_kernel(const uint32_t *sid, const float *sd, int64_t nq, int S,
                                                           int k, uint32_t *out_ids, float *out_dist) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t q = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (q >= nq) return;
    const int T = S * k;
    uint64_t *a = reinterpret_cast<uint64_t *>(smem) + (size_t)wave * T;
    const uint32_t *qi = sid + q * (int64_t)T;
    const float *qd = sd + q * (int64_t)T;
    int valid = 0;
    for (int i = lane; i - lane < T; i += 64) {
        uint64_t key = KEY_NONE;
        if (i < T && qi[i] != NSG_SENT) key = mk_key(qd[i], qi[i]);
        if (i < T) a[i] = key;
        valid += __popcll(__ballot(key != KEY_NONE));
    }
    wave_sync();
    for (int i = lane; i < T; i += 64) {
        const uint64_t key = a[i];
        if (key == KEY_NONE) continue;
        const int s = i / k;
        int rank = i - s * k;
        for (int t = 0; t < S && rank < k; ++t)
            if (t != s) rank += count_below(a + (size_t)t * k, k, key);
        if (rank < k) {
            out_ids[q * k + rank] = key_id(key);
            out_dist[q * k + rank] = key_dist(key);
        }
    }
    for (int r = valid + lane; r < k; r += 64) {
        out_ids[q * k + r] = NSG_SENT;
        out_dist[q * k + r] = INFINITY;
    }
}

}  // namespace nsg

using namespace nsg;

extern "C" void nsg_free_shards(nsg_shards *sh) {
    if (!sh) return;
    hipDeviceSynchronize();
    nsg_free_index(sh->ix);
    hipFree(sh->navs);
    delete sh;
}

extern "C" int nsg_shards_info(const nsg_shards *sh, int32_t *S, nsg_index **index) {
    if (!sh) return fail(NSG_EINVAL, "shards handle is NULL");
    if (S) *S = sh->S;
    if (index) *index = sh->ix;
    return NSG_OK;
}

extern "C" int nsg_load_shards(const float *base, int64_t n, int32_t d, const int64_t *offsets, int32_t S,
                               const uint32_t *graph, int32_t R, const uint32_t *navs, nsg_dtype storage,
                               const float *scales, void *stream, nsg_shards **out) {
    clear_error();
    if (!out) return fail(NSG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!base || !graph || !offsets || !navs) return fail(NSG_EINVAL, "NULL pointer");
    if (S < 1 || S > kMaxShards) return fail(NSG_EINVAL, "S=%d out of range [1, %d]", S, kMaxShards);
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(NSG_EINVAL, "n out of range [1, 2^31)");
    if (R < 1 || R > kMaxR) return fail(NSG_EINVAL, "R=%d out of range [1, %d]", R, kMaxR);
    if (offsets[0] != 0 || offsets[S] != n) return fail(NSG_EINVAL, "offsets must run from 0 to n");
    for (int s = 0; s < S; ++s) {
        if (offsets[s + 1] <= offsets[s]) return fail(NSG_EINVAL, "shard %d is empty or offsets decrease", s);
        if ((int64_t)navs[s] >= offsets[s + 1] - offsets[s])
            return fail(NSG_EINVAL, "navigating node %u of shard %d is not a local id", navs[s], s);
    }
    hipStream_t st = (hipStream_t)stream;
    uint32_t *g = nullptr;
    unsigned long long *bad = nullptr, hbad = 0;
    if (hipMalloc(&g, sizeof(uint32_t) * n * R) != hipSuccess || hipMalloc(&bad, sizeof(*bad)) != hipSuccess) {
        hipFree(g);
        return fail(NSG_ENOMEM, "graph staging allocation failed");
    }
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(*bad), st);
    for (int s = 0; s < S && e == hipSuccess; ++s) {
        const int64_t rows = offsets[s + 1] - offsets[s];
        const int64_t cnt = rows * R;
        const int grid = (int)std::min<int64_t>(std::max<int64_t>((cnt + 255) / 256, 1), 65536);
        hipLaunchKernelGGL(globalize_kernel, dim3(grid), dim3(256), 0, st, graph + offsets[s] * R, rows, R,
                           (uint32_t)offsets[s], (uint32_t)rows, g + offsets[s] * R, bad);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipFree(bad);
    if (e != hipSuccess) {
        hipFree(g);
        return fail(NSG_EDEVICE, "graph conversion failed: %s", hipGetErrorString(e));
    }
    if (hbad) {
        hipFree(g);
        return fail(NSG_EINVAL, "%llu graph entries are neither a local id of their shard nor the sentinel", hbad);
    }
    nsg_shards *sh = new nsg_shards();
    sh->S = S;
    sh->offsets.assign(offsets, offsets + S + 1);
    int rc = nsg_load_index(base, n, d, g, R, navs[0], storage, scales, stream, &sh->ix);
    hipStreamSynchronize(st);
    hipFree(g);
    if (rc) {
        const char *msg = nsg_last_error();
        char keep[512];
        snprintf(keep, sizeof(keep), "%s", msg);
        delete sh;
        return fail(rc, "%s", keep);
    }
    std::vector<uint32_t> gn(S);
    for (int s = 0; s < S; ++s) gn[s] = navs[s] + (uint32_t)offsets[s];
    if (hipMalloc(&sh->navs, sizeof(uint32_t) * S) != hipSuccess) {
        nsg_free_shards(sh);
        return fail(NSG_ENOMEM, "allocation failed");
    }
    if (hipMemcpy(sh->navs, gn.data(), sizeof(uint32_t) * S, hipMemcpyHostToDevice) != hipSuccess) {
        nsg_free_shards(sh);
        return fail(NSG_EDEVICE, "copy of the navigating nodes failed");
    }
    *out = sh;
    return NSG_OK;
}

extern "C" int nsg_search_shards(const nsg_shards *sh, const float *queries, int64_t nq, int32_t k, int32_t L,
                                 uint32_t *out_ids, float *out_dist, void *stream) {
    clear_error();
    if (!sh) return fail(NSG_EINVAL, "shards handle is NULL");
    if (nq < 0 || nq >= ((int64_t)1 << 31) / std::max(1, sh->S)) return fail(NSG_EINVAL, "nq out of range");
    if (k < 1 || k > kMaxK) return fail(NSG_EINVAL, "k=%d out of range [1, %d]", k, kMaxK);
    if (L < 1 || L > kMaxL) return fail(NSG_EINVAL, "L=%d out of range [1, %d]", L, kMaxL);
    if ((int64_t)sh->S * k > kMaxShardKeys)
        return fail(NSG_EUNSUPPORTED, "S * k = %d above %d", sh->S * k, kMaxShardKeys);
    if (nq == 0) return NSG_OK;
    if (!queries || !out_ids || !out_dist) return fail(NSG_EINVAL, "NULL query or output pointer");
    hipStream_t st = (hipStream_t)stream;
    const int64_t T = nq * sh->S;
    uint32_t *sid = nullptr;
    float *sd = nullptr;
    if (hipMallocAsync((void **)&sid, sizeof(uint32_t) * T * k, st) != hipSuccess ||
        hipMallocAsync((void **)&sd, sizeof(float) * T * k, st) != hipSuccess) {
        if (sid) hipFreeAsync(sid, st);
        return fail(NSG_ENOMEM, "per-subset result allocation failed");
    }
    SearchArgs a{};
    a.idx = sh->ix;
    a.queries = queries;
    a.nq = T;
    a.k_scalar = k;
    a.L_scalar = L;
    a.out_stride = k;
    a.out_ids = sid;
    a.out_dist = sd;
    a.L_cap = L;
    a.hash_bits = default_hash_bits(L);
    a.rerank = sh->ix->storage != NSG_F32;
    a.persistent = T >= 4096;
    a.start_override = NSG_SENT;
    a.self_offset = -1;
    a.shards = sh->S;
    a.shard_starts = sh->navs;
    a.stream = st;
    int rc = launch_search(a);
    if (rc == NSG_OK) {
        const size_t per_wave = (size_t)sh->S * k * 8;
        const int wpb = (int)std::max<size_t>(1, std::min<size_t>(4, (64 * 1024) / per_wave));
        const size_t lds = per_wave * wpb;
        hipLaunchKernelGGL(merge_shards_kernel, dim3((unsigned)((nq + wpb - 1) / wpb)), dim3(64 * wpb), lds, st, sid,
                           sd, nq, sh->S, k, out_ids, out_dist);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) rc = fail(NSG_EDEVICE, "merge launch failed: %s", hipGetErrorString(e));
    }
    hipFreeAsync(sid, st);
    hipFreeAsync(sd, st);
    return rc;
}
