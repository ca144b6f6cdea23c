// Host side of the batched search: launch configuration and kernel choice.
// The kernels (Algorithm 1, one wavefront per query) are in search_impl.hpp,
// instantiated per row format in search_<format>.hip.
#include "search_impl.hpp"

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

namespace nsg {

// ------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------
void pick_layout(int chunks, int max_cpl, int *lpr, int *cpl) {
    // the fewest lanes per row whose chunks fit in at most max_cpl per lane
    int l = 8;
    while (l < 64 && l * max_cpl < chunks) l <<= 1;
    int c = (chunks + l - 1) / l;
    if (c == 3) c = 4;
    *lpr = l;
    *cpl = c;
}

__global__ void reset_counter_kernel(unsigned int *c) { if (threadIdx.x == 0) c[0] = 0u; }

// Work counter of the persistent grid for calls that bring none: one per
// (device, stream), allocated on first use and kept for the life of the
// process.  Launches on one stream run in order, so they can share it; calls
// on different streams get different counters.
static int stream_counter(hipStream_t st, unsigned int **out) {
    static std::mutex mu;
    static std::map<std::pair<int, hipStream_t>, unsigned int *> counters;
    int dev = 0;
    NSG_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_pair(dev, st);
    auto it = counters.find(key);
    if (it != counters.end()) {
        *out = it->second;
        return NSG_OK;
    }
    unsigned int *c = nullptr;
    if (hipMalloc((void **)&c, 256) != hipSuccess) return fail(NSG_ENOMEM, "work counter allocation failed");
    counters[key] = c;
    *out = c;
    return NSG_OK;
}

// Longest walks first.  A batch larger than the chip's wave slots ends on
// the walks that started last; starting the queries farthest from the start
// node first (their squared distance to it, the first distance of every
// walk, tracks how long the walk runs) leaves shorter walks for the end.
// The order only needs to be approximate: one block sorts the queries into
// 1024 buckets of distance between the batch's extremes (farthest first;
// NaN last), in any order within a bucket.
__global__ void order_key_kernel(const float *queries, int64_t nq, int d, const float *srow, float *dist) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (i >= nq) return;
    const float *q = queries + i * d;
    float s = 0.0f;
    for (int j = lane; j < d; j += 64) {
        const float t = q[j] - srow[j];
        s = fmaf(t, t, s);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) dist[i] = s;
}

constexpr int kOrderBuckets = 1024;   // one per thread of the ordering block

__device__ inline int order_bucket(float x, float hi, float scale) {
    if (!(x == x)) return kOrderBuckets - 1;
    const float f = (hi - x) * scale;   // NaN when x and hi are both infinite
    if (!(f > 0.0f)) return 0;
    return f >= (float)(kOrderBuckets - 1) ? kOrderBuckets - 1 : (int)f;
}

__global__ void __launch_bounds__(kOrderBuckets) order_bucket_kernel(const float *dist, int nq, uint32_t *order) {
    __shared__ uint32_t cnt[kOrderBuckets];
    __shared__ float wlo[kOrderBuckets / 64], whi[kOrderBuckets / 64];
    __shared__ uint32_t wsum[kOrderBuckets / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    // extremes of the batch's distances
    float lo = INFINITY, hi = -INFINITY;
    for (int i = t; i < nq; i += kOrderBuckets) {
        const float x = dist[i];
        if (x == x) {
            lo = fminf(lo, x);
            hi = fmaxf(hi, x);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, o));
        hi = fmaxf(hi, __shfl_xor(hi, o));
    }
    if (lane == 0) {
        wlo[w] = lo;
        whi[w] = hi;
    }
    cnt[t] = 0u;
    __syncthreads();
    lo = wlo[0];
    hi = whi[0];
    for (int v = 1; v < kOrderBuckets / 64; ++v) {
        lo = fminf(lo, wlo[v]);
        hi = fmaxf(hi, whi[v]);
    }
    const float scale = hi > lo ? (float)kOrderBuckets / (hi - lo) : 0.0f;
    // bucket sizes
    for (int i = t; i < nq; i += kOrderBuckets) atomicAdd(&cnt[order_bucket(dist[i], hi, scale)], 1u);
    __syncthreads();
    // exclusive scan of the sizes: within each wave, then over the waves
    const uint32_t c = cnt[t];
    uint32_t incl = c;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = (uint32_t)__shfl_up((int)incl, o);
        if (lane >= o) incl += u;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t base = 0;
    for (int v = 0; v < w; ++v) base += wsum[v];
    __syncthreads();
    cnt[t] = base + incl - c;   // first position of bucket t
    __syncthreads();
    for (int i = t; i < nq; i += kOrderBuckets) order[atomicAdd(&cnt[order_bucket(dist[i], hi, scale)], 1u)] = (uint32_t)i;
}

// Scratch of the order for calls that bring none: one per (device, stream),
// like the work counter.
static int stream_order_scratch(hipStream_t st, uint32_t **out) {
    static std::mutex mu;
    static std::map<std::pair<int, hipStream_t>, uint32_t *> bufs;
    int dev = 0;
    NSG_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_pair(dev, st);
    auto it = bufs.find(key);
    if (it != bufs.end()) {
        *out = it->second;
        return NSG_OK;
    }
    uint32_t *b = nullptr;
    if (hipMalloc((void **)&b, sizeof(uint32_t) * 2 * NSG_ORDER_MAX) != hipSuccess)
        return fail(NSG_ENOMEM, "order scratch allocation failed");
    bufs[key] = b;
    *out = b;
    return NSG_OK;
}

kfn_t pick_search_kernel_f32(int lpr, int cpl, int nch);
kfn_t pick_search_kernel_f32_stop(int lpr, int cpl, int nch);
kfn_t pick_search_kernel_f32_full(int lpr, int cpl, int nch);
kfn_t pick_search_kernel_bf16(int lpr, int cpl, int nch);
kfn_t pick_search_kernel_bf16_stop(int lpr, int cpl, int nch);
kfn_t pick_search_kernel_bf16_full(int lpr, int cpl, int nch);
kfn_t pick_search_kernel_f16(int lpr, int cpl, int nch);
kfn_t pick_search_kernel_f16_stop(int lpr, int cpl, int nch);
kfn_t pick_search_kernel_f16_full(int lpr, int cpl, int nch);
kfn_t pick_search_kernel_e4m3(int lpr, int cpl, int nch);
kfn_t pick_search_kernel_e4m3_stop(int lpr, int cpl, int nch);
kfn_t pick_search_kernel_e4m3_full(int lpr, int cpl, int nch);


int launch_search(const SearchArgs &a) {
    const nsg_index *ix = a.idx;
    if (a.nq == 0) return NSG_OK;
    KParams p{};
    const bool lp = ix->storage != NSG_F32;
    p.tab.base = reinterpret_cast<const unsigned char *>(lp ? ix->base_lp : (const void *)ix->base_f32);
    p.tab.row_bytes = (uint32_t)ix->row_chunks * 16u;
    p.tab.n_rows = (uint32_t)ix->n;
    p.tab.row_chunks = ix->row_chunks;
    p.scales = ix->scales;
    p.rows_f32 = ix->base_f32;
    p.graph = a.graph_override ? a.graph_override : ix->graph;
    p.R = a.graph_override ? a.R_override : ix->R;
    p.R_pad = a.graph_override ? a.Rpad_override : ix->R_pad;
    p.d = ix->d;
    p.n_rows = (uint32_t)ix->n;
    p.row_chunks = ix->row_chunks;
    p.row_chunks_f32 = ix->row_chunks_f32;
    p.start = a.start_override != NSG_SENT ? a.start_override : ix->nav;
    p.queries = a.queries;
    p.nq = a.nq;
    p.k_arr = a.k_arr;
    p.L_arr = a.L_arr;
    p.k_scalar = a.k_scalar;
    p.L_scalar = a.L_scalar;
    p.out_stride = a.out_stride;
    p.out_ids = a.out_ids;
    p.out_dist = a.out_dist;
    p.L_cap = a.L_cap;
    p.hash_bits = a.hash_bits;
    p.rerank = a.rerank;
    p.rr_eta = ix->rr_eta;
    p.rr_rho = (float)(ix->d + 4) * 0x1p-24f;
    p.hops = a.hops;
    p.ndist = a.ndist;
    p.nedges = a.nedges;
    p.max_hops = a.max_hops;
    p.clamped = a.clamped;
    p.pool_ids = a.pool_ids;
    p.pool_dist = a.pool_dist;
    p.pool_stride = a.pool_stride;
    p.vis_ids = a.vis_ids;
    p.vis_dist = a.vis_dist;
    p.vis_cnt = a.vis_cnt;
    p.vis_cap = a.vis_cap;
    p.trace_ids = a.trace_ids;
    p.trace_cap = a.trace_cap;
    p.self_offset = a.self_offset;
    p.shards = a.shards > 1 ? a.shards : 1;
    p.shard_starts = a.shard_starts;
    p.init_ids = a.init_n > 0 ? a.init_ids : nullptr;
    p.init_n = a.init_n > 0 ? a.init_n : 0;
    // learned early stop and feature capture, fused into the search loop
    p.features = a.features;
    p.budget = a.budget;
    p.learned = 0;
    p.s_hop = a.feature_hop > 0 ? a.feature_hop : 16;
    p.s_cps = (uint64_t)(p.s_hop & 0xFFFF);
    if (a.learned) {
        const StopModel &sm = ix->stop;
        if (!sm.blob) return fail(NSG_ESTATE, "no early-stop model loaded");
        if (a.features && a.feature_hop > 0 && a.feature_hop != sm.hop)
            return fail(NSG_EINVAL, "feature hop differs from the model's decision hop");
        p.learned = 1;
        p.stop_plan = sm.blob;
        p.s_in = sm.in;
        p.s_kind = sm.kind;
        p.s_hop = sm.hop;
        p.s_cps = 0;
        for (int c = 0; c < sm.ncp; ++c) p.s_cps |= (uint64_t)(sm.cps[c] & 0xFFFF) << (16 * c);
        p.grid_n = sm.grid_n;
        p.calib_c = sm.calib_c;
    }
    int L_alloc = 1;
    while (L_alloc < a.L_cap) L_alloc <<= 1;
    p.L_alloc = L_alloc;
    // pool, visited filter, candidate ids and distances
    size_t per_wave = (size_t)L_alloc * 8 + ((size_t)4 << a.hash_bits) + kMaxR * 8;
    per_wave = (per_wave + 15) & ~(size_t)15;
    p.lds_per_wave = (int)per_wave;
    int wpb = a.waves_per_block;
    if (wpb <= 0) {
        wpb = 4;
        while (wpb > 1 && per_wave * wpb > 64 * 1024) wpb >>= 1;
    }
    if (per_wave * wpb > 160 * 1024)
        return fail(NSG_EUNSUPPORTED, "search needs %zu bytes of LDS per block", per_wave * wpb);
    int lpr, cpl;
    pick_layout(ix->row_chunks, ix->storage == NSG_E4M3 ? 2 : 4, &lpr, &cpl);
    if (a.lanes_per_row) {
        lpr = a.lanes_per_row;
        cpl = (ix->row_chunks + lpr - 1) / lpr;
        if (cpl == 3) cpl = 4;
        if (cpl > 4) return fail(NSG_EINVAL, "lanes_per_row=%d too small for %d chunks per row", lpr, ix->row_chunks);
    }
    const bool full = a.vis_ids || a.pool_ids || a.hops || a.ndist || a.nedges || a.trace_ids || a.self_offset >= 0;
    const int mode = full ? 2 : (a.learned || a.features || a.budget) ? 1 : 0;
    // pool chunks of 64 held in registers (2 * nch registers per lane); the
    // LDS copy of the pool (re-rank sort) keeps the power-of-two L_alloc
    const int nch = a.L_cap <= 128 ? 2 : a.L_cap <= 256 ? 4 : a.L_cap <= 384 ? 6 : 8;
    kfn_t fn = nullptr;
    switch (ix->storage) {
    case NSG_F32: fn = mode == 2 ? pick_search_kernel_f32_full(lpr, cpl, nch)
                       : mode == 1 ? pick_search_kernel_f32_stop(lpr, cpl, nch)
                                   : pick_search_kernel_f32(lpr, cpl, nch);
        break;
    case NSG_BF16: fn = mode == 2 ? pick_search_kernel_bf16_full(lpr, cpl, nch)
                       : mode == 1 ? pick_search_kernel_bf16_stop(lpr, cpl, nch)
                                   : pick_search_kernel_bf16(lpr, cpl, nch);
        break;
    case NSG_F16: fn = mode == 2 ? pick_search_kernel_f16_full(lpr, cpl, nch)
                       : mode == 1 ? pick_search_kernel_f16_stop(lpr, cpl, nch)
                                   : pick_search_kernel_f16(lpr, cpl, nch);
        break;
    case NSG_E4M3: fn = mode == 2 ? pick_search_kernel_e4m3_full(lpr, cpl, nch)
                       : mode == 1 ? pick_search_kernel_e4m3_stop(lpr, cpl, nch)
                                   : pick_search_kernel_e4m3(lpr, cpl, nch);
        break;
    }
    if (!fn) return fail(NSG_EUNSUPPORTED, "no search kernel for %d chunks per row", ix->row_chunks);
    size_t lds = per_wave * wpb;
    if (lds > 64 * 1024) NSG_HIP(hipFuncSetAttribute((const void *)fn,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int64_t blocks;
    if (a.persistent) {
        if (a.counter) {
            p.counter = a.counter;
        } else {
            int rc = stream_counter(a.stream, &p.counter);
            if (rc) return rc;
        }
        hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, a.stream, p.counter);
        int per_cu = 0;
        NSG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, 64 * wpb, lds));
        int dev = 0, cus = 0;
        NSG_HIP(hipGetDevice(&dev));
        NSG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        blocks = a.blocks > 0 ? a.blocks : (int64_t)std::max(1, per_cu) * cus;
        int64_t need = (a.nq + wpb - 1) / wpb;
        if (blocks > need) blocks = need;
        // every wave takes its first query from the counter too
    } else {
        blocks = (a.nq + wpb - 1) / wpb;
        p.counter = nullptr;
    }
    p.order = nullptr;
    if (a.longest_first && a.nq >= 2 && a.nq <= NSG_ORDER_MAX && p.shards == 1 && p.init_n == 0) {
        uint32_t *scr = a.order_scratch;
        if (!scr) {
            int rc = stream_order_scratch(a.stream, &scr);
            if (rc) return rc;
        }
        const float *srow = ix->base_f32 + (int64_t)p.start * (ix->row_chunks_f32 * 4);
        float *dist = reinterpret_cast<float *>(scr);
        hipLaunchKernelGGL(order_key_kernel, dim3((unsigned)((a.nq + 3) / 4)), dim3(256), 0, a.stream, a.queries,
                           a.nq, ix->d, srow, dist);
        hipLaunchKernelGGL(order_bucket_kernel, dim3(1), dim3(kOrderBuckets), 0, a.stream, dist, (int)a.nq,
                           scr + NSG_ORDER_MAX);
        p.order = scr + NSG_ORDER_MAX;
    }
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(64 * wpb), lds, a.stream, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(NSG_EDEVICE, "search launch failed: %s", hipGetErrorString(e));
    return NSG_OK;
}

}  // namespace nsg
