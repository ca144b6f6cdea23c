// Index construction on the GPU (Algorithm 2, NSGbuild(G, l, m)).
//
//  1. centroid of the base (FP64 sums, FP32 result)
//  2. navigating node: Algorithm 1 on the kNN graph from the given random
//     node, query = centroid, pool size l; its first result
//  3. search-collect (batched, one wave per node): Algorithm 1 on the kNN
//     graph from the navigating node with the node itself as query; every
//     node whose distance is computed is recorded, then the node's own kNN
//     row is visited the same way (so E = visited + kNN neighbours)
//  4. select (one wave per node): the C nearest of E by (distance, id), self
//     and duplicates removed, through the same LDS pool merge as the search;
//     then the MRNG rule in that order: keep p unless a kept r has
//     delta(p, r) < delta(v, p), at most m edges
//  5. DFS-tree repair on the host: while a node is unreached from the
//     navigating node, search the current graph for the smallest unreached id
//     u (Algorithm 1, pool size l, on the GPU), link the first pool entry that
//     has a free slot to u, continue the DFS from u.
#include "wave.hpp"

#include <algorithm>
#include <vector>

namespace nsg {

struct SelParams {
    RowTable tab;            // FP32 rows of the index copy
    int row_chunks;
    uint32_t n_rows;
    const uint32_t *vis_ids;
    const float *vis_dist;
    const int32_t *vis_cnt;
    int vis_cap;
    int64_t node0, nb;
    int C, C_alloc, m;
    uint32_t *graph;         // [n][m]
    int lds_per_wave;
};

template <int LPR, int CPL>
__global__ void __launch_bounds__(256) select_kernel(SelParams p) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, wpb = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t b = (int64_t)blockIdx.x * wpb + wave;
    if (b >= p.nb) return;
    unsigned char *wb = smem + (size_t)wave * p.lds_per_wave;
    uint64_t *pool = reinterpret_cast<uint64_t *>(wb);
    uint64_t *sbuf = pool + p.C_alloc;   // 16 staged keys (+16 spare)
    uint32_t *sel = reinterpret_cast<uint32_t *>(sbuf + 32);
    float *cdist = reinterpret_cast<float *>(sel + kMaxR);
    const uint32_t v = (uint32_t)(p.node0 + b);
    const uint32_t *vid = p.vis_ids + b * (int64_t)p.vis_cap;
    const float *vd = p.vis_dist + b * (int64_t)p.vis_cap;
    const int cntv = min(p.vis_cnt[b], p.vis_cap);
    int size = 0;
    for (int b0 = 0; b0 < cntv; b0 += 64) {
        const uint64_t worst = size >= p.C ? (pool[p.C - 1] & KEY_MASK) : KEY_NONE;
        int r = b0 + lane;
        uint64_t key = KEY_NONE;
        if (r < cntv) {
            uint32_t id = vid[r];
            if (id != v) {
                uint64_t kk = mk_key(vd[r], id);
                if (kk < worst) key = kk;
            }
        }
        int fi;
        size = merge_pool(pool, size, p.C, key, sbuf, lane, &fi);
    }
    // MRNG selection over the sorted candidates
    constexpr int EPC = 4;
    float qv[CPL][EPC], sc[CPL][EPC];
    const int li = lane % LPR;
    int s = 0;
    for (int t = 0; t < size && s < p.m; ++t) {
        const uint64_t pk = pool[t];
        uint32_t pid = key_id(pk);
        pid = pid < p.n_rows ? pid : 0u;
        const float dvp = key_dist(pk);
        bool conflict = false;
        if (s > 0) {
            const uint4 *prow = reinterpret_cast<const uint4 *>(p.tab.base) + (int64_t)pid * p.row_chunks;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                int ch = li + c * LPR;
                uint4 r = ch < p.row_chunks ? prow[ch] : make_uint4(0u, 0u, 0u, 0u);
                qv[c][0] = __uint_as_float(r.x); qv[c][1] = __uint_as_float(r.y);
                qv[c][2] = __uint_as_float(r.z); qv[c][3] = __uint_as_float(r.w);
#pragma unroll
                for (int e = 0; e < EPC; ++e) sc[c][e] = 0.0f;
            }
            gather_dist<NSG_F32, LPR, CPL>(p.tab, qv, sc, sel, cdist, s, lane);
            wave_sync();
            bool c0 = lane < s && cdist[lane] < dvp;
            bool c1 = lane + 64 < s && cdist[lane + 64] < dvp;
            conflict = __ballot(c0 || c1) != 0ull;
        }
        if (!conflict) {
            if (lane == 0) sel[s] = pid;
            ++s;
            wave_sync();
        }
    }
    uint32_t *row = p.graph + (int64_t)v * p.m;
    for (int j = lane; j < p.m; j += 64) row[j] = j < s ? sel[j] : NSG_SENT;
}

typedef void (*selfn_t)(SelParams);
static selfn_t pick_select(int lpr, int cpl) {
#define NSG_S(L_, C_) if (lpr == L_ && cpl == C_) return select_kernel<L_, C_>;
    NSG_S(8, 1) NSG_S(8, 2) NSG_S(8, 4) NSG_S(16, 1) NSG_S(16, 2) NSG_S(16, 4)
    NSG_S(32, 1) NSG_S(32, 2) NSG_S(32, 4) NSG_S(64, 1) NSG_S(64, 2) NSG_S(64, 4)
#undef NSG_S
    return nullptr;
}

// nearest node to q among mask[i] != 0, by (FP32 squared distance, id)
__global__ void nearest_masked_kernel(const float *rows, int ld, int d, int64_t n, const float *q,
                                      const unsigned char *mask, unsigned long long *best) {
    const int lane = threadIdx.x & 63;
    const int64_t w = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t i = w; i < n; i += nw) {
        if (!mask[i]) continue;
        float s = 0.0f;
        for (int j = lane; j < d; j += 64) {
            float t = q[j] - rows[i * ld + j];
            s = fmaf(t, t, s);
        }
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        if (lane == 0) atomicMin(best, ((unsigned long long)__float_as_uint(s) << 32) | (unsigned long long)i);
    }
}

static void dfs_mark(const std::vector<uint32_t> &g, int m, uint32_t root, std::vector<unsigned char> &reached,
                     std::vector<uint32_t> &stack) {
    if (reached[root]) return;
    reached[root] = 1;
    stack.clear();
    stack.push_back(root);
    while (!stack.empty()) {
        uint32_t v = stack.back();
        stack.pop_back();
        const uint32_t *row = g.data() + (size_t)v * m;
        for (int j = 0; j < m; ++j) {
            uint32_t u = row[j];
            if (u == NSG_SENT) break;
            if (!reached[u]) { reached[u] = 1; stack.push_back(u); }
        }
    }
}

}  // namespace nsg

using namespace nsg;

extern "C" int nsg_build(const float *base, int64_t n, int32_t d, const uint32_t *knn, int32_t K, int32_t Lb,
                         int32_t C, int32_t R, uint32_t rand_start, uint32_t *graph_out, uint32_t *nav_out,
                         int64_t *repair_edges, void *stream) {
    clear_error();
    if (!base || !knn || !graph_out || !nav_out) return fail(NSG_EINVAL, "NULL pointer");
    if (n < 2 || n >= ((int64_t)1 << 31)) return fail(NSG_EINVAL, "n out of range");
    if (K < 1 || K > kMaxR) return fail(NSG_EINVAL, "K=%d out of range [1, %d]", K, kMaxR);
    if (Lb < 1 || Lb > kMaxL) return fail(NSG_EINVAL, "Lb out of range");
    if (C < 1 || C > kMaxL) return fail(NSG_EINVAL, "C=%d out of range [1, %d]", C, kMaxL);
    if (R < 1 || R > kMaxR) return fail(NSG_EINVAL, "R out of range");
    if ((int64_t)rand_start >= n) return fail(NSG_EINVAL, "rand_start >= n");
    hipStream_t st = (hipStream_t)stream;
    nsg_index *kix = nullptr;
    int rc = nsg_load_index(base, n, d, knn, K, rand_start, NSG_F32, nullptr, stream, &kix);
    if (rc) return rc;
    struct Guard {
        nsg_index *ix;
        std::vector<void *> bufs;
        ~Guard() {
            for (void *b : bufs) hipFree(b);
            nsg_free_index(ix);
        }
    } guard{kix, {}};
    auto dalloc = [&](void **ptr, size_t bytes) -> int {
        if (hipMalloc(ptr, bytes) != hipSuccess) return fail(NSG_ENOMEM, "build allocation of %zu bytes failed", bytes);
        guard.bufs.push_back(*ptr);
        return NSG_OK;
    };
    // 1. centroid
    float *cen = nullptr;
    float2 *acc = nullptr;
    if ((rc = dalloc((void **)&cen, sizeof(float) * d)) ||
        (rc = dalloc((void **)&acc, sizeof(float2) * d * mean_blocks(n))))
        return rc;
    rc = launch_mean(base, n, d, cen, acc, st);
    if (rc) return rc;
    // 2. navigating node
    uint32_t *one_id = nullptr;
    float *one_d = nullptr;
    if ((rc = dalloc((void **)&one_id, 4 * (size_t)kMaxL)) || (rc = dalloc((void **)&one_d, 4 * (size_t)kMaxL))) return rc;
    SearchArgs a{};
    a.idx = kix;
    a.queries = cen;
    a.nq = 1;
    a.k_scalar = 1;
    a.L_scalar = Lb;
    a.out_stride = 1;
    a.out_ids = one_id;
    a.out_dist = one_d;
    a.L_cap = Lb;
    a.hash_bits = 13;
    a.start_override = rand_start;
    a.self_offset = -1;
    a.stream = st;
    if ((rc = launch_search(a))) return rc;
    uint32_t nav = 0;
    NSG_HIP(hipMemcpyAsync(&nav, one_id, 4, hipMemcpyDeviceToHost, st));
    NSG_HIP(hipStreamSynchronize(st));
    // 3 + 4. search-collect and select, in batches of nodes
    const int vis_cap = 8192;
    const int64_t B = std::min<int64_t>(n, 32768);
    uint32_t *vid = nullptr, *dummy_id = nullptr;
    float *vdist = nullptr, *dummy_d = nullptr;
    int32_t *vcnt = nullptr;
    if ((rc = dalloc((void **)&vid, sizeof(uint32_t) * B * vis_cap)) ||
        (rc = dalloc((void **)&vdist, sizeof(float) * B * vis_cap)) ||
        (rc = dalloc((void **)&vcnt, sizeof(int32_t) * B)) ||
        (rc = dalloc((void **)&dummy_id, sizeof(uint32_t) * B)) ||
        (rc = dalloc((void **)&dummy_d, sizeof(float) * B)))
        return rc;
    int lpr, cpl;
    pick_layout(kix->row_chunks_f32, 4, &lpr, &cpl);
    selfn_t sfn = pick_select(lpr, cpl);
    if (!sfn) return fail(NSG_EUNSUPPORTED, "no select kernel for d=%d", d);
    int C_alloc = 1;
    while (C_alloc < C) C_alloc <<= 1;
    SelParams sp{};
    sp.tab.base = reinterpret_cast<const unsigned char *>(kix->base_f32);
    sp.tab.row_bytes = (uint32_t)kix->row_chunks_f32 * 16u;
    sp.tab.n_rows = (uint32_t)n;
    sp.tab.row_chunks = kix->row_chunks_f32;
    sp.row_chunks = kix->row_chunks_f32;
    sp.n_rows = (uint32_t)n;
    sp.vis_ids = vid;
    sp.vis_dist = vdist;
    sp.vis_cnt = vcnt;
    sp.vis_cap = vis_cap;
    sp.C = C;
    sp.C_alloc = C_alloc;
    sp.m = R;
    sp.graph = graph_out;
    sp.lds_per_wave = (int)(((size_t)C_alloc * 8 + 32 * 8 + kMaxR * 4 + kMaxR * 4 + 15) & ~(size_t)15);
    const int swpb = 4;
    int64_t overflow = 0;
    std::vector<int32_t> hcnt((size_t)B);
    for (int64_t v0 = 0; v0 < n; v0 += B) {
        const int64_t nb = std::min<int64_t>(B, n - v0);
        SearchArgs c = a;
        c.queries = base + v0 * (int64_t)d;
        c.nq = nb;
        c.out_ids = dummy_id;
        c.out_dist = dummy_d;
        c.start_override = nav;
        c.vis_ids = vid;
        c.vis_dist = vdist;
        c.vis_cnt = vcnt;
        c.vis_cap = vis_cap;
        c.self_offset = v0;
        if ((rc = launch_search(c))) return rc;
        sp.node0 = v0;
        sp.nb = nb;
        hipLaunchKernelGGL(sfn, dim3((unsigned)((nb + swpb - 1) / swpb)), dim3(64 * swpb),
                           (size_t)sp.lds_per_wave * swpb, st, sp);
        NSG_HIP(hipGetLastError());
        NSG_HIP(hipMemcpyAsync(hcnt.data(), vcnt, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, st));
        NSG_HIP(hipStreamSynchronize(st));
        for (int64_t i = 0; i < nb; ++i) overflow += hcnt[i] > vis_cap;
    }
    if (overflow) return fail(NSG_EUNSUPPORTED, "%lld nodes visited more than %d nodes in search-collect",
                              (long long)overflow, vis_cap);
    // 5. DFS-tree connectivity repair
    std::vector<uint32_t> g((size_t)n * R);
    NSG_HIP(hipMemcpyAsync(g.data(), graph_out, sizeof(uint32_t) * g.size(), hipMemcpyDeviceToHost, st));
    NSG_HIP(hipStreamSynchronize(st));
    std::vector<int> deg((size_t)n);
    for (int64_t v = 0; v < n; ++v) {
        int c = 0;
        while (c < R && g[(size_t)v * R + c] != NSG_SENT) ++c;
        deg[v] = c;
    }
    std::vector<unsigned char> reached((size_t)n, 0);
    std::vector<uint32_t> stack;
    dfs_mark(g, R, nav, reached, stack);
    uint32_t *pool_id = nullptr;
    float *pool_d = nullptr;
    unsigned char *dmask = nullptr;
    unsigned long long *dbest = nullptr;
    if ((rc = dalloc((void **)&pool_id, sizeof(uint32_t) * Lb)) || (rc = dalloc((void **)&pool_d, sizeof(float) * Lb)))
        return rc;
    std::vector<uint32_t> hpool((size_t)Lb);
    int64_t added = 0;
    int64_t scan = 0;
    for (;;) {
        while (scan < n && reached[scan]) ++scan;
        if (scan >= n) break;
        const uint32_t u = (uint32_t)scan;
        SearchArgs r = a;
        r.graph_override = graph_out;
        r.R_override = R;
        r.Rpad_override = R;
        r.start_override = nav;
        r.queries = base + (int64_t)u * d;
        r.nq = 1;
        r.L_cap = Lb;
        r.L_scalar = Lb;
        r.hash_bits = default_hash_bits(Lb);
        r.pool_ids = pool_id;
        r.pool_dist = pool_d;
        r.pool_stride = Lb;
        if ((rc = launch_search(r))) return rc;
        NSG_HIP(hipMemcpyAsync(hpool.data(), pool_id, sizeof(uint32_t) * Lb, hipMemcpyDeviceToHost, st));
        NSG_HIP(hipStreamSynchronize(st));
        int64_t w = -1;
        for (int t = 0; t < Lb; ++t) {
            uint32_t c = hpool[t];
            if (c == NSG_SENT) break;
            if (reached[c] && deg[c] < R) { w = c; break; }
        }
        if (w < 0) {
            // no pool entry has a free slot: nearest reached node with one
            if (!dmask) {
                if ((rc = dalloc((void **)&dmask, (size_t)n)) || (rc = dalloc((void **)&dbest, 8))) return rc;
            }
            std::vector<unsigned char> hm((size_t)n);
            for (int64_t i = 0; i < n; ++i) hm[i] = reached[i] && deg[i] < R;
            unsigned long long init = ~0ull, hb = 0;
            NSG_HIP(hipMemcpy(dmask, hm.data(), (size_t)n, hipMemcpyHostToDevice));
            NSG_HIP(hipMemcpy(dbest, &init, 8, hipMemcpyHostToDevice));
            hipLaunchKernelGGL(nearest_masked_kernel, dim3(1024), dim3(256), 0, st, kix->base_f32,
                               kix->row_chunks_f32 * 4, d, n, base + (int64_t)u * d, dmask, dbest);
            NSG_HIP(hipMemcpyAsync(&hb, dbest, 8, hipMemcpyDeviceToHost, st));
            NSG_HIP(hipStreamSynchronize(st));
            if (hb == ~0ull) return fail(NSG_EUNSUPPORTED, "repair: no reached node has a free slot");
            w = (int64_t)(hb & 0xFFFFFFFFull);
        }
        g[(size_t)w * R + deg[w]] = u;
        NSG_HIP(hipMemcpy(graph_out + (size_t)w * R + deg[w], &u, 4, hipMemcpyHostToDevice));
        deg[w]++;
        added++;
        dfs_mark(g, R, u, reached, stack);
    }
    NSG_HIP(hipStreamSynchronize(st));
    *nav_out = nav;
    if (repair_edges) *repair_edges = added;
    return NSG_OK;
}
