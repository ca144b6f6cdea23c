// Index construction on the GPU (Algorithm 2, NSGbuild(G, l, m)).
//
//  1. centroid of the base (compensated FP32 column sums)
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
//     has a free slot to u, continue the DFS from u.  The searches run in
//     speculative batches that give the same links as one search at a time.
#include "wave.hpp"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
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
            if (id != v && id < p.n_rows) {
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

// Squared distances from every node v of [node0, node0 + nb) to the ids of
// its kNN row knn[v][0 .. K) (one wave per node, the search's gather with the
// node's own row as query); sentinel entries get +inf.
template <int LPR, int CPL>
__global__ void __launch_bounds__(256) knn_dist_kernel(RowTable tab, const uint32_t *knn, int K, int64_t node0,
                                                       int64_t nb, float *dist) {
    __shared__ uint32_t cid_s[4][kMaxR];
    __shared__ float cd_s[4][kMaxR];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t b = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (b >= nb) return;
    const int64_t v = node0 + b;
    constexpr int EPC = 4;
    float qv[CPL][EPC], sc[CPL][EPC];
    const int li = lane % LPR;
    const uint4 *vrow = reinterpret_cast<const uint4 *>(tab.base) + v * tab.row_chunks;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int ch = li + c * LPR;
        const uint4 r = ch < tab.row_chunks ? vrow[ch] : make_uint4(0u, 0u, 0u, 0u);
        qv[c][0] = __uint_as_float(r.x); qv[c][1] = __uint_as_float(r.y);
        qv[c][2] = __uint_as_float(r.z); qv[c][3] = __uint_as_float(r.w);
#pragma unroll
        for (int e = 0; e < EPC; ++e) sc[c][e] = 0.0f;
    }
    const uint32_t *row = knn + v * K;
    for (int j = lane; j < K; j += 64) {
        const uint32_t u = row[j];
        cid_s[wave][j] = u < tab.n_rows ? u : 0u;
    }
    wave_sync();
    gather_dist<NSG_F32, LPR, CPL>(tab, qv, sc, cid_s[wave], cd_s[wave], K, lane);
    wave_sync();
    for (int j = lane; j < K; j += 64) dist[v * K + j] = row[j] < tab.n_rows ? cd_s[wave][j] : INFINITY;
}

__global__ void fill_i32_kernel(int32_t *p, int64_t cnt, int32_t v) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = v;
}

typedef void (*kdfn_t)(RowTable, const uint32_t *, int, int64_t, int64_t, float *);
static kdfn_t pick_knn_dist(int lpr, int cpl) {
#define NSG_D(L_, C_) if (lpr == L_ && cpl == C_) return knn_dist_kernel<L_, C_>;
    NSG_D(8, 1) NSG_D(8, 2) NSG_D(8, 4) NSG_D(16, 1) NSG_D(16, 2) NSG_D(16, 4)
    NSG_D(32, 1) NSG_D(32, 2) NSG_D(32, 4) NSG_D(64, 1) NSG_D(64, 2) NSG_D(64, 4)
#undef NSG_D
    return nullptr;
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

// rows ids[b] of base[n][d] -> out[b][d] (one block per row)
__global__ void gather_rows_kernel(const float *base, int d, const uint32_t *ids, float *out) {
    const int64_t b = blockIdx.x;
    const float *src = base + (int64_t)ids[b] * d;
    for (int j = threadIdx.x; j < d; j += blockDim.x) out[b * d + j] = src[j];
}

// graph[pos[i]] = val[i], i < m
__global__ void scatter_u32_kernel(uint32_t *graph, const uint64_t *pos, const uint32_t *val, int64_t m) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) graph[pos[i]] = val[i];
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

// Progress lines on stderr when the environment variable NSG_LOG is set to a
// non-empty value other than "0" (long builds: one line per phase and per
// eighth of the search-collect batches).
static bool build_log_on() {
    const char *e = getenv("NSG_LOG");
    return e && *e && !(e[0] == '0' && e[1] == 0);
}
#define BUILD_LOG(...)                                   \
    do {                                                 \
        if (log_on) {                                    \
            fprintf(stderr, "[nsg_build] " __VA_ARGS__); \
            fputc('\n', stderr);                         \
            fflush(stderr);                              \
        }                                                \
    } while (0)

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
    const bool log_on = build_log_on();
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
    BUILD_LOG("n=%lld d=%d: navigating node %u", (long long)n, d, nav);
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
        const int64_t nbat = (n + B - 1) / B, bi = v0 / B + 1;
        if (bi == nbat || (bi * 8) / nbat != ((bi - 1) * 8) / nbat)
            BUILD_LOG("search-collect + select: %lld of %lld nodes", (long long)(v0 + nb), (long long)n);
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
    if (log_on) {
        int64_t un = 0;
        for (int64_t v = 0; v < n; ++v) un += !reached[v];
        BUILD_LOG("repair: %lld nodes not reached from the navigating node", (long long)un);
    }
    // The repair visits the unreached nodes in increasing id order, each
    // time searching the graph as repaired so far (as the paper's sequential
    // step does).  To avoid one launch per node, the searches of the next B
    // unreached nodes run speculatively in one launch on the graph at that
    // moment, recording the nodes each search expands; then the nodes are
    // processed in order: a search whose expanded nodes' rows did not change
    // since the launch is exactly the search the sequential order would run
    // (Algorithm 1 reads only the rows of the nodes it expands), otherwise it
    // is run again on the current graph.
    const int64_t SB = std::max<int64_t>(64, std::min<int64_t>(4096, n / 256));   // nodes per batch
    const int TC = 8 * Lb + 64;                                                  // recorded expansions
    uint32_t *pool_id = nullptr, *cand_d = nullptr, *trace_d = nullptr, *edge_val = nullptr;
    uint64_t *edge_pos = nullptr;
    float *pool_d = nullptr, *qbuf = nullptr;
    int64_t *hops_d = nullptr;
    unsigned char *dmask = nullptr;
    unsigned long long *dbest = nullptr;
    if ((rc = dalloc((void **)&pool_id, sizeof(uint32_t) * SB * Lb)) ||
        (rc = dalloc((void **)&pool_d, sizeof(float) * SB * Lb)) ||
        (rc = dalloc((void **)&cand_d, sizeof(uint32_t) * SB)) ||
        (rc = dalloc((void **)&trace_d, sizeof(uint32_t) * SB * TC)) ||
        (rc = dalloc((void **)&hops_d, sizeof(int64_t) * SB)) ||
        (rc = dalloc((void **)&qbuf, sizeof(float) * SB * d)) ||
        (rc = dalloc((void **)&edge_pos, sizeof(uint64_t) * SB)) ||
        (rc = dalloc((void **)&edge_val, sizeof(uint32_t) * SB)))
        return rc;
    std::vector<uint32_t> hpool((size_t)SB * Lb), htrace((size_t)SB * TC), cand, one_pool((size_t)Lb);
    std::vector<int64_t> hhops((size_t)SB);
    std::vector<unsigned char> changed((size_t)n, 0);
    std::vector<uint32_t> changed_list, pend_val;
    std::vector<uint64_t> pend_pos;
    int64_t added = 0, reruns = 0;
    int64_t scan = 0;
    // write the edges added since the last flush into the device graph
    auto flush = [&]() -> int {
        if (pend_pos.empty()) return NSG_OK;
        const int64_t m = (int64_t)pend_pos.size();
        for (int64_t o = 0; o < m; o += SB) {
            const int64_t c = std::min<int64_t>(SB, m - o);
            NSG_HIP(hipMemcpyAsync(edge_pos, pend_pos.data() + o, 8 * c, hipMemcpyHostToDevice, st));
            NSG_HIP(hipMemcpyAsync(edge_val, pend_val.data() + o, 4 * c, hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(scatter_u32_kernel, dim3((unsigned)((c + 255) / 256)), dim3(256), 0, st, graph_out,
                               edge_pos, edge_val, c);
            NSG_HIP(hipGetLastError());
            NSG_HIP(hipStreamSynchronize(st));
        }
        pend_pos.clear();
        pend_val.clear();
        return NSG_OK;
    };
    // Algorithm 1 on the current device graph for the nodes ids[0 .. m),
    // final pools (Lb) and expansion traces to the host
    auto run_searches = [&](const uint32_t *ids, int64_t m, uint32_t *pools, uint32_t *traces, int64_t *hops) -> int {
        NSG_HIP(hipMemcpyAsync(cand_d, ids, 4 * m, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)m), dim3(256), 0, st, base, d, cand_d, qbuf);
        NSG_HIP(hipGetLastError());
        SearchArgs r = a;
        r.graph_override = graph_out;
        r.R_override = R;
        r.Rpad_override = R;
        r.start_override = nav;
        r.queries = qbuf;
        r.nq = m;
        r.L_cap = Lb;
        r.L_scalar = Lb;
        r.hash_bits = default_hash_bits(Lb);
        r.pool_ids = pool_id;
        r.pool_dist = pool_d;
        r.pool_stride = Lb;
        r.trace_ids = traces ? trace_d : nullptr;
        r.trace_cap = TC;
        r.hops = hops ? hops_d : nullptr;
        int rc2 = launch_search(r);
        if (rc2) return rc2;
        NSG_HIP(hipMemcpyAsync(pools, pool_id, sizeof(uint32_t) * m * Lb, hipMemcpyDeviceToHost, st));
        if (traces) NSG_HIP(hipMemcpyAsync(traces, trace_d, sizeof(uint32_t) * m * TC, hipMemcpyDeviceToHost, st));
        if (hops) NSG_HIP(hipMemcpyAsync(hops, hops_d, sizeof(int64_t) * m, hipMemcpyDeviceToHost, st));
        NSG_HIP(hipStreamSynchronize(st));
        return NSG_OK;
    };
    auto t_log = std::chrono::steady_clock::now();
    int64_t batches = 0;
    for (;;) {
        if (log_on && std::chrono::steady_clock::now() - t_log > std::chrono::seconds(10)) {
            t_log = std::chrono::steady_clock::now();
            BUILD_LOG("repair: %lld batches, %lld edges added, next unreached id >= %lld", (long long)batches,
                      (long long)added, (long long)scan);
        }
        ++batches;
        // the next SB unreached nodes in id order, searched together
        cand.clear();
        for (int64_t v = scan; v < n && (int64_t)cand.size() < SB; ++v)
            if (!reached[v]) cand.push_back((uint32_t)v);
        if (cand.empty()) break;
        scan = cand.back() + 1;
        const int64_t m = (int64_t)cand.size();
        if ((rc = run_searches(cand.data(), m, hpool.data(), htrace.data(), hhops.data()))) return rc;
        for (uint32_t c : changed_list) changed[c] = 0;
        changed_list.clear();
        for (int64_t j = 0; j < m; ++j) {
            const uint32_t u = cand[j];
            if (reached[u]) continue;
            // the speculative search stands if none of the nodes it expanded
            // got an edge since the launch
            bool valid = hhops[j] <= TC;
            for (int64_t t = 0; valid && t < hhops[j]; ++t) valid = !changed[htrace[(size_t)j * TC + t]];
            const uint32_t *pool = hpool.data() + (size_t)j * Lb;
            if (!valid) {
                if ((rc = flush())) return rc;
                if ((rc = run_searches(&u, 1, one_pool.data(), nullptr, nullptr))) return rc;
                pool = one_pool.data();
                ++reruns;
            }
            int64_t w = -1;
            for (int t = 0; t < Lb; ++t) {
                uint32_t c = pool[t];
                if (c == NSG_SENT) break;
                if (reached[c] && deg[c] < R) { w = c; break; }
            }
            if (w < 0) {
                // no pool entry has a free slot: nearest reached node with one
                if (!dmask) {
                    if ((rc = dalloc((void **)&dmask, (size_t)n)) || (rc = dalloc((void **)&dbest, 8))) return rc;
                }
                std::vector<unsigned char> hm((size_t)n);
                for (int64_t i2 = 0; i2 < n; ++i2) hm[i2] = reached[i2] && deg[i2] < R;
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
            pend_pos.push_back((uint64_t)w * R + deg[w]);
            pend_val.push_back(u);
            deg[w]++;
            if (!changed[w]) {
                changed[w] = 1;
                changed_list.push_back((uint32_t)w);
            }
            added++;
            dfs_mark(g, R, u, reached, stack);
        }
        if ((rc = flush())) return rc;
    }
    BUILD_LOG("repair: %lld edges added, %lld of the batched searches run again", (long long)added,
              (long long)reruns);
    NSG_HIP(hipStreamSynchronize(st));
    *nav_out = nav;
    if (repair_edges) *repair_edges = added;
    return NSG_OK;
}

extern "C" int nsg_build_naive(const float *base, int64_t n, int32_t d, const uint32_t *knn, int32_t K,
                               int32_t R, uint32_t *graph_out, void *stream) {
    clear_error();
    if (!base || !knn || !graph_out) return fail(NSG_EINVAL, "NULL pointer");
    if (n < 2 || n >= ((int64_t)1 << 31)) return fail(NSG_EINVAL, "n out of range");
    if (K < 1 || K > kMaxR) return fail(NSG_EINVAL, "K=%d out of range [1, %d]", K, kMaxR);
    if (R < 1 || R > kMaxR) return fail(NSG_EINVAL, "R out of range");
    hipStream_t st = (hipStream_t)stream;
    // the kNN graph as an index: padded FP32 rows (with the gather tail) and
    // validation of every entry
    nsg_index *kix = nullptr;
    int rc = nsg_load_index(base, n, d, knn, K, 0, NSG_F32, nullptr, stream, &kix);
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
        if (hipMalloc(ptr, bytes) != hipSuccess) return fail(NSG_ENOMEM, "allocation of %zu bytes failed", bytes);
        guard.bufs.push_back(*ptr);
        return NSG_OK;
    };
    const int64_t B = std::min<int64_t>(n, 65536);
    float *dist = nullptr;
    int32_t *cnt = nullptr;
    if ((rc = dalloc((void **)&dist, sizeof(float) * n * K)) || (rc = dalloc((void **)&cnt, sizeof(int32_t) * B)))
        return rc;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, cnt, B, K);
    int lpr, cpl;
    pick_layout(kix->row_chunks_f32, 4, &lpr, &cpl);
    kdfn_t dfn = pick_knn_dist(lpr, cpl);
    selfn_t sfn = pick_select(lpr, cpl);
    if (!dfn || !sfn) return fail(NSG_EUNSUPPORTED, "no kernel for d=%d", d);
    RowTable tab;
    tab.base = reinterpret_cast<const unsigned char *>(kix->base_f32);
    tab.row_bytes = (uint32_t)kix->row_chunks_f32 * 16u;
    tab.n_rows = (uint32_t)n;
    tab.row_chunks = kix->row_chunks_f32;
    int C_alloc = 1;
    while (C_alloc < K) C_alloc <<= 1;
    SelParams sp{};
    sp.tab = tab;
    sp.row_chunks = kix->row_chunks_f32;
    sp.n_rows = (uint32_t)n;
    sp.vis_cnt = cnt;
    sp.vis_cap = K;
    sp.C = K;
    sp.C_alloc = C_alloc;
    sp.m = R;
    sp.graph = graph_out;
    sp.lds_per_wave = (int)(((size_t)C_alloc * 8 + 32 * 8 + kMaxR * 4 + kMaxR * 4 + 15) & ~(size_t)15);
    const int wpb = 4;
    for (int64_t v0 = 0; v0 < n; v0 += B) {
        const int64_t nb = std::min<int64_t>(B, n - v0);
        hipLaunchKernelGGL(dfn, dim3((unsigned)((nb + wpb - 1) / wpb)), dim3(64 * wpb), 0, st, tab, knn, K, v0, nb,
                           dist);
        sp.vis_ids = knn + v0 * K;
        sp.vis_dist = dist + v0 * K;
        sp.node0 = v0;
        sp.nb = nb;
        hipLaunchKernelGGL(sfn, dim3((unsigned)((nb + wpb - 1) / wpb)), dim3(64 * wpb),
                           (size_t)sp.lds_per_wave * wpb, st, sp);
        NSG_HIP(hipGetLastError());
    }
    NSG_HIP(hipStreamSynchronize(st));
    return NSG_OK;
}
