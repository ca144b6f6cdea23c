// Search kernel template (Algorithm 1, one wavefront per query), shared by
// the per-format sources search_<format>.hip.
#pragma once
#include "wave.hpp"

namespace nsg {

struct KParams {
    RowTable tab;                // search-format rows (row_chunks chunks each)
    const float *scales;         // [row_chunks * EPC] (reduced formats)
    const float *rows_f32;       // FP32 rows for re-ranking, stride row_chunks_f32 * 4
    const uint32_t *graph;
    int R, R_pad;
    uint32_t n_rows;
    int d, row_chunks, row_chunks_f32;
    uint32_t start;
    const float *queries;
    int64_t nq;
    const int32_t *k_arr, *L_arr;
    int k_scalar, L_scalar, out_stride;
    uint32_t *out_ids;
    float *out_dist;
    int L_cap, L_alloc, hash_bits, lds_per_wave;
    int rerank;
    float rr_eta;                // the index's bound E (< 0: re-rank the whole pool)
    float rr_rho;                // relative rounding bound of a computed squared distance, (d + 4) 2^-24
    unsigned int *counter;
    const uint32_t *order;       // work slot -> query index (longest walks first), or NULL: identity
    int32_t *clamped;            // queries whose k / L were clamped into range, or NULL
    int64_t *hops, *ndist, *nedges;
    int max_hops;                // expansion budget for every query (0: none)
    uint32_t *pool_ids;
    float *pool_dist;
    int pool_stride;
    uint32_t *vis_ids;
    float *vis_dist;
    int32_t *vis_cnt;
    int vis_cap;
    int64_t self_offset;         // >= 0: query i is base row self_offset + i; its own row is visited at the end
    // partitioned index: search i is query i / shards in shard i % shards,
    // started at shard_starts[i % shards] (shards = 1: one graph, `start`)
    int shards;
    const uint32_t *shard_starts;
    // random initialization: query i's initial pool is the node set
    // init_ids[i][0 .. init_n) instead of {start} (init_n = 0: start only)
    const uint32_t *init_ids;
    int init_n;
    // expanded nodes in order, [nq][trace_cap] (all-options variant), or NULL
    uint32_t *trace_ids;
    int trace_cap;
    // learned early stop, fused into the search loop (see stop_decide)
    const float *stop_plan;      // network (kernel layout, see stop_decide)
    int32_t *budget;             // chosen budget per query (0: none), or NULL
    float *features;             // raw features [nq][kStopFeatures] after expansion s_hop, or NULL
    int s_in, s_hop, grid_n;
    int s_kind;                  // network form: NSG_STOP_SCALAR or NSG_STOP_QUERY
    uint64_t s_cps;              // decision checkpoints, 16 bits each from the low end (first = s_hop), 0 ends
    float calib_c;
    int learned;                 // 1: queries with L >= 16 stop at their budget
};

// exact FP32 squared distances over the FP32 rows (re-rank): 16 lanes per
// row, 16 rows per round with all their loads issued before the reductions
__device__ inline void rerank_dist(const KParams &p, const float *q, uint64_t *pool,
                                   int size, int lane) {
    const int g = lane >> 4, li = lane & 15;
    const int rc = p.row_chunks_f32;
    for (int r0 = 0; r0 < size; r0 += 16) {
        uint32_t id[4];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int r = r0 + 4 * u + g;
            ok[u] = r < size;
            id[u] = ok[u] ? key_id(pool[r]) : 0u;
            id[u] = id[u] < p.n_rows ? id[u] : 0u;
        }
        float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int ch = li; ch < rc; ch += 16) {
            float4 x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                x[u] = ok[u] ? reinterpret_cast<const float4 *>(p.rows_f32)[(int64_t)id[u] * rc + ch]
                             : make_float4(0.f, 0.f, 0.f, 0.f);
            float qc[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int j = ch * 4 + e;
                qc[e] = j < p.d ? q[j] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float xs[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float t = qc[e] - xs[e];
                    acc[u] = fmaf(t, t, acc[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = group_sum<16>(acc[u]);
        wave_sync();
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (li == 0 && ok[u]) pool[r0 + 4 * u + g] = mk_key(acc[u], id[u]);
        wave_sync();
    }
}

// Entries of the walk-sorted pool that the FP32 re-rank has to see for its
// top kq: the prefix with walk distance <= B.  With rho the relative bound of
// a computed squared distance (walk and re-rank alike), E the index's bound on
// | ||q - x|| - ||q - xhat|| | plus the decode's absolute rounding, and W the
// kq-th walk distance: the first kq entries have exact distance at most
// a = sqrt(W / (1 - rho)) + E, so re-rank distances at most
// (1 + rho) a^2; an entry with walk distance above
// B = (1 + rho) (sqrt((1 + rho) / (1 - rho)) a + E)^2 has exact distance
// above sqrt(B / (1 + rho)) - E and a re-rank distance strictly above
// (1 + rho) a^2, so it ranks after those kq entries whatever its id.  B gets
// a relative slack of 2^-12 for its own rounding.  Returns size when the bound
// is unknown or not finite.
__device__ __attribute__((noinline)) int rerank_prefix(const KParams &p, const uint64_t *pool, int size, int kq, int lane) {
    if (p.rr_eta < 0.0f || kq <= 0 || size <= kq) return kq <= 0 ? 0 : size;
    const float rho = p.rr_rho;
    const float W = key_dist(pool[kq - 1]);
    const float a = sqrtf(W / (1.0f - rho)) + p.rr_eta;
    const float t = sqrtf((1.0f + rho) / (1.0f - rho)) * a + p.rr_eta;
    const float B = (1.0f + rho) * t * t * (1.0f + 0x1p-12f);
    if (!(B < INFINITY)) return size;
    int m = 0;
    for (int j0 = 0; j0 < size; j0 += 64) {
        const int j = j0 + lane;
        m += __popcll(__ballot(j < size && key_dist(pool[j]) <= B));
    }
    return m > kq ? m : kq;
}

// ascending bitonic sort of pool[0..n) in LDS (n <= 1024), padding with KEY_NONE
__device__ inline void lds_sort(uint64_t *a, int n, int cap, int lane) {
    int np = 1;
    while (np < n) np <<= 1;
    for (int i = n + lane; i < np && i < cap; i += 64) a[i] = KEY_NONE;
    wave_sync();
    for (int k = 2; k <= np; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < np; i += 64) {
                int ixj = i ^ j;
                if (ixj > i) {
                    uint64_t x = a[i] & KEY_MASK, y = a[ixj] & KEY_MASK;
                    bool up = (i & k) == 0;
                    if ((x > y) == up) { uint64_t t = a[i]; a[i] = a[ixj]; a[ixj] = t; }
                }
            }
            wave_sync();
        }
    }
}

// Feature i (< kStopFeatures) of a search state, FP32.  dist(r) is the
// distance of pool rank r (r < size).
template <typename DistAt>
__device__ inline float stop_feature(int i, DistAt dist, int size, float dstart, int64_t ne, int64_t hops) {
    constexpr int ranks[10] = {1, 2, 4, 9, 14, 19, 29, 39, 59, 83};
    auto at = [&](int r) { return dist(r < size ? r : size - 1); };
    const float d0 = at(0);
    const float l0 = log1pf(d0);
    if (i == 0) return l0;
    if (i == 1) {
        const float d9 = at(9);
        return d9 > 0.0f ? d0 / d9 : 1.0f;
    }
    if (i == 2) return log1pf(dstart);
    if (i == 3) return l0 - log1pf(dstart);
    if (i < 14) {
        int r = 83;
#pragma unroll
        for (int j = 0; j < 10; ++j) r = (i - 4 == j) ? ranks[j] : r;
        return log1pf(at(r)) - l0;
    }
    return hops > 0 ? (float)ne / (float)hops : 0.0f;
}

// The budget for network output o: smallest grid value >= c * 2^o (the
// largest if none is), at least the decision hop; -1 / 0 for a non-finite o.
__device__ inline int stop_budget(const float *grid, int grid_n, float calib_c, int hop, float o, int lane,
                                  int *B) {
    const float t = calib_c * exp2f(o);
    if (!isfinite(t)) { *B = 0; return -1; }
    int gi = grid_n - 1;
    for (int b = 0; b < grid_n; b += 64) {
        const int i = b + lane;
        const uint64_t bm = __ballot(i < grid_n && grid[i] >= t);
        if (bm) { gi = b + __ffsll((long long)bm) - 1; break; }
    }
    const int v = (int)grid[gi];
    *B = v < hop ? hop : v;
    return gi;
}

typedef _Float16 half2_v __attribute__((ext_vector_type(2)));

__device__ inline uint32_t pack_half2(float a, float b) {
    const half2_v v = {(_Float16)a, (_Float16)b};
    return __builtin_bit_cast(uint32_t, v);
}

// sum + a.x * b.x + a.y * b.y: FP16 operands, FP32 accumulation (v_dot2_f32_f16)
__device__ inline float dot2_h(uint32_t a, uint32_t b, float sum) {
    return __builtin_amdgcn_fdot2(__builtin_bit_cast(half2_v, a), __builtin_bit_cast(half2_v, b), sum, false);
}

// The learned stop's decision for one query, after the decision hop: the
// features of its pool (pool[0 .. size) in LDS), the raw features to
// `features` (if given), then, if `plan` is given, the network and the
// budget.  Returns the grid index of the budget (-1: no budget for a
// non-finite output) and the budget in *B (at least hop; 0 for none).  Not
// inlined: it runs once per query and would otherwise hold registers through
// the whole search loop.  Lane j evaluates hidden unit j (units past h have
// zero weights); inputs and first-layer outputs reach every lane by lane
// reads; the transposed weights are read coalesced.
//  kind NSG_STOP_SCALAR, FP32: the kStopFeatures scalar features.  Plan:
//    W1T[in][64], W2T[64][64], b1[64], b2[64], W3[64], b3, mean[in],
//    inv_std[in], grid[grid_n].
//  kind NSG_STOP_QUERY, FP16 inference: inputs = the query's d values, then
//    ln(1 + d_0), d_0 / d_9 and the expansion count; z-scored in FP32 and
//    rounded to FP16, like the weights and the hidden activations; products
//    accumulate in FP32.  Plan (32-bit words): W1[(in + 1) / 2][64] (FP16
//    pairs: inputs 2i, 2i + 1 of unit j), W2[32][64] (FP16 pairs: units 2i,
//    2i + 1), b1[64], b2[64] (FP32), W3[64] (FP16 values held in FP32), b3,
//    mean[in], inv_std[in], grid[grid_n].
__device__ __attribute__((noinline)) int stop_decide(const float *plan, int kind, int in, int grid_n,
                                                     float calib_c, int hop, const uint64_t *pool, int size,
                                                     float dstart, int64_t ne, int64_t hops, const float *q, int d,
                                                     float *features, int lane, int *B) {
    float f = 0.0f;
    if (lane < kStopFeatures)
        f = stop_feature(lane, [&](int r) { return key_dist(pool[r]); }, size, dstart, ne, hops);
    if (features && lane < kStopFeatures) features[lane] = f;
    *B = 0;
    if (!plan) return -1;
    float o;
    if (kind == NSG_STOP_QUERY) {
        const uint32_t *W1 = reinterpret_cast<const uint32_t *>(plan);
        const int np1 = (in + 1) >> 1;
        const uint32_t *W2 = W1 + (size_t)np1 * 64;
        const float *b1 = reinterpret_cast<const float *>(W2 + 32 * 64), *b2 = b1 + 64, *W3 = b2 + 64;
        const float *b3 = W3 + 64, *mean = b3 + 1, *istd = mean + in, *grid = istd + in;
        const float d0 = key_dist(pool[0]), d9 = key_dist(pool[size > 9 ? 9 : size - 1]);
        auto input = [&](int i) -> float {
            const float v = i < d ? q[i] : (i == d ? log1pf(d0) : (i == d + 1 ? (d9 > 0.0f ? d0 / d9 : 1.0f)
                                                                               : (float)hops));
            return (v - mean[i]) * istd[i];
        };
        float s1 = b1[lane];
        for (int r = 0; r < np1; r += 64) {
            // lane l packs the input pair r + l
            const int pi = r + lane;
            uint32_t xw = 0;
            if (pi < np1) xw = pack_half2(input(2 * pi), 2 * pi + 1 < in ? input(2 * pi + 1) : 0.0f);
            const int cnt = np1 - r < 64 ? np1 - r : 64;
            for (int t = 0; t < cnt; ++t)
                s1 = dot2_h(W1[(size_t)(r + t) * 64 + lane], __builtin_amdgcn_readlane(xw, t), s1);
        }
        const float a1 = s1 > 0.0f ? s1 : 0.0f;
        // lane l < 32 packs hidden units 2l, 2l + 1
        const int l2 = 2 * (lane & 31);
        const uint32_t aw = pack_half2(__shfl(a1, l2), __shfl(a1, l2 + 1));
        float s2 = b2[lane];
#pragma unroll 8
        for (int t = 0; t < 32; ++t) s2 = dot2_h(W2[t * 64 + lane], __builtin_amdgcn_readlane(aw, t), s2);
        const float a2 = (float)(_Float16)(s2 > 0.0f ? s2 : 0.0f);
        o = W3[lane] * a2;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) o += __shfl_xor(o, off);
        o += b3[0];
        return stop_budget(grid, grid_n, calib_c, hop, o, lane, B);
    }
    const float *W1T = plan;
    const float *W2T = W1T + in * 64, *b1 = W2T + 64 * 64, *b2 = b1 + 64, *W3 = b2 + 64, *b3 = W3 + 64;
    const float *mean = b3 + 1, *istd = mean + in, *grid = istd + in;
    const float x = lane < in ? (f - mean[lane < in ? lane : 0]) * istd[lane < in ? lane : 0] : 0.0f;
    float s1 = b1[lane];
    for (int i = 0; i < in; ++i) {
        const float xi = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), i));
        s1 = fmaf(W1T[i * 64 + lane], xi, s1);
    }
    const float a1 = s1 > 0.0f ? s1 : 0.0f;
    float s2 = b2[lane];
#pragma unroll 8
    for (int k = 0; k < 64; ++k) {
        const float ak = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, a1), k));
        s2 = fmaf(W2T[k * 64 + lane], ak, s2);
    }
    const float a2 = s2 > 0.0f ? s2 : 0.0f;
    o = W3[lane] * a2;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) o += __shfl_xor(o, off);
    o += b3[0];
    return stop_budget(grid, grid_n, calib_c, hop, o, lane, B);
}

// MODE selects what is compiled in: 0 the plain search only; 1 also the
// learned early stop and the feature capture at the decision hop; 2 every
// option (visited recording, pool output, counters, own-row visit).  Options
// left out keep registers free for occupancy.
// NCH: pool chunks of 64 held in registers (NCH * 64 >= the pool capacity).
// Occupancy target: 5 waves per SIMD (<= 96 registers; a few cold values go
// to scratch, measured faster) for the 2-chunk pool when the query and its
// scales take at most 32 registers per lane (FP32 up to 4 chunks per lane,
// FP16 / BF16 up to 2); otherwise none, since wider queries would spill most
// of the loop's state.
template <int DT, int CPL>
constexpr int query_regs() { return CPL * Fmt<DT>::EPC * (DT == NSG_F32 ? 1 : 2); }
template <int DT, int LPR, int CPL, int MODE, int NCH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    NCH == 2 && MODE <= 1 && DT != NSG_E4M3 && query_regs<DT, CPL>() <= 32 ? 5 : 1)))
search_kernel(KParams p) {
    constexpr int EPC = Fmt<DT>::EPC;
    constexpr bool FULL = MODE == 2;
    constexpr bool STOP = MODE >= 1;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int wpb = blockDim.x >> 6;
    unsigned char *wbase = smem + (size_t)wave * p.lds_per_wave;
    uint64_t *pool = reinterpret_cast<uint64_t *>(wbase);
    uint32_t *hash = reinterpret_cast<uint32_t *>(pool + p.L_alloc);
    uint32_t *cid = hash + (1 << p.hash_bits);          // candidate ids
    float *cdist = reinterpret_cast<float *>(cid + kMaxR);   // and distances
    const int H = 1 << p.hash_bits;

    // work slots in launch order (the counter, or the wave's place in the
    // grid), mapped to queries through the order when one is given
    int64_t slot;
    if (p.counter) {
        unsigned int t = 0;
        if (lane == 0) t = atomicAdd(p.counter, 1u);
        slot = __builtin_amdgcn_readfirstlane((int)t);
    } else {
        slot = (int64_t)blockIdx.x * wpb + wave;
    }
    while (slot < p.nq) {
        const int64_t qi = p.order ? (int64_t)__builtin_amdgcn_readfirstlane((int)p.order[slot]) : slot;
        const int64_t qrow = p.shards > 1 ? qi / p.shards : qi;
        const float *q = p.queries + qrow * (int64_t)p.d;
        int kq = p.k_arr ? p.k_arr[qi] : p.k_scalar;
        int Lq = p.L_arr ? p.L_arr[qi] : p.L_scalar;
        if (p.clamped && lane == 0 && (kq < 0 || kq > p.out_stride || Lq < 1 || Lq > p.L_cap))
            atomicAdd(p.clamped, 1);
        kq = kq < 0 ? 0 : (kq > p.out_stride ? p.out_stride : kq);
        Lq = Lq < 1 ? 1 : (Lq > p.L_cap ? p.L_cap : Lq);
        const int Lcur = Lq;
        // expansion budget: the caller's, and after the decision hop the
        // learned one (the search stops early, never later, than plain)
        const int64_t base_cap = p.max_hops > 0 ? p.max_hops : INT64_MAX;
        int64_t hcap = base_cap;
        // decision hop: features (if captured) and the learned budget
        const bool learn_q = STOP && p.learned && Lq >= 16;
        bool decide = STOP && (learn_q || p.features != nullptr);
        int Bq = 0;
        int cpi = 0;                 // next decision checkpoint
        int64_t cph = p.s_hop;       // its expansion count

        // query chunks in registers, aligned with the row chunks this lane reads
        float qv[CPL][EPC], sc[CPL][EPC];
        {
            const int li = lane % LPR;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                int ch = li + c * LPR;
#pragma unroll
                for (int e = 0; e < EPC; ++e) {
                    int j = ch * EPC + e;
                    bool ok = ch < p.row_chunks && j < p.d;
                    qv[c][e] = ok ? q[j] : 0.0f;
                    sc[c][e] = (DT != NSG_F32 && ok) ? p.scales[j] : 0.0f;
                }
            }
        }
        for (int i = lane; i < H; i += 64) hash[i] = NSG_SENT;
        wave_sync();

        const uint32_t start = p.shards > 1 ? p.shard_starts[qi % p.shards] : p.start;
        int64_t hops = 0, nd = 0, ne = 0;
        int vcount = 0;
        const bool rec = FULL && p.vis_ids != nullptr;

        RegPool<NCH> P;
        rp_init<NCH>(P);
        float dstart;
        if (p.init_n <= 0) {
            // pool <- {start}
            if (lane == 0) { cid[0] = start; hash_insert(hash, p.hash_bits, start); }
            wave_sync();
            gather_dist<DT, LPR, CPL>(p.tab, qv, sc, cid, cdist, 1, lane);
            wave_sync();
            nd = 1;
            if (rec && lane == 0 && vcount < p.vis_cap) {
                p.vis_ids[qi * (int64_t)p.vis_cap + vcount] = start;
                p.vis_dist[qi * (int64_t)p.vis_cap + vcount] = cdist[0];
            }
            vcount = 1;
            dstart = cdist[0];
            rp_insert<NCH>(P, readfirstlane64(mk_key(cdist[0], start)), Lcur, lane);
        } else {
            // pool <- the query's given node set (random initialization),
            // each node visited once, in batches of 64 through the candidate
            // arrays; a repeated id is dropped by the filter or the merge
            const uint32_t *ini = p.init_ids + qrow * (int64_t)p.init_n;
            for (int b = 0; b < p.init_n; b += 64) {
                const uint32_t u0 = b + lane < p.init_n ? ini[b + lane] : NSG_SENT;
                const uint32_t u = u0 < p.tab.n_rows ? u0 : NSG_SENT;
                const bool nw = u != NSG_SENT && hash_insert(hash, p.hash_bits, u);
                const uint64_t bm = __ballot(nw);
                const int rank = __popcll(bm & ((1ull << lane) - 1ull));
                if (nw) cid[rank] = u;
                const int cnt = __popcll(bm);
                wave_sync();
                if (cnt > 0) {
                    gather_dist<DT, LPR, CPL>(p.tab, qv, sc, cid, cdist, cnt, lane);
                    wave_sync();
                    if (rec)
                        for (int r = lane; r < cnt; r += 64)
                            if (vcount + r < p.vis_cap) {
                                p.vis_ids[qi * (int64_t)p.vis_cap + vcount + r] = cid[r];
                                p.vis_dist[qi * (int64_t)p.vis_cap + vcount + r] = cdist[r];
                            }
                    merge_cands<NCH>(P, cid, cdist, cnt, Lcur, lane);
                    wave_sync();
                }
                nd += cnt;
                vcount += cnt;
            }
            dstart = P.size > 0 ? key_dist(rp_get<NCH>(P, 0)) : 0.0f;
        }
        for (;;) {
            if (hops >= hcap) break;
            // Algorithm 1: expand the first unchecked pool entry
            uint64_t pe;
            const int i = rp_first_unchecked<NCH>(P, &pe);
            if (i < 0) break;
            rp_mark_checked<NCH>(P, i);
            uint32_t v = key_id(pe);
            v = v < p.n_rows ? v : 0u;
            if (FULL && p.trace_ids && lane == 0 && hops < p.trace_cap)
                p.trace_ids[qi * (int64_t)p.trace_cap + hops] = v;   // expansion order
            ++hops;
            // neighbour ids (one coalesced row), visited filter, compaction
            const uint32_t *grow = p.graph + (int64_t)v * p.R_pad;
            const uint32_t row0 = lane < p.R ? grow[lane] : NSG_SENT;
            const uint32_t row1 = lane + 64 < p.R ? grow[lane + 64] : NSG_SENT;
            int cnt = 0;
            for (int b = 0; b < p.R; b += 64) {
                uint32_t u = b == 0 ? row0 : row1;
                ne += __popcll(__ballot(u != NSG_SENT));
                bool nw = u != NSG_SENT && hash_insert(hash, p.hash_bits, u);
                uint64_t bm = __ballot(nw);
                int rank = __popcll(bm & ((1ull << lane) - 1ull));
                if (nw) cid[cnt + rank] = u;
                cnt += __popcll(bm);
            }
            wave_sync();
            nd += cnt;
            if (cnt > 0) {
                gather_dist<DT, LPR, CPL>(p.tab, qv, sc, cid, cdist, cnt, lane);
                wave_sync();
                if (rec) {
                    for (int r = lane; r < cnt; r += 64)
                        if (vcount + r < p.vis_cap) {
                            p.vis_ids[qi * (int64_t)p.vis_cap + vcount + r] = cid[r];
                            p.vis_dist[qi * (int64_t)p.vis_cap + vcount + r] = cdist[r];
                        }
                }
                merge_cands<NCH>(P, cid, cdist, cnt, Lcur, lane);
                wave_sync();
            }
            vcount += cnt;
            if (decide && hops >= cph) {
                // after a decision checkpoint: features of the state (captured
                // at the first), the network, the budget; the latest decision
                // replaces the budget, and the next checkpoint is taken only
                // if the budget lets the search run past it
                rp_store<NCH>(P, pool, lane);
                wave_sync();
                stop_decide(learn_q ? p.stop_plan : nullptr, p.s_kind, p.s_in, p.grid_n, p.calib_c, (int)cph, pool,
                            P.size, dstart, ne, hops, q, p.d,
                            p.features && cpi == 0 ? p.features + qi * kStopFeatures : nullptr, lane, &Bq);
                Bq = __builtin_amdgcn_readfirstlane(Bq);
                if (learn_q) hcap = Bq > 0 && Bq < base_cap ? Bq : base_cap;
                ++cpi;
                const int64_t nxt = cpi < 4 ? (int64_t)((p.s_cps >> (16 * cpi)) & 0xFFFFu) : 0;
                decide = learn_q && nxt > 0 && nxt < hcap;
                cph = nxt;
                wave_sync();
            }
        }
        if (STOP && cpi == 0 && p.features) {
            // ended before the decision hop: no features
            for (int t = lane; t < kStopFeatures; t += 64) p.features[qi * kStopFeatures + t] = NAN;
        }
        if (STOP && p.budget && lane == 0) p.budget[qi] = Bq;
        rp_store<NCH>(P, pool, lane);
        const int size = P.size;
        wave_sync();
        if (FULL && p.self_offset >= 0) {
            // index build: also visit the query node's own row (its kNN list)
            const uint32_t self = (uint32_t)(p.self_offset + qi);
            const uint32_t *grow = p.graph + (int64_t)self * p.R_pad;
            int cnt = 0;
            for (int b = 0; b < p.R; b += 64) {
                int j = b + lane;
                uint32_t u = j < p.R ? grow[j] : NSG_SENT;
                bool nw = u != NSG_SENT && hash_insert(hash, p.hash_bits, u);
                uint64_t bm = __ballot(nw);
                int rank = __popcll(bm & ((1ull << lane) - 1ull));
                if (nw) cid[cnt + rank] = u;
                cnt += __popcll(bm);
            }
            wave_sync();
            if (cnt > 0) {
                gather_dist<DT, LPR, CPL>(p.tab, qv, sc, cid, cdist, cnt, lane);
                wave_sync();
                if (rec)
                    for (int r = lane; r < cnt; r += 64)
                        if (vcount + r < p.vis_cap) {
                            p.vis_ids[qi * (int64_t)p.vis_cap + vcount + r] = cid[r];
                            p.vis_dist[qi * (int64_t)p.vis_cap + vcount + r] = cdist[r];
                        }
                vcount += cnt;
            }
        }
        if (FULL && p.pool_ids) {
            for (int j = lane; j < p.pool_stride; j += 64) {
                bool ok = j < size;
                p.pool_ids[qi * (int64_t)p.pool_stride + j] = ok ? key_id(pool[j]) : NSG_SENT;
                p.pool_dist[qi * (int64_t)p.pool_stride + j] = ok ? key_dist(pool[j]) : INFINITY;
            }
        }
        if (p.rerank) {
            wave_sync();
            const int m = rerank_prefix(p, pool, size, kq, lane);
            rerank_dist(p, q, pool, m, lane);
            lds_sort(pool, m, p.L_alloc, lane);
        }
        for (int j = lane; j < kq; j += 64) {
            bool ok = j < size;
            p.out_ids[qi * (int64_t)p.out_stride + j] = ok ? key_id(pool[j]) : NSG_SENT;
            p.out_dist[qi * (int64_t)p.out_stride + j] = ok ? key_dist(pool[j]) : INFINITY;
        }
        if (FULL && lane == 0) {
            if (p.hops) p.hops[qi] = hops;
            if (p.ndist) p.ndist[qi] = nd;
            if (p.nedges) p.nedges[qi] = ne;
            if (p.vis_cnt) p.vis_cnt[qi] = vcount;
        }
        wave_sync();
        if (!p.counter) break;
        unsigned int t = 0;
        if (lane == 0) t = atomicAdd(p.counter, 1u);
        slot = __builtin_amdgcn_readfirstlane((int)t);
    }
}


typedef void (*kfn_t)(KParams);

// Kernel for a layout (lanes per row, chunks per lane), a MODE and nch pool
// chunks of 64 held in registers (2, 4, 6 or 8: pool capacity <= 128, 256,
// 384, 512).
// Each per-format source instantiates one MODE.
template <int DT, int MODE>
static kfn_t pick_kernel_t(int lpr, int cpl, int nch) {
#define NSG_K(L_, C_)                                                                   \
    if (lpr == L_ && cpl == C_)                                                         \
        return nch <= 2 ? search_kernel<DT, L_, C_, MODE, 2>                          \
                        : nch <= 4 ? search_kernel<DT, L_, C_, MODE, 4>                 \
                        : nch <= 6 ? search_kernel<DT, L_, C_, MODE, 6> : search_kernel<DT, L_, C_, MODE, 8>;
    NSG_K(8, 1) NSG_K(8, 2) NSG_K(8, 4)
    NSG_K(16, 1) NSG_K(16, 2) NSG_K(16, 4)
    NSG_K(32, 1) NSG_K(32, 2) NSG_K(32, 4)
    NSG_K(64, 1) NSG_K(64, 2) NSG_K(64, 4)
#undef NSG_K
    return nullptr;
}

}  // namespace nsg
