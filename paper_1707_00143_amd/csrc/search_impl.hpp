// Search kernel template (Algorithm 1, one wavefront per query), shared by
// the per-format sources search_<format>.hip.
#pragma once
#include "wave.hpp"

namespace nsg {

struct KParams {
    const uint4 *rows;           // search-format rows, stride row_chunks
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
    int L_cap, L_alloc, hash_bits, lds_per_wave, feat_cap;
    int rerank;
    unsigned int *counter;
    int64_t *hops, *ndist, *nedges;
    int32_t *budget;             // chosen expansion budget per query (learned stop), or NULL
    int max_hops;                // expansion budget for every query (0: none)
    float *features;
    uint32_t *pool_ids;
    float *pool_dist;
    int pool_stride;
    uint32_t *vis_ids;
    float *vis_dist;
    int32_t *vis_cnt;
    int vis_cap;
    int64_t self_offset;         // >= 0: query i is base row self_offset + i; its own row is visited at the end
    // learned early stop
    const float *stop_f32;       // mean[in], inv_std[in], b1[h], b2[h], b3
    const _Float16 *stop_w;      // W1T[in][h], W2T[h][h], W3[h]
    const float *grid;
    int s_in, s_h, s_hop, grid_n;
    float calib_c;
    int learned;
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

// early-stop features after the decision expansion: the query, the best pool
// distance, the ratio of the 1st to the 10th pool distance, the hop count.
// Written raw to p.features (if given and WF) and z-scored into xbuf (if learned).
template <bool WF>
__device__ inline void stop_features(const KParams &p, const float *q, float d0, float d9,
                                     int64_t hops, float *xbuf, int lane, int64_t qi) {
    const int in = p.d + 3;
    const float *sf = p.stop_f32;
    asm volatile("" : "+s"(sf));   // not hoisted out of the search loop
    for (int i = lane; i < in; i += 64) {
        float f;
        if (i < p.d) f = q[i];
        else if (i == p.d) f = d0;
        else if (i == p.d + 1) f = d9 > 0.0f ? d0 / d9 : 1.0f;
        else f = (float)hops;
        if (WF && p.features) p.features[qi * (int64_t)in + i] = f;
        if (p.learned) xbuf[i] = (f - sf[i]) * sf[in + i];
    }
    wave_sync();
}

// learned early stop: z-scored features in xbuf -> MLP (FP16 weights, FP32
// accumulate) -> y = log2 pool size -> L_hat on the grid
__device__ inline int stop_predict(const KParams &p, const float *xbuf, int lane) {
    const int in = p.s_in, h = p.s_h;
    // the model is the same for every query: opaque base pointers keep the
    // compiler from hoisting its loads out of the search loop (they would
    // hold registers through every expansion)
    const float *sf = p.stop_f32;
    const _Float16 *W1T = p.stop_w;
    asm volatile("" : "+s"(sf), "+s"(W1T));
    const float *b1 = sf + 2 * in;
    const float *b2 = b1 + h;
    const float b3 = b2[h];
    const _Float16 *W2T = W1T + (int64_t)in * h;
    const _Float16 *W3 = W2T + (int64_t)h * h;
    float a1 = 0.0f;
    if (lane < h) {
        float s = b1[lane];
#pragma unroll 4
        for (int i = 0; i < in; ++i) s = fmaf((float)W1T[(int64_t)i * h + lane], xbuf[i], s);
        a1 = s > 0.0f ? s : 0.0f;
    }
    float a2 = 0.0f;
    {
        float s = lane < h ? b2[lane] : 0.0f;
#pragma unroll 4
        for (int j = 0; j < h; ++j) {
            float aj = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, a1), j));
            if (lane < h) s = fmaf((float)W2T[j * h + lane], aj, s);
        }
        a2 = (lane < h && s > 0.0f) ? s : 0.0f;
    }
    float o = lane < h ? (float)W3[lane] * a2 : 0.0f;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) o += __shfl_xor(o, off);
    o += b3;
    wave_sync();
    if (!isfinite(o)) return 0x7FFFFFFF;   // no budget: the plain search
    float t = p.calib_c * exp2f(o);
    int pick = p.grid_n > 0 ? (int)p.grid[p.grid_n - 1] : 0x7FFFFFFF;
    for (int b = 0; b < p.grid_n; b += 64) {
        int i = b + lane;
        bool ge = i < p.grid_n && p.grid[i] >= t;
        uint64_t bm = __ballot(ge);
        if (bm) { pick = (int)p.grid[b + __ffsll((long long)bm) - 1]; break; }
    }
    return pick < p.s_hop ? p.s_hop : pick;
}

// MODE selects what is compiled in: 0 the plain search only; 1 also the
// learned early stop (and the chosen budget output); 2 every option
// (feature capture, visited recording, pool output, counters,
// own-row visit).  Options left out keep registers free for occupancy.
// NCH: pool chunks of 64 held in registers (NCH * 64 >= L_alloc).
// Occupancy targets for the common 2-chunk pool: the plain search at 5 waves
// per SIMD (<= 96 registers; a few cold values go to scratch, measured
// faster), the learned-stop variant at 4 (<= 128; it needs 130 otherwise).
template <int DT, int LPR, int CPL, int MODE, int NCH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NCH == 2 ? (MODE == 0 ? 5 : (MODE == 1 ? 4 : 1)) : 1)))
search_kernel(KParams p) {
    constexpr int EPC = Fmt<DT>::EPC;
    constexpr bool FULL = MODE == 2;
    constexpr bool LEARN = MODE >= 1;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int wpb = blockDim.x >> 6;
    unsigned char *wbase = smem + (size_t)wave * p.lds_per_wave;
    uint64_t *pool = reinterpret_cast<uint64_t *>(wbase);
    uint32_t *hash = reinterpret_cast<uint32_t *>(pool + p.L_alloc);
    uint32_t *cid = hash + (1 << p.hash_bits);          // candidate ids
    float *cdist = reinterpret_cast<float *>(cid + kMaxR);   // and distances
    float *xbuf = cdist + kMaxR;                              // early-stop features
    const int H = 1 << p.hash_bits;

    int64_t qi;
    if (p.counter) {
        unsigned int t = 0;
        if (lane == 0) t = atomicAdd(p.counter, 1u);
        qi = __builtin_amdgcn_readfirstlane((int)t);
    } else {
        qi = (int64_t)blockIdx.x * wpb + wave;
    }
    while (qi < p.nq) {
        const float *q = p.queries + qi * (int64_t)p.d;
        int kq = p.k_arr ? p.k_arr[qi] : p.k_scalar;
        kq = kq < 0 ? 0 : (kq > p.out_stride ? p.out_stride : kq);
        int Lq = p.L_arr ? p.L_arr[qi] : p.L_scalar;
        Lq = Lq < 1 ? 1 : (Lq > p.L_cap ? p.L_cap : Lq);
        const bool learned = LEARN && p.learned && Lq >= 16;
        const int Lcur = Lq;
        // expansion budget: the caller's, and after the decision hop the
        // learned one (the search stops early, never later, than plain)
        int64_t hcap = p.max_hops > 0 ? p.max_hops : INT64_MAX;
        int chosen = 0;

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

        const uint32_t start = p.start;
        int64_t hops = 0, nd = 0, ne = 0;
        int vcount = 0;
        const bool rec = FULL && p.vis_ids != nullptr;

        // pool <- {start}
        if (lane == 0) { cid[0] = start; hash_insert(hash, p.hash_bits, start); }
        wave_sync();
        gather_dist<DT, LPR, CPL>(p.rows, p.row_chunks, p.n_rows, qv, sc, cid, cdist, 1, lane);
        wave_sync();
        nd = 1;
        if (rec && lane == 0 && vcount < p.vis_cap) {
            p.vis_ids[qi * (int64_t)p.vis_cap + vcount] = start;
            p.vis_dist[qi * (int64_t)p.vis_cap + vcount] = cdist[0];
        }
        vcount = 1;
        RegPool<NCH> P;
        rp_init<NCH>(P);
        rp_insert<NCH>(P, readfirstlane64(mk_key(cdist[0], start)), Lcur, lane);
        bool stopped = !learned && !(FULL && p.features);   // true once the decision hop has passed
        for (;;) {
            if (hops >= hcap) break;
            // Algorithm 1: expand the first unchecked pool entry
            uint64_t pe;
            const int i = rp_first_unchecked<NCH>(P, &pe);
            if (i < 0) break;
            rp_mark_checked<NCH>(P, i);
            uint32_t v = key_id(pe);
            v = v < p.n_rows ? v : 0u;
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
                gather_dist<DT, LPR, CPL>(p.rows, p.row_chunks, p.n_rows, qv, sc, cid, cdist, cnt, lane);
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
            if (LEARN && !stopped && hops >= p.s_hop) {
                stopped = true;
                const float d0 = key_dist(rp_get<NCH>(P, 0));
                const float d9 = key_dist(rp_get<NCH>(P, P.size > 10 ? 9 : P.size - 1));
                stop_features<FULL>(p, q, d0, d9, hops, xbuf, lane, qi);
                if (learned) {
                    chosen = stop_predict(p, xbuf, lane);
                    hcap = chosen < hcap ? chosen : hcap;
                }
            }
        }
        if (FULL && !stopped && p.features) {
            // ended before the decision point: no features (the result is the plain one)
            for (int t = lane; t < p.d + 3; t += 64) p.features[qi * (int64_t)(p.d + 3) + t] = NAN;
        }
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
                gather_dist<DT, LPR, CPL>(p.rows, p.row_chunks, p.n_rows, qv, sc, cid, cdist, cnt, lane);
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
            rerank_dist(p, q, pool, size, lane);
            lds_sort(pool, size, p.L_alloc, lane);
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
        if (LEARN && lane == 0 && p.budget) p.budget[qi] = chosen;
        wave_sync();
        if (!p.counter) break;
        unsigned int t = 0;
        if (lane == 0) t = atomicAdd(p.counter, 1u);
        qi = __builtin_amdgcn_readfirstlane((int)t);
    }
}


typedef void (*kfn_t)(KParams);

// Kernel for a layout (lanes per row, chunks per lane), a MODE and nch pool
// chunks of 64 held in registers (2, 4 or 8: pool capacity <= 128, 256, 512).
// Each per-format source instantiates one MODE.
template <int DT, int MODE>
static kfn_t pick_kernel_t(int lpr, int cpl, int nch) {
#define NSG_K(L_, C_)                                                                   \
    if (lpr == L_ && cpl == C_)                                                         \
        return nch <= 2 ? search_kernel<DT, L_, C_, MODE, 2>                          \
                        : nch <= 4 ? search_kernel<DT, L_, C_, MODE, 4> : search_kernel<DT, L_, C_, MODE, 8>;
    NSG_K(8, 1) NSG_K(8, 2) NSG_K(8, 4)
    NSG_K(16, 1) NSG_K(16, 2) NSG_K(16, 4)
    NSG_K(32, 1) NSG_K(32, 2) NSG_K(32, 4)
    NSG_K(64, 1) NSG_K(64, 2) NSG_K(64, 4)
#undef NSG_K
    return nullptr;
}

}  // namespace nsg
