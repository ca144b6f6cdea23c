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
    int prefetch;
    unsigned int *counter;
    int64_t *hops, *ndist, *nedges;
    int32_t *L_used;
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
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int off = 8; off > 0; off >>= 1) acc[u] += __shfl_xor(acc[u], off);
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
// Written raw to p.features (if given) and z-scored into xbuf (if learned).
__device__ inline void stop_features(const KParams &p, const float *q, const uint64_t *pool,
                                     int size, int64_t hops, float *xbuf, int lane, int64_t qi) {
    const int in = p.d + 3;
    const float d0 = key_dist(pool[0]);
    const float d9 = key_dist(pool[size > 10 ? 9 : size - 1]);
    for (int i = lane; i < in; i += 64) {
        float f;
        if (i < p.d) f = q[i];
        else if (i == p.d) f = d0;
        else if (i == p.d + 1) f = d9 > 0.0f ? d0 / d9 : 1.0f;
        else f = (float)hops;
        if (p.features) p.features[qi * (int64_t)in + i] = f;
        if (p.learned) xbuf[i] = (f - p.stop_f32[i]) * p.stop_f32[in + i];
    }
    wave_sync();
}

// learned early stop: z-scored features in xbuf -> MLP (FP16 weights, FP32
// accumulate) -> y = log2 pool size -> L_hat on the grid
__device__ inline int stop_predict(const KParams &p, int Lq, int kq, const float *xbuf, int lane) {
    const int in = p.s_in, h = p.s_h;
    const float *b1 = p.stop_f32 + 2 * in;
    const float *b2 = b1 + h;
    const float b3 = b2[h];
    const _Float16 *W1T = p.stop_w;
    const _Float16 *W2T = W1T + (int64_t)in * h;
    const _Float16 *W3 = W2T + (int64_t)h * h;
    float a1 = 0.0f;
    if (lane < h) {
        float s = b1[lane];
#pragma unroll 16
        for (int i = 0; i < in; ++i) s = fmaf((float)W1T[(int64_t)i * h + lane], xbuf[i], s);
        a1 = s > 0.0f ? s : 0.0f;
    }
    float a2 = 0.0f;
    {
        float s = lane < h ? b2[lane] : 0.0f;
#pragma unroll 16
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
    if (!isfinite(o)) return Lq;
    float t = p.calib_c * exp2f(o);
    int pick = p.grid_n > 0 ? (int)p.grid[p.grid_n - 1] : kMaxL;
    for (int b = 0; b < p.grid_n; b += 64) {
        int i = b + lane;
        bool ge = i < p.grid_n && p.grid[i] >= t;
        uint64_t bm = __ballot(ge);
        if (bm) { pick = (int)p.grid[b + __ffsll((long long)bm) - 1]; break; }
    }
    int lo = kq > 16 ? kq : 16;
    if (pick < lo) pick = lo;
    if (pick > p.L_cap) pick = p.L_cap;
    return pick;
}

// FULL = false compiles the plain search only (no early stop, feature capture,
// visited recording, pool output, counters or row prefetch): far less live
// uniform state in the loop, so the scalar registers do not spill.
template <int DT, int LPR, int CPL, bool FULL>
__global__ void __launch_bounds__(256) search_kernel(KParams p) {
    constexpr int EPC = Fmt<DT>::EPC;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    unsigned char *wbase = smem + (size_t)wave * p.lds_per_wave;
    uint64_t *pool = reinterpret_cast<uint64_t *>(wbase);
    uint32_t *hash = reinterpret_cast<uint32_t *>(pool + p.L_alloc);
    uint32_t *cid = hash + (1 << p.hash_bits);
    float *cdist = reinterpret_cast<float *>(cid + kMaxR);
    uint64_t *sbuf = reinterpret_cast<uint64_t *>(cdist + kMaxR);   // 16 staged keys (+16 spare)
    float *xbuf = reinterpret_cast<float *>(sbuf + 32);
    const int H = 1 << p.hash_bits;

    int64_t qi;
    if (p.counter) {
        unsigned int t = 0;
        if (lane == 0) t = atomicAdd(p.counter, 1u);
        qi = __shfl((int)t, 0);
    } else {
        qi = (int64_t)blockIdx.x * wpb + wave;
    }
    while (qi < p.nq) {
        const float *q = p.queries + qi * (int64_t)p.d;
        int kq = p.k_arr ? p.k_arr[qi] : p.k_scalar;
        kq = kq < 0 ? 0 : (kq > p.out_stride ? p.out_stride : kq);
        int Lq = p.L_arr ? p.L_arr[qi] : p.L_scalar;
        Lq = Lq < 1 ? 1 : (Lq > p.L_cap ? p.L_cap : Lq);
        const bool learned = FULL && p.learned && Lq >= 16;
        int Lcur = learned ? p.L_cap : Lq;

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
        int size = 0;
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
        if (lane == 0) pool[0] = mk_key(cdist[0], start);
        size = 1;
        wave_sync();
        int cursor = 0;
        bool stopped = !learned && !(FULL && p.features);   // true once the decision hop has passed
        // neighbour row of the predicted next expansion, loaded during the merge
        uint32_t pre_v = NSG_SENT, pre_u0 = NSG_SENT, pre_u1 = NSG_SENT;

        for (;;) {
            int i = find_unchecked(pool, cursor, size, lane);
            if (i < 0) break;
            uint64_t pe = pool[i];
            wave_sync();
            if (lane == 0) pool[i] = pe | CHECKED_BIT;
            uint32_t v = key_id(pe);
            v = v < p.n_rows ? v : 0u;
            ++hops;
            // neighbour ids (one coalesced row), visited filter, compaction
            const uint32_t *grow = p.graph + (int64_t)v * p.R_pad;
            uint32_t row0, row1;
            if (FULL && v == pre_v) {
                row0 = pre_u0;
                row1 = pre_u1;
            } else {
                row0 = lane < p.R ? grow[lane] : NSG_SENT;
                row1 = lane + 64 < p.R ? grow[lane + 64] : NSG_SENT;
            }
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
            if (cnt > 0) {
                gather_dist<DT, LPR, CPL>(p.rows, p.row_chunks, p.n_rows, qv, sc, cid, cdist, cnt, lane);
                wave_sync();
                nd += cnt;
                if (rec) {
                    for (int r = lane; r < cnt; r += 64)
                        if (vcount + r < p.vis_cap) {
                            p.vis_ids[qi * (int64_t)p.vis_cap + vcount + r] = cid[r];
                            p.vis_dist[qi * (int64_t)p.vis_cap + vcount + r] = cdist[r];
                        }
                }
                vcount += cnt;
                if (FULL && p.prefetch) {
                    // the next expansion is the better of the best new key that
                    // enters the pool and the first unchecked entry after i
                    const uint64_t worst0 = size >= Lcur ? (pool[Lcur - 1] & KEY_MASK) : KEY_NONE;
                    uint64_t kb = KEY_NONE;
                    for (int r = lane; r < cnt; r += 64) {
                        uint64_t kk = mk_key(cdist[r], cid[r]);
                        kb = kk < kb ? kk : kb;
                    }
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) {
                        uint64_t o = shfl_xor64(kb, off);
                        kb = o < kb ? o : kb;
                    }
                    int j = find_unchecked(pool, i + 1, size, lane);
                    uint64_t kj = j >= 0 ? (pool[j] & KEY_MASK) : KEY_NONE;
                    uint64_t kn = (kb < worst0 && kb < kj) ? kb : kj;
                    if (kn != KEY_NONE) {
                        pre_v = key_id(kn);
                        const uint32_t *nrow = p.graph + (int64_t)pre_v * p.R_pad;
                        pre_u0 = lane < p.R ? nrow[lane] : NSG_SENT;
                        pre_u1 = lane + 64 < p.R ? nrow[lane + 64] : NSG_SENT;
                    }
                }
                // keep candidates below the current L-th key, merge in rounds of 64
                int first = size;
                for (int b = 0; b < cnt; b += 64) {
                    const uint64_t worst = size >= Lcur ? (pool[Lcur - 1] & KEY_MASK) : KEY_NONE;
                    int r = b + lane;
                    uint64_t key = KEY_NONE;
                    if (r < cnt) {
                        uint64_t kk = mk_key(cdist[r], cid[r]);
                        if (kk < worst) key = kk;
                    }
                    int fi;
                    size = merge_pool(pool, size, Lcur, key, sbuf, lane, &fi);
                    first = fi < first ? fi : first;
                }
                cursor = (i + 1) < first ? (i + 1) : first;
            } else {
                cursor = i + 1;
            }
            if (FULL && !stopped && hops >= p.s_hop) {
                stopped = true;
                stop_features(p, q, pool, size, hops, xbuf, lane, qi);
                if (learned) {
                    Lcur = stop_predict(p, Lq, kq, xbuf, lane);
                    if (size > Lcur) size = Lcur;
                    if (cursor > size) cursor = size;
                }
            }
        }
        if (FULL && !stopped) {
            // ended before the decision point: the result equals the plain one
            if (p.features)
                for (int t = lane; t < p.d + 3; t += 64) p.features[qi * (int64_t)(p.d + 3) + t] = NAN;
            if (learned) {
                Lcur = Lq;
                if (size > Lcur) size = Lcur;
            }
        }
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
            if (p.L_used) p.L_used[qi] = Lcur;
            if (p.vis_cnt) p.vis_cnt[qi] = vcount;
        }
        wave_sync();
        if (!p.counter) break;
        unsigned int t = 0;
        if (lane == 0) t = atomicAdd(p.counter, 1u);
        qi = __shfl((int)t, 0);
    }
}


typedef void (*kfn_t)(KParams);

template <int DT>
static kfn_t pick_kernel_t(int lpr, int cpl, bool full) {
#define NSG_K(L_, C_)                                                              \
    if (lpr == L_ && cpl == C_) return full ? search_kernel<DT, L_, C_, true>      \
                                            : search_kernel<DT, L_, C_, false>;
    NSG_K(8, 1) NSG_K(8, 2) NSG_K(8, 4)
    NSG_K(16, 1) NSG_K(16, 2) NSG_K(16, 4)
    NSG_K(32, 1) NSG_K(32, 2) NSG_K(32, 4)
    NSG_K(64, 1) NSG_K(64, 2) NSG_K(64, 4)
#undef NSG_K
    return nullptr;
}

}  // namespace nsg
