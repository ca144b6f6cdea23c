// Exact kNN by brute force (serial scan) on gfx950 matrix cores.
//
// Stage 1 (matrix cores): a block owns a tile of queries and one contiguous
// split of the base.  For each tile of 64 base rows the inner products of
// centred vectors (q - mu).(x - mu) are accumulated with FP32
// v_mfma_f32_16x16x4f32, turned into rank values, and every value below the
// query's current threshold is appended to that query's candidate buffer
// (device memory: appends are rare once the threshold is tight).  A buffer
// that could overflow on the next tile is cut back to at most Kp + 32 keys
// that include its Kp best, by a radix select over the rank values (ballot
// counts, in registers) that stops as soon as a bound keeps that many; the
// bound becomes the threshold (the buffer holds Kp + 2 tiles at least, so
// cuts are rare once the threshold is tight).  Each block writes the ids of
// its Kp best per query for its split (an exact cut).
//  * d <= 128 (bf_wide_kernel): 4 waves x 32 queries per block; each wave
//    keeps its centred queries as matrix-core operands in registers for the
//    whole scan, owns all 64 rows of a tile and appends and compacts only its
//    own queries; the base tile is staged once per block, double buffered.
//  * d > 128 (bf_chunked_kernel): 4 waves x 32 queries per block and
//    128-row tiles; 32-dim chunks of the queries and of the tile are staged
//    once per block, double buffered.
// Stage 2: per query (one wave), exact FP32 squared distances sum (q_j-x_j)^2
// of all candidates of all splits, bitonic sort by (distance, id), first k.
// Centring keeps the cancellation error of the inner-product form small;
// the over-fetch margin (Kp >= k + 24) absorbs the rest before the exact pass.
#include "common.hpp"

#include <algorithm>

namespace nsg {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BX = 64;   // rows per base tile of the wide kernel
constexpr int kCutSlack = 32;   // an intermediate cut keeps at most Kp + 32 keys
// buffers hold at least Kp + 2 tiles and are cut once they could overflow on
// the next tile, so a cut must leave at most Kp + one tile (64 rows or more)
static_assert(kCutSlack <= BX, "a cut could leave too little room for the next tile");

struct BFParams {
    const float *base, *queries;
    const float *mu;       // [d] base mean
    const float *xnorm;    // [n] |x - mu|^2
    int64_t n, nq;
    int d, Kp, cap;
    int64_t split_len;
    int nsplit;
    int exclude_self;
    uint32_t *cand_ids;    // [nq][nsplit][Kp]
    uint64_t *cand_buf;    // [qtiles][nsplit][128 queries][cap] candidate buffers
};

__device__ inline void bsync() { __syncthreads(); }

// Column means in FP32 with compensated (Neumaier) sums: block b takes rows
// b, b + gridDim.x, ... and writes its partial sum and compensation per
// column; mean_finish_kernel adds the partials in block order, so the result
// is deterministic and close to the correctly rounded mean.
__global__ void colsum_part_kernel(const float *x, int64_t n, int d, float2 *part) {
    const int64_t G = gridDim.x;
    for (int j0 = 0; j0 < d; j0 += blockDim.x) {
        const int j = j0 + threadIdx.x;
        if (j >= d) continue;
        float s = 0.0f, c = 0.0f;
        int64_t i = blockIdx.x;
        for (; i + 3 * G < n; i += 4 * G) {   // four independent loads in flight, added in row order
            const float v0 = x[i * d + j], v1 = x[(i + G) * d + j];
            const float v2 = x[(i + 2 * G) * d + j], v3 = x[(i + 3 * G) * d + j];
            neumaier_add(s, c, v0);
            neumaier_add(s, c, v1);
            neumaier_add(s, c, v2);
            neumaier_add(s, c, v3);
        }
        for (; i < n; i += G) neumaier_add(s, c, x[i * d + j]);
        part[(size_t)blockIdx.x * d + j] = make_float2(s, c);
    }
}

__global__ void mean_finish_kernel(const float2 *part, int nblk, int64_t n, int d, float *mu) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= d) return;
    float s = 0.0f, c = 0.0f;
    constexpr int U = 16;   // partials loaded together, then added in block order
    int b = 0;
    for (; b + U <= nblk; b += U) {
        float2 p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) p[u] = part[(size_t)(b + u) * d + j];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            neumaier_add(s, c, p[u].x);
            c += p[u].y;
        }
    }
    for (; b < nblk; ++b) {
        const float2 p = part[(size_t)b * d + j];
        neumaier_add(s, c, p.x);
        c += p.y;
    }
    // (s + c) / n with the rounding error of s / n carried into the quotient
    const float fn = (float)n;
    const float q0 = s / fn;
    const float r = fmaf(-q0, fn, s);   // s - q0 * n (exact when n < 2^24)
    mu[j] = q0 + (r + c) / fn;
}

__global__ void cnorm_kernel(const float *x, int64_t n, int d, const float *mu, float *out) {
    // one wave per row
    const int lane = threadIdx.x & 63;
    const int64_t r = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    if (r >= n) return;
    float s = 0.0f;
    for (int j = lane; j < d; j += 64) {
        float t = x[r * d + j] - mu[j];
        s = fmaf(t, t, s);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) out[r] = s;
}

__device__ inline uint64_t bkey(float d, uint32_t id) {
    return ((uint64_t)__float_as_uint(d) << 32) | id;
}

// Sort buf[0..cnt) ascending in place (bitonic, padded with ~0 up to the next
// power of two, at most cap).  Executed by one wave.
__device__ inline void wave_sort_buf(uint64_t *buf, int cnt, int cap, int lane) {
    int np = 1;
    while (np < cnt) np <<= 1;
    if (np > cap) np = cap;
    for (int i = cnt + lane; i < np; i += 64) buf[i] = ~0ull;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int k = 2; k <= np; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < np; i += 64) {
                int ixj = i ^ j;
                if (ixj > i) {
                    uint64_t a = buf[i], b = buf[ixj];
                    bool up = (i & k) == 0;
                    if ((a > b) == up) { buf[i] = b; buf[ixj] = a; }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
}

// Order-preserving map of a float to 32 bits (ascending keys = ascending
// values, negative values included).
__device__ inline uint32_t ord_bits(float v) {
    const uint32_t u = __float_as_uint(v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float ord_float(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

__device__ inline void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Cut buf[0..c) (c in [Kp, 512]) to at least its Kp entries with the
// smallest rank values (the high words of the keys), moved to the front in no
// particular order, and return the bound B such that every kept entry and no
// dropped one has a high word below B (2^32: no bound); *kept receives their
// number.  slack = 0: exactly Kp are kept (ties at the cut taken in buffer
// order: then B is the Kp-th smallest high word and the tied ones beyond Kp
// are dropped, none of them below B).  slack > 0: at most Kp + slack (an
// intermediate cut needs no exact count: rejecting later values at or above
// B keeps every entry that can still be among the Kp best).  One wave: the
// bucket of high words holding the Kp-th smallest is narrowed bit by bit from
// the highest bit on which the keys differ (a radix select counting with
// ballots); it stops once the bucket and everything below it hold at most
// Kp + slack entries (for slack = 0: once the bucket holds exactly the
// entries still needed).  Every load precedes every store (the stores depend
// on ballots over all loaded keys).
__device__ __attribute__((noinline)) uint64_t wave_keep_smallest(uint64_t *buf, int c, int Kp, int slack, int lane,
                                                                 int *kept) {
    constexpr int M = 8;
    uint64_t key[M];
    bool ok[M];
#pragma unroll
    for (int e = 0; e < M; ++e) {
        const int j = e * 64 + lane;
        ok[e] = j < c;
        key[e] = ok[e] ? buf[j] : 0ull;
    }
    // bits on which every key agrees are the target's too: start below them
    uint32_t all_or = 0u, all_and = 0xFFFFFFFFu;
#pragma unroll
    for (int e = 0; e < M; ++e) {
        const uint32_t h = (uint32_t)(key[e] >> 32);
        all_or |= ok[e] ? h : 0u;
        all_and &= ok[e] ? h : 0xFFFFFFFFu;
    }
    for (int o = 32; o > 0; o >>= 1) {
        all_or |= (uint32_t)__shfl_xor((int)all_or, o);
        all_and &= (uint32_t)__shfl_xor((int)all_and, o);
    }
    const uint32_t diff = all_or ^ all_and;
    const int top = diff ? 31 - __builtin_clz(diff) : -1;   // highest bit on which keys differ
    uint32_t prefix = top >= 31 ? 0u : (all_and & (0xFFFFFFFFu << (top + 1)));
    int need = Kp;      // rank of the target among the entries in the bucket
    int in_bucket = c;  // entries whose high word matches the prefix on the bits examined
    uint64_t bound = 0; // > 0: early stop, keep every entry below it
    for (int b = top; b >= 0; --b) {
        const uint32_t above = b == 31 ? 0u : (0xFFFFFFFFu << (b + 1));
        int cnt = 0;
#pragma unroll
        for (int e = 0; e < M; ++e) {
            const uint32_t h = (uint32_t)(key[e] >> 32);
            if (e * 64 < c) cnt += __popcll(__ballot(ok[e] && (h & above) == prefix && ((h >> b) & 1u) == 0u));
        }
        if (cnt < need) {
            need -= cnt;
            in_bucket -= cnt;
            prefix |= 1u << b;
        } else {
            in_bucket = cnt;
        }
        if (in_bucket - need <= slack) {   // bucket [prefix, prefix + 2^b) and all below it
            bound = (uint64_t)prefix + (1ull << b);
            break;
        }
    }
    // bound: entries below it to the front; else entries below the prefix
    // value to [0, Kp - need), the first `need` equal to it to [Kp - need, Kp)
    const uint64_t below = (1ull << lane) - 1ull;
    int at_lt = 0, at_eq = Kp - need, eq_seen = 0;
#pragma unroll
    for (int e = 0; e < M; ++e) {
        if (e * 64 >= c) continue;
        const uint32_t h = (uint32_t)(key[e] >> 32);
        const bool lt = ok[e] && (bound ? (uint64_t)h < bound : h < prefix);
        const bool eq = !bound && ok[e] && h == prefix;
        const uint64_t blt = __ballot(lt), beq = __ballot(eq);
        const int rl = __popcll(blt & below), re = __popcll(beq & below);
        if (lt) buf[at_lt + rl] = key[e];
        if (eq && eq_seen + re < need) buf[at_eq + eq_seen + re] = key[e];
        at_lt += __popcll(blt);
        eq_seen += __popcll(beq);
    }
    *kept = bound ? at_lt : Kp;
    return bound ? bound : (uint64_t)prefix;
}

// the rank-value threshold for a cut's bound B: later values v are appended
// only while ord_bits(v) < B
__device__ inline float cut_threshold(uint64_t B) {
    return B > 0xFF800000ull ? INFINITY : ord_float((uint32_t)B);
}

// Stage 1 for d <= 128 with wide query tiles.  Every wave owns QW queries
// (QW / 16 matrix-core row groups whose centred operands stay in registers
// for the whole scan) and all 64 rows of each base tile.  The block stages a
// tile once in LDS for its 4 waves (double buffered, one barrier per tile;
// the next tile is loaded into registers while the current one is
// multiplied), so the base is streamed once per 4 * QW queries.  Inside the
// inner product the dimensions are permuted (any permutation applied to
// both operands gives the same sum): lane group kq takes dims [kq*S, kq*S+S)
// over the S k-steps, so one 16-byte LDS read supplies four k-steps.
// Rank value a = |x - mu|^2 - 2 (q - mu).(x - mu), which is the squared
// distance minus |q - mu|^2 and so orders a query's rows as the distance
// does.  Each wave appends its own queries' values below their thresholds
// and compacts its own buffers: appends and compaction need no block-wide
// synchronisation.  Values of rows past the split carry |x - mu|^2 = +inf
// and never pass; queries past nq get threshold -inf.
template <int DP, int QW, bool VEC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) bf_wide_kernel(BFParams p) {
    constexpr int S = DP / 4;            // k-steps of 4 dims
    constexpr int G = QW / 16;           // row groups per wave
    constexpr int LD = DP + 4;           // staged row stride (floats)
    constexpr int F4 = DP / 4;           // 16-byte pieces per staged row
    constexpr int NIT = BX * F4 / 256;   // pieces per thread per tile
    static_assert(DP % 16 == 0 && DP <= 128 && (BX * F4) % 256 == 0, "tile shape");
    extern __shared__ __align__(16) unsigned char smem[];
    float *Xs = reinterpret_cast<float *>(smem);                          // [2][BX][LD]
    float *mus = Xs + 2 * BX * LD;                                        // [DP] centre, 0 past d
    float *thr_s = mus + DP;                                              // [4][QW]
    int *cnt_s = reinterpret_cast<int *>(thr_s + 4 * QW);                 // [4][QW]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int rq = lane & 15, kq = lane >> 4;
    const int64_t qb = (int64_t)blockIdx.x * 4 * QW;   // first query of the block
    const int64_t qw0 = qb + (int64_t)w * QW;           // first query of the wave
    const int split = blockIdx.y;
    const int64_t xb = (int64_t)split * p.split_len;
    const int64_t xe = std::min<int64_t>(p.n, xb + p.split_len);
    uint64_t *buf = p.cand_buf + ((int64_t)blockIdx.x * p.nsplit + split) * (int64_t)(4 * QW) * p.cap +
                    (int64_t)w * QW * p.cap;
    float *thr_w = thr_s + w * QW;
    int *cnt_w = cnt_s + w * QW;
    for (int j = tid; j < DP; j += 256) mus[j] = j < p.d ? p.mu[j] : 0.0f;
    if (lane < QW) {
        thr_w[lane] = qw0 + lane < p.nq ? INFINITY : -INFINITY;
        cnt_w[lane] = 0;
    }
    // centred query operands: a[g][s] = q[qw0 + 16 g + rq][kq * S + s] - mu
    float a[G][S];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t qi = qw0 + 16 * g + rq;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int j = kq * S + s;
            a[g][s] = (qi < p.nq && j < p.d) ? p.queries[qi * p.d + j] - p.mu[j] : 0.0f;
        }
    }
    // base tile pieces of this thread: piece f = tid + 256 it is row f / F4,
    // dims 4 (f % F4) .. + 3; the next tile is loaded in two halves (the
    // first while the first half of the k-steps runs, the second while the
    // rest runs).  Loads use clamped in-range addresses and a select (no
    // branches); rows past the split and dims past d give 0.
    constexpr int H = NIT / 2;
    float4 xr[H];
    auto load_half = [&](int64_t x0, int h) {
        const float *tb = p.base + x0 * p.d;
        const int rows = (int)std::min<int64_t>(BX, xe - x0);
#pragma unroll
        for (int u = 0; u < H; ++u) {
            const int f = tid + 256 * (h * H + u);
            const int r = f / F4, j = 4 * (f % F4);
            const int rr = std::min(r, rows - 1);
            if (VEC) {
                const float4 v = *reinterpret_cast<const float4 *>(tb + (uint32_t)(rr * p.d + std::min(j, p.d - 4)));
                const bool ok = r < rows && j < p.d;
                xr[u] = ok ? v : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            } else {
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float w4 = tb[(uint32_t)(rr * p.d + std::min(j + e, p.d - 1))];
                    v[e] = r < rows && j + e < p.d ? w4 : 0.0f;
                }
                xr[u] = make_float4(v[0], v[1], v[2], v[3]);
            }
        }
    };
    auto store_half = [&](float *dst, int h) {
#pragma unroll
        for (int u = 0; u < H; ++u) {
            const int f = tid + 256 * (h * H + u);
            const int r = f / F4, j = 4 * (f % F4);
            const float4 m = *reinterpret_cast<const float4 *>(mus + j);
            float4 v = xr[u];
            v.x -= m.x; v.y -= m.y; v.z -= m.z; v.w -= m.w;
            *reinterpret_cast<float4 *>(dst + r * LD + j) = v;
        }
    };
    auto load_xn = [&](int64_t x0, float *xn) {
        const int rows = (int)std::min<int64_t>(BX, xe - x0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int r = 16 * t + rq;
            const float u = p.xnorm[x0 + std::min(r, rows - 1)];
            xn[t] = r < rows ? u : INFINITY;
        }
    };
    bsync();   // centre and counters visible
    float thr[G][4];
    auto load_thr = [&]() {
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int i = 0; i < 4; ++i) thr[g][i] = thr_w[16 * g + 4 * kq + i];
    };
    load_thr();
    if (xb < xe) {
        load_half(xb, 0);
        store_half(Xs, 0);
        load_half(xb, 1);
        store_half(Xs, 1);
    }
    bsync();
    int cur = 0;
    for (int64_t x0 = xb; x0 < xe; x0 += BX) {
        const bool more = x0 + BX < xe;
        float xn[4];
        load_xn(x0, xn);
        if (more) load_half(x0 + BX, 0);
        const float *Xc = Xs + cur * BX * LD;
        float *Xn = Xs + (cur ^ 1) * BX * LD;
        f32x4 acc[G][4];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[g][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s4 = 0; s4 < S; s4 += 4) {
            if (s4 == S / 2 && more) {
                store_half(Xn, 0);
                load_half(x0 + BX, 1);
            }
            float4 b[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) b[t] = *reinterpret_cast<const float4 *>(Xc + (16 * t + rq) * LD + kq * S + s4);
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float bv = e == 0 ? b[t].x : e == 1 ? b[t].y : e == 2 ? b[t].z : b[t].w;
#pragma unroll
                    for (int g = 0; g < G; ++g)
                        acc[g][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[g][s4 + e], bv, acc[g][t], 0, 0, 0);
                }
        }
        // epilogue: lane holds queries 16 g + 4 kq + i of the wave, row 16 t + rq
        // of the tile; rank values in place, a query's own row made +inf in
        // the one tile that can hold it (exclude_self)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[g][t][i] = fmaf(-2.0f, acc[g][t][i], xn[t]);
        if (p.exclude_self && x0 < qw0 + QW && qw0 < x0 + BX) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (x0 + 16 * t + rq == qw0 + 16 * g + 4 * kq + i) acc[g][t][i] = INFINITY;
        }
        // per query row: the lane's 4 values are tested one by one only when
        // their minimum passes (rare once the threshold is tight)
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float m = fminf(fminf(acc[g][0][i], acc[g][1][i]), fminf(acc[g][2][i], acc[g][3][i]));
                if (m < thr[g][i]) {
                    const int r = 16 * g + 4 * kq + i;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const float v = acc[g][t][i];
                        if (v < thr[g][i]) {
                            const int slot = atomicAdd(&cnt_w[r], 1);
                            buf[(size_t)r * p.cap + slot] =
                                ((uint64_t)ord_bits(v) << 32) | (uint32_t)(x0 + 16 * t + rq);
                        }
                    }
                }
            }
        wave_fence();
        // compaction of this wave's buffers that could overflow on the next tile
        uint64_t full = __builtin_amdgcn_ballot_w64(lane < QW && cnt_w[lane < QW ? lane : 0] > p.cap - BX);
        if (full) {
            while (full) {
                const int r = __builtin_ctzll(full);
                full &= full - 1;
                const int c = cnt_w[r];
                int kept = 0;
                const float tnew = cut_threshold(wave_keep_smallest(buf + (size_t)r * p.cap, c, p.Kp, kCutSlack,
                                                                    lane, &kept));
                wave_fence();
                if (lane == 0) {
                    cnt_w[r] = kept;
                    thr_w[r] = tnew;
                }
                wave_fence();
            }
            load_thr();
        }
        if (more) store_half(Xn, 1);
        cur ^= 1;
        bsync();
    }
    // final: cut each buffer of the wave to its Kp smallest, write their ids
    // (order free: stage 2 sorts; sentinel padded)
    for (int r = 0; r < QW; ++r) {
        const int64_t qi = qw0 + r;
        if (qi >= p.nq) break;
        const int c = cnt_w[r];
        uint64_t *br = buf + (size_t)r * p.cap;
        if (c > p.Kp) {
            int kept = 0;
            wave_keep_smallest(br, c, p.Kp, 0, lane, &kept);
            wave_fence();
        }
        uint32_t *dst = p.cand_ids + (qi * p.nsplit + split) * (int64_t)p.Kp;
        for (int j = lane; j < p.Kp; j += 64) dst[j] = j < c ? (uint32_t)(br[j] & 0xFFFFFFFFu) : NSG_SENT;
        wave_fence();
    }
}

// Stage 1 for d > 128 (bf_chunked_kernel): 4 waves x 32 queries per block and
// 128-row base tiles; each wave owns all 128 rows of a tile for its queries
// (2 row groups x 8 column groups of accumulators).  The dimensions stream
// in chunks of 32: the block stages each chunk of its 128 centred queries
// and of the tile's 128 centred rows in LDS (double buffered, one barrier per
// chunk; the next chunk is loaded into registers in two halves while the
// current one is multiplied).  The query chunks are read again for every
// tile (from L2 or the last-level cache); a 128 x 128 output tile keeps that
// traffic at 64 flops per byte.  Operand reads are 16 bytes wide through the
// same permutation of the dimensions as the wide kernel (lane group kq takes
// dims [8 kq, 8 kq + 8) of each chunk).  Rank values, appends, cuts and the
// final write are those of the wide kernel.
constexpr int CQ = 128, CX = 128, KC = 32, CLD = KC + 4;

template <bool VEC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) bf_chunked_kernel(BFParams p) {
    constexpr int QW = 32, G = 2, T = 8, F4 = KC / 4;   // queries per wave, row / column groups, pieces per row
    static_assert(256 % F4 == 0 && (CQ * F4) % 256 == 0 && CQ == CX, "staging shape");
    extern __shared__ __align__(16) unsigned char smem[];
    float *As = reinterpret_cast<float *>(smem);                       // [2][CQ][CLD]
    float *Bs = As + 2 * CQ * CLD;                                     // [2][CX][CLD]
    float *thr_s = Bs + 2 * CX * CLD;                                  // [4][QW]
    int *cnt_s = reinterpret_cast<int *>(thr_s + 4 * QW);              // [4][QW]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int rq = lane & 15, kq = lane >> 4;
    const int64_t qb = (int64_t)blockIdx.x * CQ;
    const int64_t qw0 = qb + (int64_t)w * QW;
    const int split = blockIdx.y;
    const int64_t xb = (int64_t)split * p.split_len;
    const int64_t xe = std::min<int64_t>(p.n, xb + p.split_len);
    uint64_t *buf = p.cand_buf + ((int64_t)blockIdx.x * p.nsplit + split) * (int64_t)CQ * p.cap +
                    (int64_t)w * QW * p.cap;
    float *thr_w = thr_s + w * QW;
    int *cnt_w = cnt_s + w * QW;
    const int nchunk = (p.d + KC - 1) / KC;
    if (lane < QW) {
        thr_w[lane] = qw0 + lane < p.nq ? INFINITY : -INFINITY;
        cnt_w[lane] = 0;
    }
    const int qrows = (int)std::min<int64_t>(CQ, p.nq - qb);   // >= 1
    // one operand's chunk: 128 rows x 32 dims = 1024 pieces of 16 bytes, 4 per
    // thread; piece f = tid + 256 u is row f / 8, dims k0 + 4 (f % 8) .. + 3.
    // Clamped in-range addresses and a select: rows past the end and dims past
    // d give 0.
    float4 xr[4];
    float mv[4];   // the centre at this thread's 4 dims of the chunk (see store_op)
    auto load_op = [&](const float *rows, int nrows, int k0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = k0 + 4 * (tid % F4) + e;
            const float m = p.mu[std::min(j, p.d - 1)];
            mv[e] = j < p.d ? m : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int f = tid + 256 * u;
            const int r = f / F4, j = k0 + 4 * (f % F4);
            const int rr = std::min(r, nrows - 1);
            if (VEC) {
                const float4 v = *reinterpret_cast<const float4 *>(rows + (int64_t)rr * p.d + std::min(j, p.d - 4));
                xr[u] = r < nrows && j < p.d ? v : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            } else {
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float x = rows[(int64_t)rr * p.d + std::min(j + e, p.d - 1)];
                    v[e] = r < nrows && j + e < p.d ? x : 0.0f;
                }
                xr[u] = make_float4(v[0], v[1], v[2], v[3]);
            }
        }
    };
    // centred into LDS; a thread's pieces all sit at dims k0 + c .. + 3 with
    // c = 4 (tid % 8), so load_op reads those 4 values of the centre once,
    // with the operand (0 past d)
    auto store_op = [&](float *dst) {
        const int c = 4 * (tid % F4);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = (tid + 256 * u) / F4;
            float4 v = xr[u];
            v.x -= mv[0]; v.y -= mv[1]; v.z -= mv[2]; v.w -= mv[3];
            *reinterpret_cast<float4 *>(dst + r * CLD + c) = v;
        }
    };
    const float *qrow0 = p.queries + qb * p.d;
    auto tile_rows = [&](int64_t x0) { return (int)std::min<int64_t>(CX, xe - x0); };
    bsync();   // counters visible
    float thr[G][4];
    auto load_thr = [&]() {
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int i = 0; i < 4; ++i) thr[g][i] = thr_w[16 * g + 4 * kq + i];
    };
    load_thr();
    if (xb < xe) {
        load_op(qrow0, qrows, 0);
        store_op(As);
        load_op(p.base + xb * p.d, tile_rows(xb), 0);
        store_op(Bs);
    }
    bsync();
    int cur = 0;
    for (int64_t x0 = xb; x0 < xe; x0 += CX) {
        float xn[T];
        {
            const int rows = tile_rows(x0);
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const int r = 16 * t + rq;
                const float u = p.xnorm[x0 + std::min(r, rows - 1)];
                xn[t] = r < rows ? u : INFINITY;
            }
        }
        f32x4 acc[G][T];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int t = 0; t < T; ++t) acc[g][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int ch = 0; ch < nchunk; ++ch) {
            // the chunk staged next: the following chunk of this tile, else
            // the first chunk of the next tile
            const bool more = ch + 1 < nchunk || x0 + CX < xe;
            const int64_t nx0 = ch + 1 < nchunk ? x0 : x0 + CX;
            const int nk0 = ch + 1 < nchunk ? (ch + 1) * KC : 0;
            const float *Ac = As + cur * CQ * CLD, *Bc = Bs + cur * CX * CLD;
            float *An = As + (cur ^ 1) * CQ * CLD, *Bn = Bs + (cur ^ 1) * CX * CLD;
            if (more) load_op(qrow0, qrows, nk0);
#pragma unroll
            for (int s4 = 0; s4 < KC / 4; s4 += 4) {
                if (s4 == 4 && more) {
                    store_op(An);
                    load_op(p.base + nx0 * p.d, tile_rows(nx0), nk0);
                }
                float4 a4[G];
#pragma unroll
                for (int g = 0; g < G; ++g)
                    a4[g] = *reinterpret_cast<const float4 *>(Ac + (QW * w + 16 * g + rq) * CLD + 8 * kq + s4);
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    const float4 b4 = *reinterpret_cast<const float4 *>(Bc + (16 * t + rq) * CLD + 8 * kq + s4);
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        acc[g][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[g].x, b4.x, acc[g][t], 0, 0, 0);
                        acc[g][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[g].y, b4.y, acc[g][t], 0, 0, 0);
                        acc[g][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[g].z, b4.z, acc[g][t], 0, 0, 0);
                        acc[g][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[g].w, b4.w, acc[g][t], 0, 0, 0);
                    }
                }
            }
            if (more) store_op(Bn);
            cur ^= 1;
            bsync();
        }
        // epilogue: lane holds queries 16 g + 4 kq + i of the wave, row 16 t + rq
        // of the tile; rank values in place, a query's own row made +inf
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[g][t][i] = fmaf(-2.0f, acc[g][t][i], xn[t]);
        if (p.exclude_self && x0 < qw0 + QW && qw0 < x0 + CX) {
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (x0 + 16 * t + rq == qw0 + 16 * g + 4 * kq + i) acc[g][t][i] = INFINITY;
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float m = acc[g][0][i];
#pragma unroll
                for (int t = 1; t < T; ++t) m = fminf(m, acc[g][t][i]);
                if (m < thr[g][i]) {
                    const int r = 16 * g + 4 * kq + i;
#pragma unroll
                    for (int t = 0; t < T; ++t) {
                        const float v = acc[g][t][i];
                        if (v < thr[g][i]) {
                            const int slot = atomicAdd(&cnt_w[r], 1);
                            buf[(size_t)r * p.cap + slot] =
                                ((uint64_t)ord_bits(v) << 32) | (uint32_t)(x0 + 16 * t + rq);
                        }
                    }
                }
            }
        wave_fence();
        // cut this wave's buffers that could overflow on the next tile
        uint64_t full = __builtin_amdgcn_ballot_w64(lane < QW && cnt_w[lane < QW ? lane : 0] > p.cap - CX);
        if (full) {
            while (full) {
                const int r = __builtin_ctzll(full);
                full &= full - 1;
                const int c = cnt_w[r];
                int kept = 0;
                const float tnew = cut_threshold(wave_keep_smallest(buf + (size_t)r * p.cap, c, p.Kp, kCutSlack,
                                                                    lane, &kept));
                wave_fence();
                if (lane == 0) {
                    cnt_w[r] = kept;
                    thr_w[r] = tnew;
                }
                wave_fence();
            }
            load_thr();
        }
    }
    // final: cut each buffer of the wave to its Kp smallest, write their ids
    for (int r = 0; r < QW; ++r) {
        const int64_t qi = qw0 + r;
        if (qi >= p.nq) break;
        const int c = cnt_w[r];
        uint64_t *br = buf + (size_t)r * p.cap;
        if (c > p.Kp) {
            int kept = 0;
            wave_keep_smallest(br, c, p.Kp, 0, lane, &kept);
            wave_fence();
        }
        uint32_t *dst = p.cand_ids + (qi * p.nsplit + split) * (int64_t)p.Kp;
        for (int j = lane; j < p.Kp; j += 64) dst[j] = j < c ? (uint32_t)(br[j] & 0xFFFFFFFFu) : NSG_SENT;
        wave_fence();
    }
}

// one wave per query: exact distances of all candidates, sort, first k.
// vec4 (d % 4 == 0, 16-byte aligned rows): 8 candidates per round, 8 lanes
// each reading 16 bytes at a time; else 4 candidates of 16 lanes, 4 bytes.
// sort_n is a power of two of at least 32 (ncand >= Kp >= 32).
__global__ void __launch_bounds__(256) bf_rerank_kernel(const float *base, const float *queries, int64_t nq,
                                                        int d, const uint32_t *cand, int ncand, int k,
                                                        int sort_n, int vec4, uint32_t *out_ids,
                                                        float *out_dist) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t qi = (int64_t)blockIdx.x * (blockDim.x >> 6) + w;
    uint64_t *a = reinterpret_cast<uint64_t *>(smem) + (size_t)w * sort_n;
    if (qi >= nq) return;
    const float *q = queries + qi * d;
    const uint32_t *c = cand + qi * (int64_t)ncand;
    if (vec4) {
        const int g = lane >> 3, li = lane & 7, d4 = d >> 2;
        const float4 *q4 = reinterpret_cast<const float4 *>(q);
        for (int r0 = 0; r0 < sort_n; r0 += 8) {
            const int r = r0 + g;
            const uint32_t id = r < ncand ? c[r] : NSG_SENT;
            float acc = 0.0f;
            if (id != NSG_SENT) {
                const float4 *x4 = reinterpret_cast<const float4 *>(base + (int64_t)id * d);
                for (int j = li; j < d4; j += 8) {
                    const float4 u = q4[j], v = x4[j];
                    const float t0 = u.x - v.x, t1 = u.y - v.y, t2 = u.z - v.z, t3 = u.w - v.w;
                    acc = fmaf(t0, t0, acc);
                    acc = fmaf(t1, t1, acc);
                    acc = fmaf(t2, t2, acc);
                    acc = fmaf(t3, t3, acc);
                }
            }
            for (int o = 4; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
            if (li == 0) a[r] = id == NSG_SENT ? ~0ull : bkey(acc, id);
        }
    } else {
        const int g = lane >> 4, li = lane & 15;
        for (int r0 = 0; r0 < sort_n; r0 += 4) {
            const int r = r0 + g;
            const uint32_t id = r < ncand ? c[r] : NSG_SENT;
            float acc = 0.0f;
            if (id != NSG_SENT) {
                const float *x = base + (int64_t)id * d;
                for (int j = li; j < d; j += 16) {
                    const float t = q[j] - x[j];
                    acc = fmaf(t, t, acc);
                }
            }
            for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
            if (li == 0) a[r] = id == NSG_SENT ? ~0ull : bkey(acc, id);
        }
    }
    wave_sort_buf(a, sort_n, sort_n, lane);
    for (int j = lane; j < k; j += 64) {
        uint64_t v = a[j];
        bool ok = v != ~0ull;
        out_ids[qi * k + j] = ok ? (uint32_t)(v & 0xFFFFFFFFu) : NSG_SENT;
        out_dist[qi * k + j] = ok ? __uint_as_float((uint32_t)(v >> 32)) : INFINITY;
    }
}

int mean_blocks(int64_t n) { return (int)std::min<int64_t>(n, 1024); }

constexpr int kWideQW = 32;   // queries per wave of the wide stage 1

int launch_mean(const float *x, int64_t n, int d, float *mu, float2 *part, hipStream_t st) {
    const int nblk = mean_blocks(n);
    hipLaunchKernelGGL(colsum_part_kernel, dim3((unsigned)nblk), dim3(d < 256 ? (d + 63) / 64 * 64 : 256), 0, st,
                       x, n, d, part);
    hipLaunchKernelGGL(mean_finish_kernel, dim3((d + 255) / 256), dim3(256), 0, st, part, nblk, n, d, mu);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(NSG_EDEVICE, "mean kernels failed: %s", hipGetErrorString(e));
    return NSG_OK;
}

// the wide stage-1 kernel for rows padded to DP dims, and its LDS bytes
struct WideKernel {
    const void *fn;
    size_t lds;
};

template <int DP, bool VEC>
WideKernel wide_kernel_t() {
    return {(const void *)bf_wide_kernel<DP, kWideQW, VEC>,
            (size_t)2 * BX * (DP + 4) * 4 + (size_t)DP * 4 + (size_t)4 * kWideQW * 8};
}

template <bool VEC>
WideKernel wide_kernel_v(int d) {
    const int DP = (d + 31) / 32 * 32;
    return DP == 32 ? wide_kernel_t<32, VEC>()
           : DP == 64 ? wide_kernel_t<64, VEC>()
           : DP == 96 ? wide_kernel_t<96, VEC>()
                      : wide_kernel_t<128, VEC>();
}

// Launch plan of one brute force: stage-1 kernel, splits of the base,
// candidate counts, and the offsets of its scratch in one block of memory.
struct BFPlan {
    WideKernel wk;
    int Kp, cap, nsplit, ncand, sort_n, vec4;
    int64_t qtiles, split_len;
    size_t off_mu, off_xnorm, off_cand, off_cbuf, bytes;
};

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// arguments are validated by the caller
static int bf_plan(const float *base, int64_t n, const float *queries, int64_t nq, int d, int k, BFPlan *pl) {
    BFPlan &P = *pl;
    // over-fetch margin 24 for the inner-product form's rounding
    P.Kp = (k + 24 + 31) / 32 * 32;
    // d <= 128: wide query tiles (4 waves x kWideQW queries, 64-row tiles);
    // d > 128: chunked dimensions (4 waves x 32 queries, 128-row tiles)
    const bool wide = d <= 128;
    const int tile = wide ? BX : CX;
    const bool vec4 = d % 4 == 0 && (reinterpret_cast<uintptr_t>(base) & 15) == 0 &&
                      (reinterpret_cast<uintptr_t>(queries) & 15) == 0;
    const int bq = wide ? 4 * kWideQW : CQ;
    P.qtiles = (nq + bq - 1) / bq;
    P.vec4 = vec4 ? 1 : 0;
    if (wide) {
        P.wk = vec4 ? wide_kernel_v<true>(d) : wide_kernel_v<false>(d);
    } else {
        const size_t lds = (size_t)4 * CQ * CLD * 4 + (size_t)8 * 32 * 4;
        P.wk = {vec4 ? (const void *)bf_chunked_kernel<true> : (const void *)bf_chunked_kernel<false>, lds};
    }
    // splits of the base: with fewer query tiles than resident blocks, enough
    // splits for one full round of blocks (fewer splits keep the exact pass
    // short); at least a few tiles per split
    NSG_HIP(hipFuncSetAttribute(P.wk.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.wk.lds));
    int dev = 0, cus = 0, per_cu = 0;
    NSG_HIP(hipGetDevice(&dev));
    NSG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    NSG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, P.wk.fn, 256, P.wk.lds));
    const int64_t slots = std::max<int64_t>(1, (int64_t)cus * per_cu);
    const int64_t want = std::max<int64_t>(1, slots / P.qtiles);
    const int64_t max_split = std::max<int64_t>(1, n / (BX * 8));
    P.nsplit = (int)std::min<int64_t>(std::min<int64_t>(want, max_split), std::max(1, 4096 / P.Kp));
    P.split_len = (n + P.nsplit - 1) / P.nsplit;
    P.split_len = (P.split_len + BX - 1) / BX * BX;
    P.nsplit = (int)((n + P.split_len - 1) / P.split_len);
    // candidate buffers: Kp + two tiles at least; 512 (what a cut handles)
    // while all of them stay within 8 GiB, so that a cut absorbs more appends
    P.cap = 1;
    while (P.cap < P.Kp + 2 * tile) P.cap <<= 1;
    if ((double)P.qtiles * P.nsplit * bq * 512 * sizeof(uint64_t) <= 8.0 * (1 << 30)) P.cap = 512;
    P.ncand = P.nsplit * P.Kp;
    P.sort_n = 1;
    while (P.sort_n < P.ncand) P.sort_n <<= 1;
    if (P.sort_n * 8 > 64 * 1024) return fail(NSG_EUNSUPPORTED, "too many candidates per query (%d)", P.ncand);
    // scratch: column partial sums, mean, centred row norms, candidate ids,
    // candidate buffers; each 256-byte aligned
    P.off_mu = align256(sizeof(float2) * d * mean_blocks(n));
    P.off_xnorm = P.off_mu + align256(sizeof(float) * d);
    P.off_cand = P.off_xnorm + align256(sizeof(float) * n);
    P.off_cbuf = P.off_cand + align256(sizeof(uint32_t) * nq * P.ncand);
    P.bytes = P.off_cbuf + align256(sizeof(uint64_t) * P.qtiles * P.nsplit * bq * P.cap);
    return NSG_OK;
}

static int bf_launch(const BFPlan &P, const float *base, int64_t n, const float *queries, int64_t nq, int d, int k,
                     int exclude_self, uint32_t *out_ids, float *out_dist, unsigned char *ws, hipStream_t st) {
    float2 *acc = reinterpret_cast<float2 *>(ws);
    float *mu = reinterpret_cast<float *>(ws + P.off_mu);
    float *xnorm = reinterpret_cast<float *>(ws + P.off_xnorm);
    uint32_t *cand = reinterpret_cast<uint32_t *>(ws + P.off_cand);
    uint64_t *cbuf = reinterpret_cast<uint64_t *>(ws + P.off_cbuf);
    if (int rc = launch_mean(base, n, d, mu, acc, st)) return rc;
    hipLaunchKernelGGL(cnorm_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, base, n, d, mu, xnorm);
    BFParams p{};
    p.base = base;
    p.queries = queries;
    p.mu = mu;
    p.xnorm = xnorm;
    p.n = n;
    p.nq = nq;
    p.d = d;
    p.Kp = P.Kp;
    p.cap = P.cap;
    p.split_len = P.split_len;
    p.nsplit = P.nsplit;
    p.exclude_self = exclude_self ? 1 : 0;
    p.cand_ids = cand;
    p.cand_buf = cbuf;
    void *args[] = {&p};
    const hipError_t le =
        hipLaunchKernel(P.wk.fn, dim3((unsigned)P.qtiles, (unsigned)P.nsplit), dim3(256), args, P.wk.lds, st);
    // stage 2 reads the candidates stage 1 wrote: launched only after it
    if (le == hipSuccess) {
        const int wpb = std::max(1, std::min(4, (int)(64 * 1024 / ((size_t)P.sort_n * 8))));
        hipLaunchKernelGGL(bf_rerank_kernel, dim3((unsigned)((nq + wpb - 1) / wpb)), dim3(64 * wpb),
                           (size_t)P.sort_n * 8 * wpb, st, base, queries, nq, d, cand, P.ncand, k, P.sort_n, P.vec4,
                           out_ids, out_dist);
    }
    const hipError_t e = le != hipSuccess ? le : hipGetLastError();
    if (e != hipSuccess) return fail(NSG_EDEVICE, "brute-force launch failed: %s", hipGetErrorString(e));
    return NSG_OK;
}

// For callers that run many brute forces back to back (the inverted-file
// graph): the scratch one call takes, and the call on scratch the caller
// owns (256-byte aligned, at least that many bytes, not used by another
// call in flight).  Arguments as nsg_knn_bruteforce's, validated by the
// caller.
int bf_scratch_bytes(const float *base, int64_t n, const float *queries, int64_t nq, int d, int k, size_t *bytes) {
    BFPlan P{};
    if (int rc = bf_plan(base, n, queries, nq, d, k, &P)) return rc;
    *bytes = P.bytes;
    return NSG_OK;
}

int bf_with_scratch(const float *base, int64_t n, const float *queries, int64_t nq, int d, int k, int exclude_self,
                    uint32_t *out_ids, float *out_dist, void *scratch, size_t scratch_bytes, hipStream_t st) {
    BFPlan P{};
    if (int rc = bf_plan(base, n, queries, nq, d, k, &P)) return rc;
    if (P.bytes > scratch_bytes)
        return fail(NSG_EINVAL, "brute-force scratch of %zu bytes, %zu needed", scratch_bytes, P.bytes);
    return bf_launch(P, base, n, queries, nq, d, k, exclude_self, out_ids, out_dist,
                     static_cast<unsigned char *>(scratch), st);
}

}  // namespace nsg

using namespace nsg;

extern "C" int nsg_knn_bruteforce(const float *base, int64_t n, const float *queries, int64_t nq, int32_t d,
                                  int32_t k, int32_t exclude_self, uint32_t *out_ids, float *out_dist,
                                  void *stream) {
    clear_error();
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(NSG_EINVAL, "n out of range");
    if (nq < 0 || nq >= ((int64_t)1 << 31)) return fail(NSG_EINVAL, "nq out of range");
    if (d < 1 || d > 65536) return fail(NSG_EINVAL, "d out of range");
    if (k < 1 || k > 160) return fail(NSG_EINVAL, "k=%d out of range [1, 160]", k);
    if (nq == 0) return NSG_OK;
    if (!base || !queries || !out_ids || !out_dist) return fail(NSG_EINVAL, "NULL pointer");
    if (exclude_self && nq > n) return fail(NSG_EINVAL, "exclude_self needs queries = base rows");
    hipStream_t st = (hipStream_t)stream;
    BFPlan P{};
    if (int rc = bf_plan(base, n, queries, nq, d, k, &P)) return rc;
    // stream-ordered scratch, released on every exit
    unsigned char *ws = nullptr;
    if (hipMallocAsync((void **)&ws, P.bytes, st) != hipSuccess)
        return fail(NSG_ENOMEM, "brute-force scratch allocation of %zu bytes failed", P.bytes);
    const int rc = bf_launch(P, base, n, queries, nq, d, k, exclude_self, out_ids, out_dist, ws, st);
    hipFreeAsync(ws, st);
    return rc;
}
