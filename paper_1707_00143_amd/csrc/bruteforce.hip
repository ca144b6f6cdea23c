// Exact kNN by brute force (serial scan) on gfx950 matrix cores.
//
// Stage 1 (matrix cores): a block owns 64 queries and one contiguous split of
// the base.  For each tile of 64 base rows, the 64x64 block of inner products
// of centred vectors (q - mu).(x - mu) is accumulated with FP32
// v_mfma_f32_16x16x4f32 (each of the 4 waves: 16 queries x 64 rows), turned
// into approximate squared distances |q-mu|^2 + |x-mu|^2 - 2 (q-mu).(x-mu),
// and every value below the query's current threshold is appended to that
// query's candidate buffer (device memory: appends are rare once the
// threshold is tight, and LDS then holds only the staged base chunk, the
// thresholds and a sort scratch per wave, so several blocks share a CU).  A
// buffer that could overflow on the next tile is sorted (in the wave's LDS
// scratch) and cut back to its Kp best, which tightens the threshold (the
// buffer holds Kp + 2 tiles, so sorts are rare once the threshold is tight).
// With d <= 128 each wave keeps its 16 centred queries as matrix-core
// operands in registers for the whole scan and only base rows are staged.
// Each block writes Kp candidates per query for its split.
// Stage 2: per query (one wave), exact FP32 squared distances sum (q_j-x_j)^2
// of all candidates of all splits, bitonic sort by (distance, id), first k.
// Centring keeps the cancellation error of the inner-product form small;
// the over-fetch margin (Kp >= k + 32) absorbs the rest before the exact pass.
#include "common.hpp"

#include <algorithm>

namespace nsg {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BQ = 64, BX = 64, KB = 32, KPAD = 68;

struct BFParams {
    const float *base, *queries;
    const float *mu;       // [d] base mean
    const float *xnorm;    // [n] |x - mu|^2
    const float *qnorm;    // [nq] |q - mu|^2
    int64_t n, nq;
    int d, Kp, cap;
    int64_t split_len;
    int nsplit;
    int exclude_self;
    uint32_t *cand_ids;    // [nq][nsplit][Kp]
    uint64_t *cand_buf;    // [qtiles][nsplit][BQ][cap] candidate buffers
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
    for (int b = 0; b < nblk; ++b) {
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

// sort buf[0..cnt) ascending (padded to cap with +inf), keep the first Kp.
// Executed by one wave.
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

template <bool AREG>
__global__ void __launch_bounds__(256) bf_tile_kernel(BFParams p) {
    extern __shared__ __align__(16) unsigned char smem[];
    float *Xs = reinterpret_cast<float *>(smem);               // [KB][KPAD]
    float *Qs = Xs + KB * KPAD;                                 // [KB][KPAD] (d > 128 only)
    float *thr = Qs + (AREG ? 0 : KB * KPAD);                   // [BQ]
    int *cnt = reinterpret_cast<int *>(thr + BQ);               // [BQ]
    uint64_t *scratch = reinterpret_cast<uint64_t *>(cnt + BQ); // [4][cap]: one sort buffer per wave
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t q0 = (int64_t)blockIdx.x * BQ;
    const int split = blockIdx.y;
    const int64_t xb = (int64_t)split * p.split_len;
    const int64_t xe = std::min<int64_t>(p.n, xb + p.split_len);
    uint64_t *buf = p.cand_buf + ((int64_t)blockIdx.x * p.nsplit + split) * (int64_t)BQ * p.cap;
    uint64_t *sw = scratch + (size_t)w * p.cap;
    if (tid < BQ) { thr[tid] = INFINITY; cnt[tid] = 0; }
    bsync();
    const int rq = lane & 15, kq = lane >> 4;   // MFMA operand row / k group of this lane
    // centred query operands of this wave (AREG: d <= 128, k-step s uses a[s])
    float a_reg[AREG ? 32 : 1];
    if (AREG) {
        const int64_t qi = q0 + 16 * w + rq;
#pragma unroll
        for (int s4 = 0; s4 < (AREG ? 32 : 1); ++s4) {
            const int j = 4 * s4 + kq;
            a_reg[s4] = (qi < p.nq && j < p.d) ? p.queries[qi * p.d + j] - p.mu[j] : 0.0f;
        }
    }
    // |q - mu|^2 of the 4 query rows this lane's accumulators hold
    float qn[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t qi = q0 + 16 * w + 4 * kq + i;
        qn[i] = qi < p.nq ? p.qnorm[qi] : 0.0f;
    }
    // base chunk (64 rows x 32 dims) of the next step, loaded into registers
    // while the matrix cores work on the current one (AREG path)
    float xr[(BX * KB) / 256];
    const int kk_t = tid % KB;   // the dimension offset this thread stages (fixed: 256 % KB == 0)
    auto load_chunk = [&](int64_t cx0, int ck0) {
#pragma unroll
        for (int it = 0; it < (BX * KB) / 256; ++it) {
            const int r = (tid + it * 256) / KB;
            const int j = ck0 + kk_t;
            const int64_t xi = cx0 + r;
            xr[it] = (xi < xe && j < p.d) ? p.base[xi * p.d + j] : 0.0f;
        }
    };
    if (AREG) load_chunk(xb, 0);
    for (int64_t x0 = xb; x0 < xe; x0 += BX) {
        f32x4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k0 = 0; k0 < (AREG ? 128 : 65536); k0 += KB) {
            if (k0 >= p.d) break;   // AREG: a constant trip count keeps a_reg in registers
            if (AREG) {
                // stage the prefetched chunk, centred, k-major; then prefetch the next
                bsync();
                const int j = k0 + kk_t;
                const float mj = j < p.d ? p.mu[j] : 0.0f;
#pragma unroll
                for (int it = 0; it < (BX * KB) / 256; ++it) {
                    const int r = (tid + it * 256) / KB;
                    Xs[kk_t * KPAD + r] = (x0 + r < xe && j < p.d) ? xr[it] - mj : 0.0f;
                }
                bsync();
                const bool more_k = k0 + KB < p.d;
                const int64_t nx0 = more_k ? x0 : x0 + BX;
                if (nx0 < xe) load_chunk(nx0, more_k ? k0 + KB : 0);
            } else {
                // stage centred Q and X chunks, k-major: 64 rows x 32 dims each
#pragma unroll
                for (int it = 0; it < (BQ * KB) / 256; ++it) {
                    int e = tid + it * 256;
                    int r = e / KB, kk = e % KB;
                    int j = k0 + kk;
                    int64_t qi = q0 + r, xi = x0 + r;
                    float mj = j < p.d ? p.mu[j] : 0.0f;
                    Qs[kk * KPAD + r] = (qi < p.nq && j < p.d) ? p.queries[qi * p.d + j] - mj : 0.0f;
                    Xs[kk * KPAD + r] = (xi < xe && j < p.d) ? p.base[xi * p.d + j] - mj : 0.0f;
                }
                bsync();
            }
#pragma unroll
            for (int kk = 0; kk < KB; kk += 4) {
                float a = AREG ? a_reg[((k0 + kk) >> 2) & 31] : Qs[(kk + kq) * KPAD + 16 * w + rq];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    float b = Xs[(kk + kq) * KPAD + 16 * t + rq];
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
                }
            }
            if (!AREG) bsync();
        }
        // epilogue: lane holds rows 4*kq + i of this wave's 16 queries, column rq of tile t
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            int64_t xi = x0 + 16 * t + rq;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int r = 16 * w + 4 * kq + i;
                int64_t qi = q0 + r;
                if (xi < xe && qi < p.nq && !(p.exclude_self && xi == qi)) {
                    float dd = qn[i] + p.xnorm[xi] - 2.0f * acc[t][i];
                    dd = fmaxf(dd, 0.0f);
                    if (dd < thr[r]) {
                        int s = atomicAdd(&cnt[r], 1);
                        buf[(size_t)r * p.cap + s] = bkey(dd, (uint32_t)xi);
                    }
                }
            }
        }
        bsync();
        // compaction when the next tile could overflow: wave w handles queries w, w+4, ...
        for (int r = w; r < BQ; r += 4) {
            int c = cnt[r];
            if (c > p.cap - BX) {
                uint64_t *br = buf + (size_t)r * p.cap;
                for (int j = lane; j < c; j += 64) sw[j] = br[j];
                wave_sort_buf(sw, c, p.cap, lane);
                for (int j = lane; j < p.Kp; j += 64) br[j] = sw[j];
                if (lane == 0) {
                    cnt[r] = p.Kp;
                    thr[r] = __uint_as_float((uint32_t)(sw[p.Kp - 1] >> 32));
                }
            }
        }
        bsync();
    }
    // final: sort each buffer, write Kp candidates (sentinel padded)
    for (int r = w; r < BQ; r += 4) {
        int64_t qi = q0 + r;
        if (qi >= p.nq) continue;
        int c = cnt[r];
        const uint64_t *br = buf + (size_t)r * p.cap;
        for (int j = lane; j < c; j += 64) sw[j] = br[j];
        wave_sort_buf(sw, c, p.cap, lane);
        uint32_t *dst = p.cand_ids + (qi * p.nsplit + split) * (int64_t)p.Kp;
        for (int j = lane; j < p.Kp; j += 64)
            dst[j] = j < c ? (uint32_t)(sw[j] & 0xFFFFFFFFu) : NSG_SENT;
    }
}

// one wave per query: exact distances of all candidates, sort, first k
__global__ void __launch_bounds__(256) bf_rerank_kernel(const float *base, const float *queries, int64_t nq,
                                                        int d, const uint32_t *cand, int ncand, int k,
                                                        int sort_n, uint32_t *out_ids, float *out_dist) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t qi = (int64_t)blockIdx.x * (blockDim.x >> 6) + w;
    uint64_t *a = reinterpret_cast<uint64_t *>(smem) + (size_t)w * sort_n;
    if (qi >= nq) return;
    const float *q = queries + qi * d;
    const uint32_t *c = cand + qi * (int64_t)ncand;
    const int g = lane >> 4, li = lane & 15;
    for (int r0 = 0; r0 < sort_n; r0 += 4) {
        int r = r0 + g;
        uint32_t id = r < ncand ? c[r] : NSG_SENT;
        float acc = 0.0f;
        if (id != NSG_SENT) {
            const float *x = base + (int64_t)id * d;
            for (int j = li; j < d; j += 16) {
                float t = q[j] - x[j];
                acc = fmaf(t, t, acc);
            }
        }
        for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (li == 0) a[r] = id == NSG_SENT ? ~0ull : bkey(acc, id);
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

int launch_mean(const float *x, int64_t n, int d, float *mu, float2 *part, hipStream_t st) {
    const int nblk = mean_blocks(n);
    hipLaunchKernelGGL(colsum_part_kernel, dim3((unsigned)nblk), dim3(d < 256 ? (d + 63) / 64 * 64 : 256), 0, st,
                       x, n, d, part);
    hipLaunchKernelGGL(mean_finish_kernel, dim3((d + 255) / 256), dim3(256), 0, st, part, nblk, n, d, mu);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(NSG_EDEVICE, "mean kernels failed: %s", hipGetErrorString(e));
    return NSG_OK;
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
    // over-fetch margin 24 for the inner-product form's rounding; buffer of
    // Kp + two tiles (next power of two)
    const int Kp = (k + 24 + 31) / 32 * 32;
    int cap = 1;
    while (cap < Kp + 2 * BX) cap <<= 1;
    // splits: enough blocks to fill the machine, at least a few tiles each
    int64_t qtiles = (nq + BQ - 1) / BQ;
    int64_t want = std::max<int64_t>(1, 2048 / std::max<int64_t>(qtiles, 1));
    int64_t max_split = std::max<int64_t>(1, n / (BX * 8));
    int nsplit = (int)std::min<int64_t>(std::min<int64_t>(want, max_split), std::max(1, 4096 / Kp));
    int64_t split_len = (n + nsplit - 1) / nsplit;
    split_len = (split_len + BX - 1) / BX * BX;
    nsplit = (int)((n + split_len - 1) / split_len);
    const int ncand = nsplit * Kp;
    int sort_n = 1;
    while (sort_n < ncand) sort_n <<= 1;
    if (sort_n * 8 > 64 * 1024) return fail(NSG_EUNSUPPORTED, "too many candidates per query (%d)", ncand);
    float *mu = nullptr, *xnorm = nullptr, *qnorm = nullptr;
    float2 *acc = nullptr;
    uint32_t *cand = nullptr;
    uint64_t *cbuf = nullptr;
    NSG_HIP(hipMallocAsync((void **)&acc, sizeof(float2) * d * mean_blocks(n), st));
    NSG_HIP(hipMallocAsync((void **)&mu, sizeof(float) * d, st));
    NSG_HIP(hipMallocAsync((void **)&xnorm, sizeof(float) * n, st));
    NSG_HIP(hipMallocAsync((void **)&qnorm, sizeof(float) * nq, st));
    NSG_HIP(hipMallocAsync((void **)&cand, sizeof(uint32_t) * nq * ncand, st));
    NSG_HIP(hipMallocAsync((void **)&cbuf, sizeof(uint64_t) * qtiles * nsplit * BQ * cap, st));
    if (int rc = launch_mean(base, n, d, mu, acc, st)) return rc;
    hipLaunchKernelGGL(cnorm_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, base, n, d, mu, xnorm);
    hipLaunchKernelGGL(cnorm_kernel, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, st, queries, nq, d, mu, qnorm);
    BFParams p{};
    p.base = base;
    p.queries = queries;
    p.mu = mu;
    p.xnorm = xnorm;
    p.qnorm = qnorm;
    p.n = n;
    p.nq = nq;
    p.d = d;
    p.Kp = Kp;
    p.cap = cap;
    p.split_len = split_len;
    p.nsplit = nsplit;
    p.exclude_self = exclude_self ? 1 : 0;
    p.cand_ids = cand;
    p.cand_buf = cbuf;
    const size_t lds = (size_t)(d <= 128 ? 1 : 2) * KB * KPAD * 4 + BQ * 8 + (size_t)4 * cap * 8;
    if (d <= 128) {
        NSG_HIP(hipFuncSetAttribute((const void *)bf_tile_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds));
        hipLaunchKernelGGL(bf_tile_kernel<true>, dim3((unsigned)qtiles, (unsigned)nsplit), dim3(256), lds, st, p);
    } else {
        NSG_HIP(hipFuncSetAttribute((const void *)bf_tile_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds));
        hipLaunchKernelGGL(bf_tile_kernel<false>, dim3((unsigned)qtiles, (unsigned)nsplit), dim3(256), lds, st, p);
    }
    const int wpb = std::max(1, std::min(4, (int)(64 * 1024 / ((size_t)sort_n * 8))));
    hipLaunchKernelGGL(bf_rerank_kernel, dim3((unsigned)((nq + wpb - 1) / wpb)), dim3(64 * wpb),
                       (size_t)sort_n * 8 * wpb, st, base, queries, nq, d, cand, ncand, k, sort_n, out_ids, out_dist);
    hipError_t e = hipGetLastError();
    hipFreeAsync(acc, st);
    hipFreeAsync(mu, st);
    hipFreeAsync(xnorm, st);
    hipFreeAsync(qnorm, st);
    hipFreeAsync(cand, st);
    hipFreeAsync(cbuf, st);
    if (e != hipSuccess) return fail(NSG_EDEVICE, "brute-force launch failed: %s", hipGetErrorString(e));
    return NSG_OK;
}
