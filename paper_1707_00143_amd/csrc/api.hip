// C ABI of libnsg.so: index residency, argument checks, error reporting and
// the search entry points.  Kernels live in the other sources of this library.
#include "common.hpp"

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>
#include <cmath>

namespace nsg {

static thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = 0; }

// ---------------------------------------------------------------------------
// load-time kernels: padding fill, graph validation, per-dimension scales,
// reduced-precision encoding
// ---------------------------------------------------------------------------
__global__ void fill_u32_kernel(uint32_t *p, int64_t cnt, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void validate_graph_kernel(const uint32_t *g, int64_t n, int R, int R_pad,
                                      unsigned long long *bad) {
    unsigned long long cnt = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * R;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t v = i / R;
        int j = (int)(i % R);
        uint32_t u = g[v * R_pad + j];
        if (u != NSG_SENT && (int64_t)u >= n) ++cnt;
    }
    if (cnt) atomicAdd(bad, cnt);
}

// column max |x_ij| as FP32 bits (non-negative floats order like their bits):
// block b takes rows b, b + gridDim.x, ...; threads walk a row's dimensions
__global__ void colmax_kernel(const float *x, int64_t n, int d, int ld, unsigned int *mx) {
    for (int j0 = 0; j0 < d; j0 += blockDim.x) {
        int j = j0 + threadIdx.x;
        float m = 0.0f;
        if (j < d)
            for (int64_t i = blockIdx.x; i < n; i += gridDim.x) m = fmaxf(m, fabsf(x[i * ld + j]));
        if (j < d) atomicMax(&mx[j], __float_as_uint(m));
    }
}

// s_j = max_i |x_ij| / M, or 1 for an all-zero column
__global__ void scales_finish_kernel(const unsigned int *mx, int d, float M, float *s) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < d) {
        float m = __uint_as_float(mx[j]);
        s[j] = m > 0.0f ? m / M : 1.0f;
    }
}

// round-to-nearest-even encoders with saturation to the largest finite value
__device__ inline uint32_t enc_f16(float x) {
    if (isnan(x)) return 0x7E00u | (signbit(x) ? 0x8000u : 0u);
    x = fminf(fmaxf(x, -65504.0f), 65504.0f);
    return (uint32_t)__builtin_bit_cast(unsigned short, (_Float16)x);
}

__device__ inline uint32_t enc_bf16(float x) {
    uint32_t sgn = __float_as_uint(x) & 0x80000000u;
    if (isnan(x)) return (sgn >> 16) | 0x7FC0u;
    const float mx = __uint_as_float(0x7F7F0000u);
    x = fminf(fmaxf(x, -mx), mx);
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

__device__ inline uint32_t enc_e4m3(float x) {
    uint32_t sgn = (__float_as_uint(x) >> 24) & 0x80u;
    if (isnan(x)) return sgn | 0x7Fu;
    float a = fminf(fabsf(x), 448.0f);
    if (a < 0x1p-6f) {                              // subnormal binade: quantum 2^-9
        uint32_t r = (uint32_t)rintf(a * 512.0f);     // 0..8; 8 is the smallest normal
        return sgn | r;
    }
    int e = (int)((__float_as_uint(a) >> 23) & 0xFFu) - 127;   // a in [2^e, 2^(e+1))
    float r = rintf(a * __uint_as_float((uint32_t)(127 - (e - 3)) << 23));  // a / 2^(e-3), in [8, 16]
    uint32_t ri = (uint32_t)r;
    if (ri == 16u) { e += 1; ri = 8u; }
    return sgn | ((uint32_t)(e + 7) << 3) | (ri - 8u);
}

// codes[n][row_chunks * EPC] from x[n][d] (ld floats per row) and s[d]
__global__ void encode_kernel(const float *x, int64_t n, int d, int ld, const float *s, int storage,
                              void *codes, int row_elems) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * row_elems;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t v = i / row_elems;
        int j = (int)(i % row_elems);
        uint32_t c = 0;
        if (j < d) {
            float y = x[v * ld + j] / s[j];
            c = storage == NSG_F16 ? enc_f16(y) : storage == NSG_BF16 ? enc_bf16(y) : enc_e4m3(y);
        }
        if (storage == NSG_E4M3) reinterpret_cast<uint8_t *>(codes)[i] = (uint8_t)c;
        else reinterpret_cast<uint16_t *>(codes)[i] = (uint16_t)c;
    }
}

// Bound E of the index for the prefix re-rank: the maximum over rows of
// ||xhat - x|| + 2^-22 ||xhat||, where xhat is the stored row as the search
// decodes it (code times scale; the FP32 row itself for FP32 storage).  The
// first term bounds | ||q - x|| - ||q - xhat|| | (triangle inequality); the
// second covers a decode whose product s * c is rounded before the
// difference.  Each row sum is scaled by 1 + 2^-12 for its own rounding
// (d <= 1024 additions, one rounding per difference and per sqrt).  One
// wave per row; the maximum is kept per wave, then per block (LDS), and one
// atomic max per block leaves it as the float bit pattern in *out
// (non-negative floats order like their bits).  Block size 256.
__global__ void rr_eta_kernel(const float *x, int64_t n, int d, int ld, const float *s, int storage,
                              const void *codes, int row_elems, unsigned int *out) {
    __shared__ unsigned int wmax[4];
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    unsigned int best = 0u;
    for (int64_t r = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); r < n; r += waves) {
        float S = 0.0f, N = 0.0f;
        for (int j = lane; j < d; j += 64) {
            const float xv = x[r * ld + j];
            float c = xv, sj = 1.0f;
            if (storage != NSG_F32) {
                const int64_t e = r * row_elems + j;
                if (storage == NSG_F16)
                    c = (float)__builtin_bit_cast(_Float16, reinterpret_cast<const uint16_t *>(codes)[e]);
                else if (storage == NSG_BF16)
                    c = __uint_as_float((uint32_t)reinterpret_cast<const uint16_t *>(codes)[e] << 16);
                else
                    c = __builtin_amdgcn_cvt_pk_f32_fp8((int)reinterpret_cast<const uint8_t *>(codes)[e], false)[0];
                sj = s[j];
            }
            const float t = fmaf(sj, c, -xv);
            const float h = sj * c;
            S = fmaf(t, t, S);
            N = fmaf(h, h, N);
        }
        for (int o = 32; o > 0; o >>= 1) {
            S += __shfl_xor(S, o);
            N += __shfl_xor(N, o);
        }
        const float eta = (sqrtf(S) + 0x1p-22f * sqrtf(N)) * (1.0f + 0x1p-12f);
        const unsigned int b = __float_as_uint(eta);
        best = b > best ? b : best;
    }
    if (lane == 0) wmax[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int m = wmax[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = wmax[w] > m ? wmax[w] : m;
        atomicMax(out, m);
    }
}

static int grid_for(int64_t cnt) {
    int64_t b = (cnt + 255) / 256;
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 65536);
}

const int64_t kPersistentMinBatch = 4096;
// batches that fill the chip's wave slots more than once: longest walks first
const int64_t kLongestFirstMinBatch = 8192;

// a query visits roughly 25 nodes per pool entry; size the filter to that
// (it forgets beyond, which only costs recomputation)
int default_hash_bits(int L) {
    // 24 L slots, within [1024, 2048]: a larger filter forgets fewer nodes
    // (fewer repeated distance evaluations) but its LDS lowers the number of
    // resident wavefronts, which costs more at every pool size measured
    int want = L * 24, bits = 10;
    while ((1 << bits) < want && bits < 11) ++bits;
    return bits;
}

}  // namespace nsg

using namespace nsg;

extern "C" const char *nsg_last_error(void) { return g_err; }

extern "C" int nsg_index_info(const nsg_index *idx, int64_t *n, int32_t *d, int32_t *R,
                              uint32_t *nav, int32_t *storage) {
    if (!idx) return fail(NSG_EINVAL, "index is NULL");
    if (n) *n = idx->n;
    if (d) *d = idx->d;
    if (R) *R = idx->R;
    if (nav) *nav = idx->nav;
    if (storage) *storage = idx->storage;
    return NSG_OK;
}

extern "C" void nsg_free_index(nsg_index *idx) {
    if (!idx) return;
    hipDeviceSynchronize();
    hipFree(idx->base_f32);
    hipFree(idx->base_lp);
    hipFree(idx->scales);
    hipFree(idx->graph);
    hipFree(idx->stop.blob);
    delete idx;
}

extern "C" int nsg_load_index(const float *base, int64_t n, int32_t d, const uint32_t *graph,
                              int32_t R, uint32_t nav_node, nsg_dtype storage, const float *scales,
                              void *stream, nsg_index **out) {
    clear_error();
    if (!out) return fail(NSG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!base || !graph) return fail(NSG_EINVAL, "base or graph is NULL");
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(NSG_EINVAL, "n=%lld out of range [1, 2^31)", (long long)n);
    if (d < 1 || d > kMaxD) return fail(NSG_EINVAL, "d=%d out of range [1, %d]", d, kMaxD);
    if (R < 1 || R > kMaxR) return fail(NSG_EINVAL, "R=%d out of range [1, %d]", R, kMaxR);
    if ((int64_t)nav_node >= n) return fail(NSG_EINVAL, "navigating node %u >= n", nav_node);
    if (storage < NSG_F32 || storage > NSG_E4M3) return fail(NSG_EINVAL, "unknown storage %d", (int)storage);
    hipStream_t st = (hipStream_t)stream;
    nsg_index *ix = new nsg_index();
    ix->n = n;
    ix->d = d;
    ix->R = R;
    ix->R_pad = (R + 31) / 32 * 32;
    ix->nav = nav_node;
    ix->storage = storage;
    ix->row_chunks_f32 = (d + 3) / 4;
    const int epc = elems_per_chunk(storage);
    ix->row_chunks = (d + epc - 1) / epc;
    hipGetDevice(&ix->device);
    const int ld32 = ix->row_chunks_f32 * 4;
    auto cleanup = [&](int rc) { nsg_free_index(ix); return rc; };
    // row tables carry kRowTailBytes of zeros past the last row (gathers read
    // a row group's full width at any row)
    const size_t f32_bytes = sizeof(float) * n * ld32;
    if (hipMalloc(&ix->base_f32, f32_bytes + kRowTailBytes) != hipSuccess ||
        hipMalloc(&ix->graph, sizeof(uint32_t) * n * ix->R_pad) != hipSuccess)
        return cleanup(fail(NSG_ENOMEM, "device allocation of the index failed"));
    hipError_t e = hipMemsetAsync((char *)ix->base_f32 + f32_bytes, 0, kRowTailBytes, st);
    if (e == hipSuccess && ld32 != d) e = hipMemsetAsync(ix->base_f32, 0, f32_bytes, st);
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(ix->base_f32, sizeof(float) * ld32, base, sizeof(float) * d,
                             sizeof(float) * d, n, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n * ix->R_pad)), dim3(256), 0, st,
                           ix->graph, n * ix->R_pad, NSG_SENT);
        e = hipMemcpy2DAsync(ix->graph, sizeof(uint32_t) * ix->R_pad, graph, sizeof(uint32_t) * R,
                             sizeof(uint32_t) * R, n, hipMemcpyDeviceToDevice, st);
    }
    if (e != hipSuccess) return cleanup(fail(NSG_EDEVICE, "index copy failed: %s", hipGetErrorString(e)));
    unsigned long long *bad = nullptr, hbad = 0;
    if (hipMalloc(&bad, sizeof(*bad)) != hipSuccess) return cleanup(fail(NSG_ENOMEM, "alloc failed"));
    hipMemsetAsync(bad, 0, sizeof(*bad), st);
    hipLaunchKernelGGL(validate_graph_kernel, dim3(grid_for(n * R)), dim3(256), 0, st, ix->graph, n, R,
                       ix->R_pad, bad);
    e = hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipFree(bad);
    if (e != hipSuccess) return cleanup(fail(NSG_EDEVICE, "graph validation failed: %s", hipGetErrorString(e)));
    if (hbad) return cleanup(fail(NSG_EINVAL, "%llu graph entries are neither < n nor the sentinel", hbad));
    if (hipMalloc(&ix->scales, sizeof(float) * ld32) != hipSuccess)
        return cleanup(fail(NSG_ENOMEM, "alloc failed"));
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(256), 0, st, reinterpret_cast<uint32_t *>(ix->scales),
                       (int64_t)ld32, 0x3F800000u /* 1.0f */);
    if (storage != NSG_F32) {
        if (scales) {
            e = hipMemcpyAsync(ix->scales, scales, sizeof(float) * d, hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return cleanup(fail(NSG_EDEVICE, "scale copy failed"));
        } else {
            unsigned int *mx = nullptr;
            if (hipMalloc(&mx, sizeof(unsigned int) * d) != hipSuccess) return cleanup(fail(NSG_ENOMEM, "alloc failed"));
            hipMemsetAsync(mx, 0, sizeof(unsigned int) * d, st);
            hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)std::min<int64_t>(n, 1024)),
                               dim3(d < 256 ? (d + 63) / 64 * 64 : 256), 0, st, ix->base_f32, n, d, ld32, mx);
            hipLaunchKernelGGL(scales_finish_kernel, dim3((d + 255) / 256), dim3(256), 0, st, mx, d,
                               storage == NSG_E4M3 ? 448.0f : 1.0f, ix->scales);
            hipStreamSynchronize(st);
            hipFree(mx);
        }
        const int row_elems = ix->row_chunks * epc;
        const size_t esz = storage == NSG_E4M3 ? 1 : 2;
        const size_t lp_bytes = esz * n * row_elems;
        if (hipMalloc(&ix->base_lp, lp_bytes + kRowTailBytes) != hipSuccess)
            return cleanup(fail(NSG_ENOMEM, "alloc of reduced rows failed"));
        if (hipMemsetAsync((char *)ix->base_lp + lp_bytes, 0, kRowTailBytes, st) != hipSuccess)
            return cleanup(fail(NSG_EDEVICE, "clearing the row tail failed"));
        hipLaunchKernelGGL(encode_kernel, dim3(grid_for(n * row_elems)), dim3(256), 0, st, ix->base_f32, n, d,
                           ld32, ix->scales, (int)storage, ix->base_lp, row_elems);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return cleanup(fail(NSG_EDEVICE, "load kernels failed: %s", hipGetErrorString(e)));
    {
        unsigned int *dmax = nullptr, hmax = 0;
        if (hipMalloc(&dmax, sizeof(*dmax)) != hipSuccess) return cleanup(fail(NSG_ENOMEM, "alloc failed"));
        e = hipMemsetAsync(dmax, 0, sizeof(*dmax), st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(rr_eta_kernel, dim3((unsigned)std::min<int64_t>((n + 3) / 4, 8192)), dim3(256), 0, st,
                               ix->base_f32, n, d, ld32, ix->scales, (int)storage, ix->base_lp,
                               ix->row_chunks * epc, dmax);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(&hmax, dmax, sizeof(hmax), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        hipFree(dmax);
        if (e != hipSuccess) return cleanup(fail(NSG_EDEVICE, "re-rank bound failed: %s", hipGetErrorString(e)));
        const float eta = __builtin_bit_cast(float, hmax);
        ix->rr_eta = eta < INFINITY ? eta : -1.0f;   // NaN or inf rows: re-rank whole pools
    }
    *out = ix;
    return NSG_OK;
}

static int check_search_common(const nsg_index *idx, const float *queries, int64_t nq,
                               const void *ids, const void *dist) {
    if (!idx) return fail(NSG_EINVAL, "index is NULL");
    if (nq < 0) return fail(NSG_EINVAL, "nq=%lld < 0", (long long)nq);
    if (nq >= ((int64_t)1 << 31)) return fail(NSG_EINVAL, "nq too large");
    if (nq > 0 && (!queries || !ids || !dist)) return fail(NSG_EINVAL, "NULL query or output pointer");
    return NSG_OK;
}

static int stop_ready(const nsg_index *idx) { return idx->stop.enabled && idx->stop.blob; }


extern "C" int nsg_search(const nsg_index *idx, const float *queries, int64_t nq, int32_t k, int32_t L,
                          uint32_t *out_ids, float *out_dist, void *stream) {
    clear_error();
    int rc = check_search_common(idx, queries, nq, out_ids, out_dist);
    if (rc) return rc;
    if (k < 1 || k > kMaxK) return fail(NSG_EINVAL, "k=%d out of range [1, %d]", k, kMaxK);
    if (L < 1 || L > kMaxL) return fail(NSG_EINVAL, "L=%d out of range [1, %d]", L, kMaxL);
    if (nq == 0) return NSG_OK;
    SearchArgs a{};
    a.idx = idx;
    a.queries = queries;
    a.nq = nq;
    a.k_scalar = k;
    a.L_scalar = L;
    a.out_stride = k;
    a.out_ids = out_ids;
    a.out_dist = out_dist;
    a.learned = stop_ready(idx) && L >= 16;
    a.L_cap = L;
    a.hash_bits = default_hash_bits(L);
    a.rerank = idx->storage != NSG_F32;
    // large batches: persistent grid (work stealing evens out per-query cost)
    a.persistent = nq >= kPersistentMinBatch;
    a.longest_first = nq >= kLongestFirstMinBatch;
    a.start_override = NSG_SENT;
    a.self_offset = -1;
    a.stream = (hipStream_t)stream;
    return launch_search(a);
}

// visited-filter size of a batched call: the caller's, else the default for L
static int opts_hash_bits(int L_cap, const nsg_search_opts &o) {
    int hb = default_hash_bits(L_cap);
    if (o.hash_slots) { hb = 0; while ((1 << hb) < o.hash_slots) ++hb; }
    return hb;
}

extern "C" int nsg_search_batched(const nsg_index *idx, const float *queries, int64_t nq, const int32_t *k,
                                  const int32_t *L, int32_t k_scalar, int32_t L_scalar, int32_t out_stride,
                                  uint32_t *out_ids, float *out_dist, const nsg_search_opts *opts,
                                  void *stream) {
    clear_error();
    int rc = check_search_common(idx, queries, nq, out_ids, out_dist);
    if (rc) return rc;
    if (L_scalar < 1 || L_scalar > kMaxL)
        return fail(NSG_EINVAL, "L_scalar=%d out of range [1, %d] (it bounds every L[i])", L_scalar, kMaxL);
    if (!k && (k_scalar < 1 || k_scalar > kMaxK)) return fail(NSG_EINVAL, "k_scalar=%d out of range", k_scalar);
    if (out_stride < 1 || out_stride > kMaxK || (!k && out_stride < k_scalar))
        return fail(NSG_EINVAL, "out_stride=%d invalid", out_stride);
    nsg_search_opts o{};
    if (opts) o = *opts;
    if (o.hash_slots && (o.hash_slots & (o.hash_slots - 1)))
        return fail(NSG_EINVAL, "hash_slots must be a power of two");
    if (o.hash_slots && (o.hash_slots < 64 || o.hash_slots > 16384))
        return fail(NSG_EINVAL, "hash_slots out of range [64, 16384]");
    if (o.waves_per_block < 0 || o.waves_per_block > 4)
        return fail(NSG_EINVAL, "waves_per_block=%d out of range [0, 4]", o.waves_per_block);
    if (o.pool_ids && (o.pool_stride < 1 || !o.pool_dist)) return fail(NSG_EINVAL, "pool output needs stride and dist");
    if (o.learned_stop < 0 || o.learned_stop > 1) return fail(NSG_EINVAL, "learned_stop must be 0 or 1");
    if (o.learned_stop && !stop_ready(idx)) return fail(NSG_ESTATE, "no early-stop model loaded and enabled");
    if (o.feature_hop < 0 || o.feature_hop > 65535) return fail(NSG_EINVAL, "feature_hop out of [0, 65535]");
    if (o.max_hops < 0) return fail(NSG_EINVAL, "max_hops < 0");
    if (o.lanes_per_row && o.lanes_per_row != 8 && o.lanes_per_row != 16 && o.lanes_per_row != 32 &&
        o.lanes_per_row != 64)
        return fail(NSG_EINVAL, "lanes_per_row must be 0, 8, 16, 32 or 64");
    if (o.blocks < 0) return fail(NSG_EINVAL, "blocks < 0");
    if (o.init_n < 0 || o.init_n > kMaxL) return fail(NSG_EINVAL, "init_n=%d out of range [0, %d]", o.init_n, kMaxL);
    if (o.init_n > 0 && !o.init_ids) return fail(NSG_EINVAL, "init_n > 0 needs init_ids");
    if (o.longest_first != 0 && o.longest_first != 1) return fail(NSG_EINVAL, "longest_first must be 0 or 1");
    if (nq == 0) return NSG_OK;
    SearchArgs a{};
    a.idx = idx;
    a.queries = queries;
    a.nq = nq;
    a.k_arr = k;
    a.L_arr = L;
    a.k_scalar = k_scalar;
    a.L_scalar = L_scalar;
    a.out_stride = out_stride;
    a.out_ids = out_ids;
    a.out_dist = out_dist;
    a.learned = o.learned_stop;
    a.L_cap = L_scalar;
    a.hash_bits = opts_hash_bits(a.L_cap, o);
    a.waves_per_block = o.waves_per_block;
    a.persistent = o.persistent;
    a.blocks = o.blocks;
    a.rerank = o.rerank == 0 ? (idx->storage != NSG_F32) : (o.rerank > 0);
    a.hops = o.hops;
    a.ndist = o.ndist;
    a.budget = o.budget;
    a.max_hops = o.max_hops;
    a.features = o.features;
    a.feature_hop = o.feature_hop;
    a.nedges = o.nedges;
    a.lanes_per_row = o.lanes_per_row;
    a.counter = o.counter;
    a.longest_first = o.longest_first;
    a.order_scratch = o.order_scratch;
    a.clamped = o.clamped;
    a.init_ids = o.init_ids;
    a.init_n = o.init_n;
    a.pool_ids = o.pool_ids;
    a.pool_dist = o.pool_dist;
    a.pool_stride = o.pool_stride;
    a.start_override = NSG_SENT;
    a.self_offset = -1;
    a.stream = (hipStream_t)stream;
    return launch_search(a);
}


// ---------------------------------------------------------------------------
// learned early stop: model residency
// ---------------------------------------------------------------------------
extern "C" int nsg_load_stop_model(nsg_index *idx, const void *blob, size_t bytes, int32_t kind, int32_t in,
                                   int32_t h, int32_t hop, int32_t grid_n) {
    clear_error();
    if (!idx || !blob) return fail(NSG_EINVAL, "NULL index or blob");
    if (idx->stop_graphs.load() > 0)
        return fail(NSG_ESTATE, "%d search graph(s) captured with the early stop still use the model",
                    idx->stop_graphs.load());
    if (kind != NSG_STOP_SCALAR && kind != NSG_STOP_QUERY) return fail(NSG_EINVAL, "unknown model kind %d", kind);
    const int want_in = kind == NSG_STOP_SCALAR ? kStopFeatures : idx->d + 3;
    if (in != want_in) return fail(NSG_EINVAL, "model input %d must be %d for this kind", in, want_in);
    if (h < 1 || h > 64) return fail(NSG_EUNSUPPORTED, "hidden width %d outside [1, 64]", h);
    if (hop < 1 || hop > 65535) return fail(NSG_EINVAL, "hop must be in [1, 65535]");
    if (grid_n < 1 || grid_n > 256) return fail(NSG_EINVAL, "grid_n out of range [1, 256]");
    const size_t nf = (size_t)2 * in + (size_t)h * in + h + (size_t)h * h + h + h + 1 + grid_n;
    if (bytes != nf * sizeof(float)) return fail(NSG_EINVAL, "blob has %zu bytes, expected %zu", bytes, nf * 4);
    const float *b = static_cast<const float *>(blob);
    const float *grid = b + nf - grid_n;
    for (int i = 0; i < grid_n; ++i) {
        if (!(grid[i] >= 1.0f && grid[i] <= 1048576.0f)) return fail(NSG_EINVAL, "grid value out of [1, 2^20]");
        if (i && grid[i] <= grid[i - 1]) return fail(NSG_EINVAL, "grid must be strictly ascending");
    }
    // kernel layout of the form (hidden units past h are zero):
    //  scalar: W1T[in][64], W2T[64][64], b1[64], b2[64], W3[64], b3, mean[in], inv_std[in], grid
    //  query:  W1[(in+1)/2][64] and W2[32][64] as FP16 pairs, then the same FP32 tail (W3 FP16-rounded)
    const float *mean = b, *istd = b + in, *W1 = istd + in, *b1 = W1 + (size_t)h * in, *W2 = b1 + h;
    const float *b2 = W2 + (size_t)h * h, *W3 = b2 + h, *b3 = W3 + h;
    const size_t w1_words = kind == NSG_STOP_SCALAR ? (size_t)in * 64 : (size_t)((in + 1) / 2) * 64;
    const size_t w2_words = kind == NSG_STOP_SCALAR ? 64 * 64 : 32 * 64;
    std::vector<float> pl(w1_words + w2_words + 3 * 64 + 1 + 2 * (size_t)in + grid_n, 0.0f);
    float *pW1T = pl.data(), *pW2T = pW1T + w1_words, *pb1 = pW2T + w2_words, *pb2 = pb1 + 64;
    float *pW3 = pb2 + 64, *pb3 = pW3 + 64, *pmean = pb3 + 1, *pistd = pmean + in, *pgrid = pistd + in;
    auto f16 = [](float v) -> uint16_t { return __builtin_bit_cast(uint16_t, (_Float16)v); };
    for (int j = 0; j < h; ++j) {
        if (kind == NSG_STOP_SCALAR) {
            for (int i = 0; i < in; ++i) pW1T[(size_t)i * 64 + j] = W1[(size_t)j * in + i];
            for (int k = 0; k < h; ++k) pW2T[(size_t)k * 64 + j] = W2[(size_t)j * h + k];
            pW3[j] = W3[j];
        } else {
            uint32_t *w1 = reinterpret_cast<uint32_t *>(pW1T), *w2 = reinterpret_cast<uint32_t *>(pW2T);
            for (int i = 0; i < in; i += 2) {
                const uint32_t hi = i + 1 < in ? f16(W1[(size_t)j * in + i + 1]) : 0u;
                w1[(size_t)(i / 2) * 64 + j] = f16(W1[(size_t)j * in + i]) | hi << 16;
            }
            for (int k = 0; k < h; k += 2) {
                const uint32_t hi = k + 1 < h ? f16(W2[(size_t)j * h + k + 1]) : 0u;
                w2[(size_t)(k / 2) * 64 + j] = f16(W2[(size_t)j * h + k]) | hi << 16;
            }
            pW3[j] = (float)(_Float16)W3[j];
        }
        pb1[j] = b1[j];
        pb2[j] = b2[j];
    }
    *pb3 = *b3;
    for (int i = 0; i < in; ++i) {
        pmean[i] = mean[i];
        pistd[i] = istd[i];
    }
    for (int i = 0; i < grid_n; ++i) pgrid[i] = grid[i];
    StopModel sm;
    if (hipMalloc(&sm.blob, pl.size() * 4) != hipSuccess) return fail(NSG_ENOMEM, "model allocation failed");
    hipError_t e = hipMemcpy(sm.blob, pl.data(), pl.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(sm.blob);
        return fail(NSG_EDEVICE, "model copy failed: %s", hipGetErrorString(e));
    }
    sm.kind = kind;
    sm.in = in;
    sm.h = h;
    sm.ncp = 1;
    sm.cps[0] = hop;
    sm.hop = hop;
    sm.grid_n = grid_n;
    sm.enabled = idx->stop.enabled;
    sm.calib_c = idx->stop.calib_c;
    hipDeviceSynchronize();
    hipFree(idx->stop.blob);
    idx->stop = sm;
    return NSG_OK;
}

extern "C" int nsg_set_stop_checkpoints(nsg_index *idx, const int32_t *hops, int32_t n) {
    clear_error();
    if (!idx || !hops) return fail(NSG_EINVAL, "NULL index or checkpoints");
    if (!idx->stop.blob) return fail(NSG_ESTATE, "no early-stop model loaded");
    if (idx->stop_graphs.load() > 0)
        return fail(NSG_ESTATE, "%d search graph(s) captured with the early stop hold its checkpoints",
                    idx->stop_graphs.load());
    if (n < 1 || n > 4) return fail(NSG_EINVAL, "%d checkpoints, expected 1 to 4", n);
    for (int c = 0; c < n; ++c) {
        if (hops[c] < 1 || hops[c] > 65535) return fail(NSG_EINVAL, "checkpoint %d out of [1, 65535]", hops[c]);
        if (c && hops[c] <= hops[c - 1]) return fail(NSG_EINVAL, "checkpoints must be strictly ascending");
    }
    idx->stop.ncp = n;
    for (int c = 0; c < 4; ++c) idx->stop.cps[c] = c < n ? hops[c] : 0;
    idx->stop.hop = hops[0];
    return NSG_OK;
}

extern "C" int nsg_set_stop_mode(nsg_index *idx, int32_t enabled, float calib_c) {
    clear_error();
    if (!idx) return fail(NSG_EINVAL, "index is NULL");
    if (idx->stop_graphs.load() > 0)
        return fail(NSG_ESTATE, "%d search graph(s) captured with the early stop hold its calibration",
                    idx->stop_graphs.load());
    if (enabled && !idx->stop.blob) return fail(NSG_ESTATE, "no early-stop model loaded");
    if (!(calib_c > 0.0f) || !std::isfinite(calib_c)) return fail(NSG_EINVAL, "calibration must be finite and > 0");
    idx->stop.enabled = enabled ? 1 : 0;
    idx->stop.calib_c = calib_c;
    return NSG_OK;
}

// ---------------------------------------------------------------------------
// batches as HIP graphs
// ---------------------------------------------------------------------------
struct nsg_search_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned int *counter = nullptr;
    uint32_t *order = nullptr;             // scratch of the longest-first order
    const nsg_index *stop_idx = nullptr;   // index whose early-stop model the graph holds
};

extern "C" void nsg_search_graph_destroy(nsg_search_graph *g) {
    if (!g) return;
    hipDeviceSynchronize();
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    hipFree(g->counter);
    hipFree(g->order);
    if (g->stop_idx) g->stop_idx->stop_graphs.fetch_sub(1);
    delete g;
}

extern "C" int nsg_search_graph_create(const nsg_index *idx, const float *queries, int64_t nq, const int32_t *k,
                                       const int32_t *L, int32_t k_scalar, int32_t L_scalar, int32_t out_stride,
                                       uint32_t *out_ids, float *out_dist, const nsg_search_opts *opts,
                                       nsg_search_graph **out) {
    clear_error();
    if (!out) return fail(NSG_EINVAL, "out is NULL");
    *out = nullptr;
    if (nq < 1) return fail(NSG_EINVAL, "a captured batch needs nq >= 1");
    nsg_search_graph *g = new nsg_search_graph();
    nsg_search_opts o{};
    if (opts) o = *opts;
    if (o.persistent && !o.counter) {
        if (hipMalloc(&g->counter, sizeof(unsigned int) * 64) != hipSuccess) {
            delete g;
            return fail(NSG_ENOMEM, "counter allocation failed");
        }
        o.counter = g->counter;
    }
    if (o.longest_first && !o.order_scratch) {
        if (hipMalloc(&g->order, sizeof(uint32_t) * 2 * NSG_ORDER_MAX) != hipSuccess) {
            nsg_search_graph_destroy(g);
            return fail(NSG_ENOMEM, "order scratch allocation failed");
        }
        o.order_scratch = g->order;
    }
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        nsg_search_graph_destroy(g);
        return fail(NSG_EDEVICE, "stream creation failed");
    }
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    int rc = NSG_OK;
    if (e == hipSuccess) {
        rc = nsg_search_batched(idx, queries, nq, k, L, k_scalar, L_scalar, out_stride, out_ids, out_dist, &o, cs);
        hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
        if (rc == NSG_OK && e2 != hipSuccess) rc = fail(NSG_EDEVICE, "capture failed: %s", hipGetErrorString(e2));
    } else {
        rc = fail(NSG_EDEVICE, "begin capture failed: %s", hipGetErrorString(e));
    }
    if (rc == NSG_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = fail(NSG_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    hipStreamDestroy(cs);
    if (rc != NSG_OK) {
        nsg_search_graph_destroy(g);
        return rc;
    }
    if (o.learned_stop) {
        g->stop_idx = idx;
        idx->stop_graphs.fetch_add(1);
    }
    *out = g;
    return NSG_OK;
}

extern "C" int nsg_search_graph_launch(nsg_search_graph *g, void *stream) {
    clear_error();
    if (!g || !g->exec) return fail(NSG_EINVAL, "graph is NULL");
    NSG_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return NSG_OK;
}

// ---------------------------------------------------------------------------
// autotuner: time launch configurations on the caller's batch
// ---------------------------------------------------------------------------
extern "C" int nsg_autotune(const nsg_index *idx, const float *queries, int64_t nq, int32_t k, int32_t L,
                            int32_t trials, nsg_search_opts *best, float *best_ms, void *stream) {
    clear_error();
    if (!idx || !queries || !best || !best_ms) return fail(NSG_EINVAL, "NULL pointer");
    if (nq < 1 || k < 1 || k > kMaxK || L < 1 || L > kMaxL || trials < 1) return fail(NSG_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    uint32_t *ids = nullptr;
    float *dist = nullptr;
    unsigned int *ctr = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        hipFree(ids);
        hipFree(dist);
        hipFree(ctr);
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
    };
    if (hipMalloc(&ids, sizeof(uint32_t) * nq * k) != hipSuccess || hipMalloc(&dist, sizeof(float) * nq * k) != hipSuccess ||
        hipMalloc(&ctr, 256) != hipSuccess || hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(NSG_ENOMEM, "autotune allocation failed");
    }
    int lpr0, cpl0;
    pick_layout(idx->row_chunks, 4, &lpr0, &cpl0);
    const int learned = best->learned_stop;   // the one input field of *best
    const int lprs[4] = {8, 16, 32, 64};
    const int hashes[3] = {1024, 2048, 4096};
    const int wpbs[3] = {1, 2, 4};
    float bestt = 1e30f;
    nsg_search_opts bo{};
    int rc = NSG_OK;
    for (int li = 0; li < 4 && rc == NSG_OK; ++li) {
        int c = (idx->row_chunks + lprs[li] - 1) / lprs[li];
        if (c > 4 || (lprs[li] / 2 >= idx->row_chunks && lprs[li] != lpr0))
            continue;   // too few lanes for the row, or half of them idle
        for (int hi = 0; hi < 3 && rc == NSG_OK; ++hi) {
            for (int wi = 0; wi < 3 && rc == NSG_OK; ++wi)
                for (int tr = 0; tr < 4 && rc == NSG_OK; ++tr) {
                    const int pers = tr & 1, lf = tr >> 1;
                    if (lf && nq > NSG_ORDER_MAX) continue;
                    nsg_search_opts o{};
                    o.lanes_per_row = lprs[li];
                    o.hash_slots = hashes[hi];
                    o.waves_per_block = wpbs[wi];
                    o.persistent = pers;
                    o.longest_first = lf;
                    o.learned_stop = learned;
                    o.counter = ctr;
                    int r = nsg_search_batched(idx, queries, nq, nullptr, nullptr, k, L, k, ids, dist, &o, stream);
                    if (r == NSG_EUNSUPPORTED) { clear_error(); continue; }
                    if (r != NSG_OK) { rc = r; break; }
                    hipEventRecord(e0, st);
                    for (int t = 0; t < trials && rc == NSG_OK; ++t)
                        rc = nsg_search_batched(idx, queries, nq, nullptr, nullptr, k, L, k, ids, dist, &o, stream);
                    hipEventRecord(e1, st);
                    if (hipEventSynchronize(e1) != hipSuccess) { rc = fail(NSG_EDEVICE, "autotune sync failed"); break; }
                    float ms = 0.0f;
                    hipEventElapsedTime(&ms, e0, e1);
                    ms /= (float)trials;
                    if (ms < bestt) { bestt = ms; bo = o; }
                }
        }
    }
    cleanup();
    if (rc != NSG_OK) return rc;
    bo.counter = nullptr;
    *best = bo;
    *best_ms = bestt;
    return NSG_OK;
}
