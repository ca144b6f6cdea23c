// Training kernels for the early-stop network (in -> h -> h -> 1, ReLU, MSE),
// FP32 on the vector ALUs.  Parameter layout: W1[h][in], b1[h], W2[h][h],
// b2[h], W3[h], b3.
//
// mlp_rows_kernel: one wave per sample, lane j = hidden unit j; forward pass,
//   then the backward deltas d2 = dL/dz2 and d1 = dL/dz1 of that sample.
// mlp_grad_kernel: one thread per parameter, summing its per-sample terms in
//   sample order (deterministic; no atomics).
#include "common.hpp"

#include <algorithm>
#include <cmath>

namespace nsg {

struct MlpRows {
    const float *P;   // params
    int in, h;
    const float *X, *y;
    int64_t B;
    float *yhat;
    float *A1, *A2, *D1, *D2, *E;   // [B][h] x4, [B]
};

__global__ void __launch_bounds__(256) mlp_rows_kernel(MlpRows p) {
    extern __shared__ float sm[];
    const int in = p.in, h = p.h;
    float *W1 = sm;                        // [h][in]
    float *W2 = W1 + (size_t)h * in;       // [h][h]
    float *b1 = W2 + (size_t)h * h;
    float *b2 = b1 + h;
    float *W3 = b2 + h;
    float *xb = W3 + h + 1;                // per wave: [in] input + [h] a1 + [h] d2
    const int np = h * in + h + h * h + h + h + 1;
    // stage parameters (W1, b1, W2, b2, W3, b3 in global order -> LDS layout above)
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        float v = p.P[i];
        int o = i;
        if (o < h * in) { W1[o] = v; continue; }
        o -= h * in;
        if (o < h) { b1[o] = v; continue; }
        o -= h;
        if (o < h * h) { W2[o] = v; continue; }
        o -= h * h;
        if (o < h) { b2[o] = v; continue; }
        o -= h;
        W3[o] = v;   // W3[0..h), then b3 at W3[h]
    }
    __syncthreads();
    const float b3 = W3[h];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wpb = blockDim.x >> 6;
    float *x = xb + (size_t)w * (in + 2 * h);
    float *a1s = x + in;
    float *d2s = a1s + h;
    for (int64_t b = (int64_t)blockIdx.x * wpb + w; b < p.B; b += (int64_t)gridDim.x * wpb) {
        for (int i = lane; i < in; i += 64) x[i] = p.X[b * in + i];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float z1 = 0.0f, a1 = 0.0f;
        if (lane < h) {
            float s = b1[lane];
            for (int i = 0; i < in; ++i) s = fmaf(W1[lane * in + i], x[i], s);
            z1 = s;
            a1 = s > 0.0f ? s : 0.0f;
            a1s[lane] = a1;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float z2 = 0.0f, a2 = 0.0f;
        if (lane < h) {
            float s = b2[lane];
            for (int k = 0; k < h; ++k) s = fmaf(W2[lane * h + k], a1s[k], s);
            z2 = s;
            a2 = s > 0.0f ? s : 0.0f;
        }
        float o = lane < h ? W3[lane] * a2 : 0.0f;
        for (int off = 32; off > 0; off >>= 1) o += __shfl_xor(o, off);
        o += b3;
        if (lane == 0 && p.yhat) p.yhat[b] = o;
        if (!p.y) continue;
        const float e = o - p.y[b];
        const float go = 2.0f * e / (float)p.B;
        float d2 = (lane < h && z2 > 0.0f) ? go * W3[lane] : 0.0f;
        if (lane < h) d2s[lane] = d2;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float d1 = 0.0f;
        if (lane < h && z1 > 0.0f) {
            float s = 0.0f;
            for (int j = 0; j < h; ++j) s = fmaf(W2[j * h + lane], d2s[j], s);
            d1 = s;
        }
        if (lane < h) {
            p.A1[b * h + lane] = a1;
            p.A2[b * h + lane] = a2;
            p.D1[b * h + lane] = d1;
            p.D2[b * h + lane] = d2;
        }
        if (lane == 0) p.E[b] = e;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// one thread per parameter; the extra thread np computes the loss
__global__ void mlp_grad_kernel(int in, int h, const float *X, int64_t B, const float *A1, const float *A2,
                                const float *D1, const float *D2, const float *E, float *grad, float *loss) {
    const int np = h * in + h + h * h + h + h + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t > np) return;
    const float inv = 2.0f / (float)B;
    float s = 0.0f;
    if (t == np) {
        if (loss) {
            for (int64_t b = 0; b < B; ++b) s = fmaf(E[b], E[b], s);
            *loss = s / (float)B;
        }
        return;
    }
    int o = t;
    if (o < h * in) {
        int k = o / in, i = o % in;
        for (int64_t b = 0; b < B; ++b) s = fmaf(D1[b * h + k], X[b * in + i], s);
    } else if ((o -= h * in) < h) {
        for (int64_t b = 0; b < B; ++b) s += D1[b * h + o];
    } else if ((o -= h) < h * h) {
        int j = o / h, k = o % h;
        for (int64_t b = 0; b < B; ++b) s = fmaf(D2[b * h + j], A1[b * h + k], s);
    } else if ((o -= h * h) < h) {
        for (int64_t b = 0; b < B; ++b) s += D2[b * h + o];
    } else if ((o -= h) < h) {
        for (int64_t b = 0; b < B; ++b) s = fmaf(E[b] * inv, A2[b * h + o], s);
    } else {
        for (int64_t b = 0; b < B; ++b) s = fmaf(E[b], inv, s);
    }
    grad[t] = s;
}

__global__ void adam_kernel(float *P, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float gi = g[i];
        float mi = b1 * m[i] + (1.0f - b1) * gi;
        float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__global__ void recall_hits_kernel(const uint32_t *found, int64_t nq, int G, int k, const uint32_t *truth,
                                   int kt, int32_t *hits) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nq * G) return;
    int64_t q = t / G;
    const uint32_t *f = found + t * k;
    const uint32_t *tr = truth + q * kt;
    int c = 0;
    for (int a = 0; a < k; ++a) {
        uint32_t id = f[a];
        if (id == NSG_SENT) continue;
        for (int b = 0; b < k; ++b)
            if (tr[b] == id) { ++c; break; }
    }
    hits[t] = c;
}

// per-column mean and 1/std, one thread per column, rows in order
// (deterministic), two passes of compensated FP32 sums (mean, then the mean
// squared deviation); std floored at 1e-12 of the mean magnitude and 1e-30.
// NaN rows (searches that ended before the feature hop) are skipped.
__global__ void column_stats_kernel(const float *X, int64_t B, int in, float *mean, float *inv_std) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= in) return;
    float s = 0.0f, cs = 0.0f;
    int64_t cnt = 0;
    for (int64_t b = 0; b < B; ++b) {
        const float v = X[b * in + j];
        if (isnan(v)) continue;
        neumaier_add(s, cs, v);
        ++cnt;
    }
    const float m = cnt ? (s + cs) / (float)cnt : 0.0f;
    float q = 0.0f, cq = 0.0f;
    for (int64_t b = 0; b < B; ++b) {
        const float v = X[b * in + j];
        if (isnan(v)) continue;
        const float dv = v - m;
        neumaier_add(q, cq, dv * dv);
    }
    const float var = cnt ? (q + cq) / (float)cnt : 0.0f;
    const float sd = sqrtf(var > 0.0f ? var : 0.0f);
    const float floor_ = fmaxf(1e-12f * fabsf(m), 1e-30f);
    mean[j] = m;
    inv_std[j] = 1.0f / (sd > floor_ ? sd : 1.0f);
}

static int mlp_rows(const float *params, int in, int h, const float *X, const float *y, int64_t B, float *yhat,
                    float *ws, hipStream_t st) {
    MlpRows r{};
    r.P = params;
    r.in = in;
    r.h = h;
    r.X = X;
    r.y = y;
    r.B = B;
    r.yhat = yhat;
    if (ws) {
        r.A1 = ws;
        r.A2 = ws + B * h;
        r.D1 = ws + 2 * B * h;
        r.D2 = ws + 3 * B * h;
        r.E = ws + 4 * B * h;
    }
    const int wpb = 4;
    size_t lds = sizeof(float) * ((size_t)h * in + (size_t)h * h + 3 * (size_t)h + 1 + (size_t)wpb * (in + 2 * h));
    if (lds > 160 * 1024) return fail(NSG_EUNSUPPORTED, "network too large for LDS");
    if (lds > 64 * 1024)
        NSG_HIP(hipFuncSetAttribute((const void *)mlp_rows_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int blocks = (int)std::min<int64_t>((B + wpb - 1) / wpb, 1024);
    hipLaunchKernelGGL(mlp_rows_kernel, dim3(std::max(blocks, 1)), dim3(64 * wpb), lds, st, r);
    NSG_HIP(hipGetLastError());
    return NSG_OK;
}

}  // namespace nsg

using namespace nsg;

extern "C" int nsg_mlp_forward(const float *params, int32_t in, int32_t h, const float *X, int64_t B, float *yhat,
                               void *stream) {
    clear_error();
    if (!params || !X || !yhat) return fail(NSG_EINVAL, "NULL pointer");
    if (in < 1 || in > 4096 || h < 1 || h > 64) return fail(NSG_EINVAL, "bad network shape");
    if (B < 0) return fail(NSG_EINVAL, "B < 0");
    if (B == 0) return NSG_OK;
    return mlp_rows(params, in, h, X, nullptr, B, yhat, nullptr, (hipStream_t)stream);
}

extern "C" int nsg_mlp_forward_backward(const float *params, int32_t in, int32_t h, const float *X, const float *y,
                                        int64_t B, float *yhat, float *grad, float *loss, void *stream) {
    clear_error();
    if (!params || !X || !y || !grad) return fail(NSG_EINVAL, "NULL pointer");
    if (in < 1 || in > 4096 || h < 1 || h > 64) return fail(NSG_EINVAL, "bad network shape");
    if (B < 1) return fail(NSG_EINVAL, "B must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    float *ws = nullptr;
    NSG_HIP(hipMallocAsync((void **)&ws, sizeof(float) * (4 * B * h + B), st));
    int rc = mlp_rows(params, in, h, X, y, B, yhat, ws, st);
    if (rc == NSG_OK) {
        const int np = h * in + h + h * h + h + h + 1;
        hipLaunchKernelGGL(mlp_grad_kernel, dim3((np + 1 + 255) / 256), dim3(256), 0, st, in, h, X, B, ws, ws + B * h,
                           ws + 2 * B * h, ws + 3 * B * h, ws + 4 * B * h, grad, loss);
        if (hipGetLastError() != hipSuccess) rc = fail(NSG_EDEVICE, "gradient kernel failed");
    }
    hipFreeAsync(ws, st);
    return rc;
}

extern "C" int nsg_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t P, int64_t t, float lr,
                            float beta1, float beta2, float eps, void *stream) {
    clear_error();
    if (!params || !grad || !m || !v) return fail(NSG_EINVAL, "NULL pointer");
    if (P < 1 || t < 1) return fail(NSG_EINVAL, "P and t must be >= 1");
    float c1 = 1.0f - (float)std::pow((double)beta1, (double)t);
    float c2 = 1.0f - (float)std::pow((double)beta2, (double)t);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)std::min<int64_t>((P + 255) / 256, 4096)), dim3(256), 0,
                       (hipStream_t)stream, params, grad, m, v, P, lr, beta1, beta2, eps, c1, c2);
    NSG_HIP(hipGetLastError());
    return NSG_OK;
}

extern "C" int nsg_recall_hits(const uint32_t *found, int64_t nq, int32_t G, int32_t k, const uint32_t *truth,
                               int32_t k_truth, int32_t *hits, void *stream) {
    clear_error();
    if (nq < 0 || G < 1 || k < 1 || k_truth < k) return fail(NSG_EINVAL, "bad shape");
    if (nq == 0) return NSG_OK;
    if (!found || !truth || !hits) return fail(NSG_EINVAL, "NULL pointer");
    int64_t t = nq * G;
    hipLaunchKernelGGL(recall_hits_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       found, nq, G, k, truth, k_truth, hits);
    NSG_HIP(hipGetLastError());
    return NSG_OK;
}

extern "C" int nsg_column_stats(const float *X, int64_t B, int32_t in, float *mean, float *inv_std, void *stream) {
    clear_error();
    if (!X || !mean || !inv_std) return fail(NSG_EINVAL, "NULL pointer");
    if (B < 1 || in < 1) return fail(NSG_EINVAL, "bad shape");
    hipLaunchKernelGGL(column_stats_kernel, dim3((in + 255) / 256), dim3(256), 0, (hipStream_t)stream, X, B, in,
                       mean, inv_std);
    NSG_HIP(hipGetLastError());
    return NSG_OK;
}
