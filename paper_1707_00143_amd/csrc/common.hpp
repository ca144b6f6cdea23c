// Internal declarations shared by the sources of libnsg.so (GPU library only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <atomic>

#include "../../include/nsg.h"

#define NSG_SENT 0xFFFFFFFFu

namespace nsg {

constexpr int kMaxL = 512;
constexpr int kMaxR = 128;
constexpr int kMaxK = 512;
constexpr int kMaxD = 1024;
constexpr int kWave = 64;
// zero bytes every row table carries past its last row: the widest gather
// layout (64 lanes x 4 chunks of 16 bytes) may read that far
constexpr int kRowTailBytes = 64 * 4 * 16;

// ---- error reporting (thread-local message) -------------------------------
int fail(int code, const char *fmt, ...);
void clear_error();

#define NSG_HIP(call)                                                          \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess)                                                  \
            return ::nsg::fail(NSG_EDEVICE, "%s failed: %s (%s:%d)", #call,     \
                               hipGetErrorString(e_), __FILE__, __LINE__);     \
    } while (0)

// ---- the index object ------------------------------------------------------
// Early-stop features per query, taken after the decision hop (stop_feature
// in search_impl.hpp).
constexpr int kStopFeatures = 15;

struct StopModel {
    float *blob = nullptr;     // device, the kernel layout of the network form (see stop_decide)
    int kind = NSG_STOP_SCALAR;
    int in = 0, h = 0, hop = 0, grid_n = 0;
    int ncp = 1;                 // decision checkpoints (cps[0] = hop)
    int cps[4] = {0, 0, 0, 0};
    int enabled = 0;
    float calib_c = 1.0f;
};

}  // namespace nsg

struct nsg_index {
    int64_t n = 0;
    int32_t d = 0;
    int32_t R = 0, R_pad = 0;
    uint32_t nav = 0;
    int32_t storage = NSG_F32;
    int32_t row_chunks = 0;      // 16-byte chunks per row of the search format
    int32_t row_chunks_f32 = 0;  // 16-byte chunks per FP32 row
    float *base_f32 = nullptr;   // [n][row_chunks_f32 * 4]
    void *base_lp = nullptr;     // [n][row_chunks * 16 bytes] for reduced formats
    float *scales = nullptr;     // [row_chunks_f32 * 4]
    uint32_t *graph = nullptr;   // [n][R_pad]
    // bound E on | ||q - x_i|| - (walk distance of row i)^(1/2) | from the
    // stored format (max_i ||xhat_i - x_i|| plus an absolute term for the
    // decode's rounding), used to re-rank only the prefix of the pool that can
    // hold the FP32 top k; < 0: unknown (the whole pool is re-ranked)
    float rr_eta = -1.0f;
    int device = 0;
    nsg::StopModel stop;
    // live search graphs captured with the early stop (they hold the model's
    // device pointer and calibration as captured)
    mutable std::atomic<int> stop_graphs{0};
};

namespace nsg {

// elements per 16-byte chunk of a storage format
inline int elems_per_chunk(int storage) {
    return storage == NSG_F32 ? 4 : (storage == NSG_E4M3 ? 16 : 8);
}

struct SearchArgs {
    const nsg_index *idx;
    const float *queries;
    int64_t nq;
    const int32_t *k_arr;
    const int32_t *L_arr;
    int32_t k_scalar, L_scalar, out_stride;
    uint32_t *out_ids;
    float *out_dist;
    int32_t L_cap;          // pool capacity in LDS
    int32_t hash_bits;
    int32_t waves_per_block;
    int32_t persistent;
    int32_t blocks;
    int32_t rerank;
    int32_t learned;
    int64_t *hops;
    int64_t *ndist;
    int64_t *nedges;          // valid neighbour entries read, summed over expansions
    int32_t feature_hop;      // decision / trace hop (0: 16)
    int32_t lanes_per_row;    // 0: default layout
    unsigned int *counter;    // persistent work counter (NULL: the calling stream's library counter)
    int longest_first;        // start the queries in order of decreasing distance to the start node
    uint32_t *order_scratch;  // NSG_ORDER_MAX * 8 bytes for that order (NULL: the stream's library buffer)
    int32_t *clamped;         // queries whose k[i] / L[i] were clamped (device counter), or NULL
    int32_t *budget;
    int32_t max_hops;
    float *features;
    uint32_t *pool_ids;
    float *pool_dist;
    int32_t pool_stride;
    // search a caller-supplied graph instead of idx->graph (index build)
    const uint32_t *graph_override;
    int32_t R_override, Rpad_override;
    uint32_t start_override;  // NSG_SENT: use idx->nav
    // per-query start node (index build: NULL)
    const uint32_t *start_arr;
    // record visited nodes (index build): [nq][vis_cap] ids and distances, counts
    uint32_t *vis_ids;
    float *vis_dist;
    int32_t *vis_cnt;
    int32_t vis_cap;
    int64_t self_offset;      // >= 0: query i is base row self_offset + i (index build), else -1
    // partitioned index: nq counts (query, shard) searches, search i is query
    // i / shards in shard i % shards from shard_starts[i % shards] (device)
    int32_t shards;           // 0 or 1: one graph
    const uint32_t *shard_starts;
    const uint32_t *init_ids; // [nq][init_n] initial pool node sets (device), or NULL
    int32_t init_n;
    uint32_t *trace_ids;      // [nq][trace_cap] expanded nodes in order (index build), or NULL
    int32_t trace_cap;
    hipStream_t stream;
};

int launch_search(const SearchArgs &a);

// FP32 mean of the rows of x[n][d] (compensated FP32 sums); part holds
// mean_blocks(n) * d partial sums
int mean_blocks(int64_t n);
int launch_mean(const float *x, int64_t n, int d, float *mu, float2 *part, hipStream_t st);

// compensated (Neumaier) summation step: s + c tracks the exact running sum
__device__ inline void neumaier_add(float &s, float &c, float v) {
    const float t = s + v;
    c += fabsf(s) >= fabsf(v) ? (s - t) + v : (v - t) + s;
    s = t;
}

// visited-filter size (log2 slots) used for a pool of L entries
int default_hash_bits(int L);

// choose lanes-per-row and chunks-per-lane for a row of `chunks` chunks
void pick_layout(int chunks, int max_cpl, int *lpr, int *cpl);

}  // namespace nsg
