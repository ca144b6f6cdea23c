/*
 * nsg.h — C ABI of libnsg.so, the MI355X (gfx950) implementation of search on
 * a Navigating Spreading-out Graph (Fu, Xiang, Wang, Cai, PVLDB; arXiv
 * 1707.00143).
 *
 * General conventions
 *   - Pointers are HIP device pointers unless a comment says "host".
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  Every call enqueues its work on `stream` and returns; results
 *     are valid once the stream has been synchronised.  Host-side argument
 *     checks happen before anything is enqueued: on any error nothing is
 *     written to caller memory.
 *   - Distances are SQUARED l2 distances in FP32 (the paper's delta is the l2
 *     distance, Sec. 2; squaring keeps its order).  Results are ordered by
 *     (distance, id) ascending.
 *   - Missing results (k larger than the final candidate pool, or than the
 *     number of points) are padded with id 0xFFFFFFFF and distance +inf.
 *   - Graphs are [n][R] uint32, row-major: each row is its valid prefix of
 *     neighbour ids followed by 0xFFFFFFFF sentinels (fixed out-degree
 *     storage for contiguous access, Sec. 4.1.3).
 *   - Return value: NSG_OK (0) or a negative nsg_status; nsg_last_error()
 *     gives a message for the calling host thread.  No C++ exception crosses
 *     this ABI.
 *   - Limits: n < 2^31, 1 <= d <= 1024, 1 <= R <= 128, 1 <= L <= 512,
 *     1 <= k <= 512 (nsg_knn_bruteforce: 1 <= k <= 160).  Arguments outside
 *     them return NSG_EINVAL before anything is enqueued.
 */
#ifndef NSG_H
#define NSG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nsg_index nsg_index;            /* opaque, owned by the library */

typedef enum {
    NSG_F32 = 0,   /* FP32 rows */
    NSG_BF16 = 1,  /* bfloat16 codes with per-dimension FP32 scales */
    NSG_F16 = 2,   /* IEEE binary16 codes with per-dimension FP32 scales */
    NSG_E4M3 = 3   /* OCP FP8 E4M3 codes with per-dimension FP32 scales */
} nsg_dtype;

typedef enum {
    NSG_OK = 0,
    NSG_EINVAL = -1,       /* bad argument */
    NSG_ENOMEM = -2,       /* device allocation failed */
    NSG_EDEVICE = -3,      /* a HIP call failed */
    NSG_ESTATE = -4,       /* call not valid in the current state */
    NSG_EUNSUPPORTED = -5  /* outside the compiled limits */
} nsg_status;

/* Message for the last failing call on this host thread (host pointer, valid
 * until the next call on the same thread). */
const char *nsg_last_error(void);

/* ------------------------------------------------------------------------ */
/* Index                                                                     */
/* ------------------------------------------------------------------------ */

/*
 * Make an index resident on the current device: the point set S (Sec. 2.1)
 * as base[n][d] FP32, its graph[n][R] and the navigating node (the fixed start
 * of every search, Sec. 3.4 step ii and Sec. 3.5).
 *   storage: row format the search gathers.  For reduced formats the scale of
 *            dimension j is s_j = max_i |base[i][j]| / M (M = 448 for E4M3,
 *            1 for BF16 / FP16; s_j = 1 for an all-zero column) unless
 *            `scales` (device, [d]) is given; codes are round-to-nearest-even
 *            of base/s_j with saturation.  The FP32 rows are kept as well: they
 *            re-rank the final pool exactly (only the prefix of the pool that
 *            can hold the FP32 top k, by a bound on the stored format's error
 *            computed here: the same result as re-ranking the whole pool).
 * The library copies base and graph into its own padded layout; the caller
 * may free its buffers after synchronising `stream`.  Graph entries must be
 * < n or the sentinel, nav < n (checked on the device; a violation returns
 * NSG_EINVAL).  *out receives the handle.
 */
int nsg_load_index(const float *base, int64_t n, int32_t d,
                   const uint32_t *graph, int32_t R, uint32_t nav_node,
                   nsg_dtype storage, const float *scales,
                   void *stream, nsg_index **out);

/* Release an index (NULL is a no-op).  Synchronises the device first. */
void nsg_free_index(nsg_index *idx);

/* Shape of a loaded index (host outputs; any may be NULL). */
int nsg_index_info(const nsg_index *idx, int64_t *n, int32_t *d, int32_t *R,
                   uint32_t *nav, int32_t *storage);

/* ------------------------------------------------------------------------ */
/* Search (Algorithm 1, Search-on-Graph, started at the navigating node)     */
/* ------------------------------------------------------------------------ */

/*
 * For each of nq queries[nq][d] (FP32, row-major) run Algorithm 1 from the
 * navigating node with candidate pool size L: repeatedly expand the nearest
 * unchecked pool entry, compute the distance of every not yet visited
 * neighbour, keep the L nearest by (distance, id); stop when no unchecked
 * entry remains; return the first k.  With reduced-precision storage the
 * walk uses the decoded rows s_j * code and the final pool is re-ranked with
 * exact FP32 distances before the first k are emitted.
 * Outputs out_ids[nq][k], out_dist[nq][k] (device, caller-allocated).
 * nq = 0 is a no-op.  Batches of 4096 queries or more run on a persistent
 * grid whose work counter the library allocates once per stream (the first
 * such call on a stream allocates it; later calls on that stream reuse it).
 * Batches of 8192 .. NSG_ORDER_MAX queries start the queries farthest from
 * the navigating node first (nsg_search_opts.longest_first; same results),
 * with an order buffer held per stream in the same way.
 */
int nsg_search(const nsg_index *idx, const float *queries, int64_t nq,
               int32_t k, int32_t L, uint32_t *out_ids, float *out_dist,
               void *stream);

/*
 * nsg_search for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * same arguments, result and kernels as nsg_search, and no hipMalloc /
 * hipFree or other allocating call.  Its scratch memory is the persistent
 * grid's work counter (batches of 4096 queries or more; one 32-bit word),
 * held in a 256-byte device array of the library that each GPU keeps until
 * the process ends; no input size changes what it must hold.  The counter is
 * cleared by a kernel at the start of every call.  All calls on one GPU
 * share that array: calls that overlap in time on one GPU (different
 * streams or threads) race and must not be issued.
 */
int nsg_search_noalloc(const nsg_index *idx, const float *queries, int64_t nq,
                       int32_t k, int32_t L, uint32_t *out_ids, float *out_dist,
                       void *stream);

/* Options of nsg_search_batched (host struct; zero-initialise, then set). */
typedef struct nsg_search_opts {
    int32_t persistent;      /* 1: persistent grid with an atomic work counter */
    int32_t waves_per_block; /* 0: default; else 1..4 (the kernels are built for <= 256 threads) */
    int32_t hash_slots;      /* visited-filter slots per query (power of 2); 0: default */
    int32_t blocks;          /* persistent grid size; 0: one wave per resident slot */
    int32_t learned_stop;    /* 1: use the loaded early-stop model (queries with L >= 16) */
    int32_t rerank;          /* 0: default (on for reduced storage), 1: on, -1: off */
    int64_t *hops;           /* device [nq] expansions per query, or NULL */
    int64_t *ndist;          /* device [nq] distance evaluations per query, or NULL */
    int32_t *budget;         /* device [nq] expansion budget chosen by the early stop (0: none), or NULL */
    float *features;         /* device [nq][NSG_STOP_FEATURES] early-stop features (see the
                                network below) after expansion `feature_hop`; NaN rows for
                                searches that ended earlier; or NULL */
    uint32_t *pool_ids;      /* device [nq][pool_stride] final pool ids, or NULL */
    float *pool_dist;        /* device [nq][pool_stride] final pool distances */
    int32_t pool_stride;
    int32_t feature_hop;     /* hop at which `features` are taken (0: 16; at most 65535; the model's hop when learned) */
    int64_t *nedges;         /* device [nq] valid neighbour entries read over all expansions, or NULL */
    int32_t lanes_per_row;   /* lanes that gather one row (8, 16, 32, 64); 0: default */
    uint32_t *counter;       /* device scratch word for the persistent work counter (reset by the
                                call); NULL: the library's counter for the calling stream, allocated
                                on the first persistent search on that stream and kept */
    int32_t max_hops;        /* > 0: every query stops after this many expansions; 0: no budget */
    int32_t *clamped;        /* device int32 counter (caller-initialised), or NULL: incremented
                                once for every query whose k[i] lies outside [0, out_stride] or
                                whose L[i] lies outside [1, L_scalar] (see below) */
    const uint32_t *init_ids; /* device [nq][init_n] node ids, or NULL: query i's initial pool is
                                the set of these nodes (each visited once, the L nearest kept)
                                instead of the navigating node -- random initialization (the
                                search of the NSG-Naive baseline, Sec. 4.1.2) or random starts
                                (Sec. 4.1.3); ids >= n are ignored */
    int32_t init_n;          /* 0 .. 512; 0: start at the navigating node */
    int32_t longest_first;   /* 1: start the batch's queries in order of decreasing squared distance
                                to the start node (the first distance of every walk), so that the
                                walks that tend to run longest start first and the batch does not
                                end on a few late long walks; results are unchanged.  Applies to
                                batches of 2 .. NSG_ORDER_MAX queries on one graph (larger batches,
                                and partitioned or randomly started searches, run in the given
                                order); 0: the given order */
    uint32_t *order_scratch; /* device scratch of NSG_ORDER_MAX * 8 bytes for longest_first, or
                                NULL: the calling stream's library buffer (allocated on first use,
                                kept; calls on one stream share it in stream order) */
} nsg_search_opts;

/* largest batch that longest_first orders */
#define NSG_ORDER_MAX 65536

/*
 * Batched search with a per-query k[i] and L[i] (device int32 arrays, NULL =
 * use k_scalar / L_scalar).  Outputs are [nq][out_stride] with
 * out_stride >= max k; entries past k[i] are left untouched.  `opts` may be
 * NULL.  Same algorithm and result definition as nsg_search: every query's
 * output equals its own nsg_search at (k[i], L[i]).
 * The per-query arrays live on the device, so they are not checked on the
 * host: a k[i] outside [0, out_stride] is clamped into it (k[i] = 0 writes
 * nothing) and an L[i] outside [1, L_scalar] is clamped into that range; each
 * such query is counted in opts->clamped when it is given.  The persistent
 * grid (opts->persistent) with opts->counter NULL uses a work counter the
 * library allocates once per stream (the first call on a stream allocates).
 */
int nsg_search_batched(const nsg_index *idx, const float *queries, int64_t nq,
                       const int32_t *k, const int32_t *L,
                       int32_t k_scalar, int32_t L_scalar, int32_t out_stride,
                       uint32_t *out_ids, float *out_dist,
                       const nsg_search_opts *opts, void *stream);

/* ------------------------------------------------------------------------ */
/* Partitioned index (one NSG per subset; Sec. 4.2 "Search On DEEP100M",     */
/* Sec. 4.3 "Experiments On Taobao Data")                                    */
/* ------------------------------------------------------------------------ */

typedef struct nsg_shards nsg_shards;   /* opaque, owned by the library */

/*
 * Make a partitioned index resident: the point set base[n][d] (FP32) split
 * into S subsets of consecutive rows, offsets (host, [S + 1]) with
 * offsets[0] = 0 < offsets[1] < ... < offsets[S] = n, 1 <= S <= 64.  Each
 * subset has its own NSG: graph[n][R] (device) row i holds the out-neighbours
 * of point i as ids LOCAL to its subset (0 .. offsets[s+1] - offsets[s] - 1),
 * sentinel-padded; navs (host, [S]) holds each subset's navigating node as a
 * local id.  storage / scales as in nsg_load_index (scales computed over the
 * whole set).  The library keeps one copy of the rows and a graph of global
 * ids; an entry that is neither a local id of its subset nor the sentinel,
 * or a navigating node outside its subset, returns NSG_EINVAL.  Synchronous.
 */
int nsg_load_shards(const float *base, int64_t n, int32_t d, const int64_t *offsets,
                    int32_t S, const uint32_t *graph, int32_t R, const uint32_t *navs,
                    nsg_dtype storage, const float *scales, void *stream,
                    nsg_shards **out);

/* Release a partitioned index (NULL is a no-op).  Synchronises the device. */
void nsg_free_shards(nsg_shards *sh);

/* Number of subsets and the underlying index (rows, global-id graph) of a
 * partitioned index (host outputs; either may be NULL). */
int nsg_shards_info(const nsg_shards *sh, int32_t *S, nsg_index **index);

/*
 * Search every query in every subset and merge: Algorithm 1 from each
 * subset's navigating node with pool size L (one wavefront per (query,
 * subset) pair, the kernels of nsg_search, re-rank included for reduced
 * storage), each giving its top k by (distance, id); the result is the k
 * smallest (distance, id) keys of the union of the S lists (global ids).
 * out_ids / out_dist [nq][k] (device); padding as in nsg_search.
 * S * k <= 8192.  The S per-subset lists (nq * S * k * 8 bytes) are
 * allocated and freed on `stream` (stream-ordered allocations).
 */
int nsg_search_shards(const nsg_shards *sh, const float *queries, int64_t nq,
                      int32_t k, int32_t L, uint32_t *out_ids, float *out_dist,
                      void *stream);

/* ------------------------------------------------------------------------ */
/* Batches as HIP graphs, and the launch autotuner                           */
/* ------------------------------------------------------------------------ */

typedef struct nsg_search_graph nsg_search_graph;   /* opaque, owned by the library */

/*
 * Capture one nsg_search_batched call (same arguments) into a HIP graph and
 * instantiate it.  The buffers are bound at capture: refill `queries` (and
 * k / L) in place, then nsg_search_graph_launch replays the whole batch with
 * one launch.  With opts->persistent the graph owns its work counter.  A
 * graph captured with opts->learned_stop holds the index's early-stop model
 * and calibration as they were at capture: while such a graph exists,
 * nsg_load_stop_model and nsg_set_stop_mode on that index return NSG_ESTATE.
 */
int nsg_search_graph_create(const nsg_index *idx, const float *queries, int64_t nq,
                            const int32_t *k, const int32_t *L, int32_t k_scalar,
                            int32_t L_scalar, int32_t out_stride, uint32_t *out_ids,
                            float *out_dist, const nsg_search_opts *opts,
                            nsg_search_graph **out);
int nsg_search_graph_launch(nsg_search_graph *g, void *stream);
void nsg_search_graph_destroy(nsg_search_graph *g);   /* NULL-safe; synchronises */

/*
 * Time candidate launch configurations of nsg_search_batched (lanes per row,
 * waves per block, visited-filter size, persistent grid, longest_first for
 * batches of at most NSG_ORDER_MAX queries) on the given batch
 * (scalar k, L) and return the fastest in *best (host; other fields zeroed)
 * with its mean time per call in *best_ms (host).  On input, best->learned_stop
 * is honoured (every candidate is timed with it; the other input fields are
 * ignored).  `trials` timed calls per candidate after one warm-up.
 * Synchronous; writes no caller memory except *best and *best_ms.
 */
int nsg_autotune(const nsg_index *idx, const float *queries, int64_t nq, int32_t k,
                 int32_t L, int32_t trials, nsg_search_opts *best, float *best_ms,
                 void *stream);

/* ------------------------------------------------------------------------ */
/* Exact K nearest neighbours (serial scan, Sec. 4.1.2 item 1; K-NNS, Sec. 2.1) */
/* ------------------------------------------------------------------------ */

/*
 * Exact k nearest base rows of every query by squared l2 distance, ordered by
 * (distance, id).  Candidates come from FP32 matrix-core tiles
 * (|x - mu|^2 - 2 (q - mu).(x - mu) with mu the base mean: the squared
 * distance minus a per-query constant), over-fetched, then re-ranked with exact FP32
 * differences (sum of (q_j - x_j)^2).  exclude_self != 0: queries are the base
 * rows themselves and query i never returns row i (kNN graph).  base[n][d],
 * queries[nq][d] FP32; out_ids / out_dist [nq][k].  1 <= k <= 160, 1 <= d <=
 * 65536.  Scratch memory is allocated and freed on `stream` (stream-ordered
 * allocations): candidate buffers of 512 keys (8 bytes each) per query and
 * base split while they total at most 8 GiB (fewer keys per query above
 * that), plus O(n + nq * k) words.  Returns NSG_ENOMEM if an allocation fails.
 */
int nsg_knn_bruteforce(const float *base, int64_t n, const float *queries,
                       int64_t nq, int32_t d, int32_t k, int32_t exclude_self,
                       uint32_t *out_ids, float *out_dist, void *stream);

/* ------------------------------------------------------------------------ */
/* Index construction on the GPU (Algorithm 2, NSGbuild(G, l, m))            */
/* ------------------------------------------------------------------------ */

/*
 * Build an NSG from base[n][d] and a kNN graph knn[n][K] (Algorithm 2):
 * centroid; navigating node = Algorithm 1 on the kNN graph from `rand_start`
 * with the centroid as query; for every node, search-collect on the kNN
 * graph from the navigating node (every visited node plus the K kNN
 * neighbours, nearest C kept) and MRNG edge selection with at most m = R
 * edges; then DFS-tree connectivity repair from the navigating node.
 * graph_out [n][R] (device), *nav_out (host).  *repair_edges (host, may be
 * NULL) receives the number of edges the repair added.  Synchronous.
 * With the environment variable NSG_LOG set (non-empty, not "0") it writes
 * one progress line per phase to stderr.
 */
int nsg_build(const float *base, int64_t n, int32_t d, const uint32_t *knn,
              int32_t K, int32_t Lb, int32_t C, int32_t R, uint32_t rand_start,
              uint32_t *graph_out, uint32_t *nav_out, int64_t *repair_edges,
              void *stream);

/*
 * Approximate kNN graph by an inverted file (step (i) of the build, which the
 * paper leaves replaceable: nn-descent on the CPU, Faiss on the GPU for
 * DEEP100M; Sec. 3.5, indexing complexity).  Cells are the nlist pivot
 * points base[pivots[c]] (pivots: device, nlist ids < n, chosen by the
 * caller, e.g. a seeded random sample); a point's probes are its nprobe
 * nearest pivots by (FP32 squared distance, c) and its cell the nearest.
 * Row i of the output: the K points nearest to i by (FP32 squared distance,
 * id) among the points other than i whose cell is one of i's probes
 * (sentinel / +inf padded when there are fewer).  nprobe = nlist gives the
 * exact kNN graph.  out_ids [n][K], out_dist [n][K] (device).  Limits:
 * 1 <= nlist <= n, 1 <= nprobe <= min(nlist, 160), 1 <= K <= 159,
 * n * nprobe < 2^31.  Temporary device memory ≈ n (8 K + 24 nprobe + 24)
 * bytes plus, twice (consecutive cells run on two streams), the largest
 * cell's member and probing-point rows and the brute-force scratch of the
 * largest cell (about 4.5 KiB per probing point, for at least 65,536
 * points), all allocated before the first cell.  Synchronous.
 */
int nsg_knn_ivf(const float *base, int64_t n, int32_t d, const uint32_t *pivots,
                int32_t nlist, int32_t nprobe, int32_t K, uint32_t *out_ids,
                float *out_dist, void *stream);

/*
 * NSG-Naive, the baseline of Sec. 4.1.2: the MRNG edge selection of Algorithm
 * 2 applied to each node's own kNN list only (candidates = the K neighbours
 * of knn[n][K], sorted by (distance, id)), at most R edges per node; no
 * navigating node, no search-collect, no connectivity repair.  Searches on it
 * start from random nodes (nsg_search_opts.init_ids).  graph_out [n][R]
 * (device, sentinel padded).  Synchronous.
 */
int nsg_build_naive(const float *base, int64_t n, int32_t d, const uint32_t *knn,
                    int32_t K, int32_t R, uint32_t *graph_out, void *stream);

/* ------------------------------------------------------------------------ */
/* Learned early termination (an extension; not in the paper)                */
/* ------------------------------------------------------------------------ */

/*
 * Two network forms.  In both, the inputs are z-scored with mean[in] /
 * inv_std[in]; two ReLU hidden layers of h <= 64 units; one linear output
 * y = predicted log2 of the expansion budget, taken from the search state
 * after `hop` expansions.  d_r below is the distance of pool rank
 * min(r, size - 1) (FP32 squared distance of the search format), d_s the
 * distance to the start node.
 *
 * NSG_STOP_SCALAR (in = NSG_STOP_FEATURES = 15 features, FP32 inference):
 *   0 ln(1 + d_0)        1 d_0 / d_9 (1 if d_9 = 0)
 *   2 ln(1 + d_s)        3 ln(1 + d_0) - ln(1 + d_s)
 *   4..13 ln(1 + d_r) - ln(1 + d_0) for r = 1, 2, 4, 9, 14, 19, 29, 39, 59, 83
 *   14 valid neighbour entries read per expansion so far
 * NSG_STOP_QUERY (in = d + 3, FP16 inference): the query's d values, then
 *   ln(1 + d_0), d_0 / d_9 (1 if d_9 = 0) and the expansion count.  The
 *   z-scored inputs (computed in FP32), the weights and the hidden
 *   activations are rounded to FP16 (nearest even); products accumulate in
 *   FP32; biases stay FP32.
 *
 * The query then stops after B = max(hop, smallest grid value >= c * 2^y)
 * expansions (the largest grid value if none is), or earlier when no
 * unchecked entry remains: its result is the plain search's after
 * min(B, its own expansion count) expansions, with the same L.  A
 * non-finite y sets no budget.  The decision is fused into the search loop:
 * after expansion `hop` the wavefront forms the inputs from its pool and its
 * query, evaluates the network and continues with the budget.
 * blob (host) holds FP32 in both forms: mean[in], inv_std[in], W1[h][in],
 * b1[h], W2[h][h], b2[h], W3[h], b3, then `grid_n` FP32 grid values
 * (expansion counts in [1, 2^20]) ascending.  Errors: NSG_EINVAL for a
 * wrong kind, input width or blob size, or a grid out of range.
 */
#define NSG_STOP_FEATURES 15
#define NSG_STOP_SCALAR 0
#define NSG_STOP_QUERY 1
int nsg_load_stop_model(nsg_index *idx, const void *blob, size_t bytes, int32_t kind,
                        int32_t in, int32_t h, int32_t hop, int32_t grid_n);

/*
 * Decision checkpoints of the loaded model (host array of n ints, 1 <= n <= 4,
 * strictly ascending, each in [1, 65535]; hops[0] becomes the model's decision
 * hop).  After expansion hops[j] a query still allowed to run past it forms
 * the inputs again, evaluates the network and replaces its budget by
 * max(hops[j], the grid pick); the next checkpoint is taken only if the new
 * budget lets the search pass it.  With the query form the expansion count
 * input then differs between checkpoints.  Loading a model resets the list
 * to its hop.  NSG_ESTATE without a model or while a search graph captured
 * with the early stop exists.
 */
int nsg_set_stop_checkpoints(nsg_index *idx, const int32_t *hops, int32_t n);

/* Enable (1) or disable (0) the early stop and set its calibration c > 0.
 * Both this call and nsg_load_stop_model return NSG_ESTATE while a search
 * graph captured with the early stop exists on the index (see above). */
int nsg_set_stop_mode(nsg_index *idx, int32_t enabled, float calib_c);

/*
 * Training kernels (FP32, vector ALU).  params layout: W1[h][in], b1[h],
 * W2[h][h], b2[h], W3[h], b3 (P = h*in + h + h*h + h + h + 1 floats).
 * X[B][in], y[B] device FP32.  Writes yhat[B] (may be NULL), grad[P] and
 * *loss (device scalar, may be NULL) for loss = mean (yhat - y)^2.
 */
int nsg_mlp_forward_backward(const float *params, int32_t in, int32_t h,
                             const float *X, const float *y, int64_t B,
                             float *yhat, float *grad, float *loss, void *stream);

/* Adam step t (1-based) over P parameters: params, m, v updated in place. */
int nsg_mlp_adam(float *params, const float *grad, float *m, float *v,
                 int64_t P, int64_t t, float lr, float beta1, float beta2,
                 float eps, void *stream);

/* Forward only (inference), FP32: yhat[B]. */
int nsg_mlp_forward(const float *params, int32_t in, int32_t h,
                    const float *X, int64_t B, float *yhat, void *stream);

/*
 * Per-column z-score statistics of X[B][in] (device): mean[in] and
 * inv_std[in] = 1 / standard deviation (1 for a constant column).  Rows whose
 * entry is NaN are skipped for that column.
 */
int nsg_column_stats(const float *X, int64_t B, int32_t in, float *mean,
                     float *inv_std, void *stream);

/*
 * Labels for training: for each query i and grid column j, the number of
 * ids of found[i][j][0..k) that appear in truth[i][0..k) (found is
 * [nq][G][k], truth [nq][k_truth] with k_truth >= k).  hits[nq][G] int32.
 */
int nsg_recall_hits(const uint32_t *found, int64_t nq, int32_t G, int32_t k,
                    const uint32_t *truth, int32_t k_truth, int32_t *hits,
                    void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NSG_H */
