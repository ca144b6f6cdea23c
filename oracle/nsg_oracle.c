/*
 * CPU oracle for NSG search (Fu, Xiang, Wang, Cai: "Fast Approximate Nearest
 * Neighbor Search With The Navigating Spreading-out Graph", PVLDB).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header, table or helper with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math), so
 * every FP32 subtraction, product and sum is rounded on its own, in the order
 * written here.
 *
 * Conventions used throughout (the paper's delta is the l2 distance, Sec. 2):
 *   - distances are SQUARED l2; squaring keeps the order of delta.
 *   - the FP32 squared distance sums (q_j - x_j)^2 sequentially for
 *     j = 0..d-1, no fused multiply-add.
 *   - keys are ordered lexicographically by (distance, id); this extends the
 *     paper's index tie-break for isosceles triangles (Sec. 3.3, after the MRNG
 *     definition) to every ordering the method needs.
 *   - a graph is [n][R] uint32, a row is its valid prefix followed by
 *     0xFFFFFFFF sentinels (fixed out-degree storage, Sec. 4.1.3 item 3).
 *
 * Where the paper is silent or garbled, the reading taken is stated at the
 * function that needs it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define SENT 0xFFFFFFFFu

/* ------------------------------------------------------------------------ */
/* Distances                                                                 */
/* ------------------------------------------------------------------------ */

/* Squared l2 distance in FP32, summed in index order (Sec. 2 delta(p,q)). */
float oracle_l2sq_f32(const float *a, const float *b, int d)
{
    float s = 0.0f;
    for (int j = 0; j < d; ++j) {
        float t = a[j] - b[j];
        float p = t * t;
        s = s + p;
    }
    return s;
}

/* Squared l2 distance evaluated in FP64 from the FP32 inputs. */
double oracle_l2sq_f64(const float *a, const float *b, int d)
{
    double s = 0.0;
    for (int j = 0; j < d; ++j) {
        double t = (double)a[j] - (double)b[j];
        s += t * t;
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Exact K nearest neighbours (K-NNS definition, Sec. 2.1; serial scan,      */
/* Sec. 4.1.2 item 1).                                                       */
/* ------------------------------------------------------------------------ */

typedef struct { double key; uint32_t id; } dkey_t;

static int dkey_less(double ka, uint32_t ia, double kb, uint32_t ib)
{
    return ka < kb || (ka == kb && ia < ib);
}

/*
 * For every query, order all n base points by (key, id) and return the first
 * k.  key is the FP64 squared distance when prec == 64 and the FP32 one when
 * prec == 32.  When exclude_self != 0 the queries are the base rows
 * themselves and query i never returns base row i (used for the kNN graph).
 * Returns 0, or -1 on bad arguments.  Output: ids[nq][k], dists[nq][k]
 * (FP64 value of the key that ordered them); slots beyond the number of
 * candidates hold (SENT, +inf).
 */
int oracle_knn(const float *base, int64_t n, int d, const float *queries,
               int64_t nq, int k, int prec, int exclude_self,
               uint32_t *ids, double *dists)
{
    if (n < 0 || nq < 0 || d < 1 || k < 1 || (prec != 32 && prec != 64))
        return -1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t qi = 0; qi < nq; ++qi) {
        dkey_t *top = (dkey_t *)malloc(sizeof(dkey_t) * (size_t)k);
        if (!top) { bad = 1; continue; }
        int cnt = 0;
        const float *q = queries + qi * (int64_t)d;
        for (int64_t i = 0; i < n; ++i) {
            if (exclude_self && i == qi) continue;
            const float *x = base + i * (int64_t)d;
            double key = prec == 64 ? oracle_l2sq_f64(q, x, d)
                                    : (double)oracle_l2sq_f32(q, x, d);
            uint32_t id = (uint32_t)i;
            if (cnt == k && !dkey_less(key, id, top[k - 1].key, top[k - 1].id))
                continue;
            /* insertion into the sorted top list */
            int pos = cnt < k ? cnt : k - 1;
            while (pos > 0 && dkey_less(key, id, top[pos - 1].key, top[pos - 1].id)) {
                top[pos] = top[pos - 1];
                --pos;
            }
            top[pos].key = key;
            top[pos].id = id;
            if (cnt < k) ++cnt;
        }
        for (int j = 0; j < k; ++j) {
            ids[qi * k + j] = j < cnt ? top[j].id : SENT;
            dists[qi * k + j] = j < cnt ? top[j].key : INFINITY;
        }
        free(top);
    }
    return bad ? -2 : 0;
}

/* ------------------------------------------------------------------------ */
/* Approximate kNN graph by an inverted file: step (i) of the build, which    */
/* the paper leaves replaceable (nn-descent on CPU; Faiss on GPU for          */
/* DEEP100M, Sec. 3.5 indexing complexity).                                  */
/* ------------------------------------------------------------------------ */

/*
 * Cells: the nlist pivot points base[pivots[c]].  The probes of point i are
 * its nprobe nearest pivots, ordered by (FP32 squared distance, c); its cell
 * is its first probe.  Row i of the graph: the K points nearest to i by
 * (FP32 squared distance, id) among the points other than i whose cell is
 * one of i's probes.  Output ids[n][K] (SENT padded), dists[n][K] (FP32 keys,
 * +inf padded), and, if probes_out is given, the probes [n][nprobe].
 * Returns 0, -1 on bad arguments, -2 on allocation failure.
 */
int oracle_knn_ivf(const float *base, int64_t n, int d, const uint32_t *pivots, int nlist, int nprobe,
                   int K, uint32_t *ids, float *dists, uint32_t *probes_out)
{
    if (n < 1 || d < 1 || nlist < 1 || nprobe < 1 || nprobe > nlist || nprobe > 160 || K < 1) return -1;
    for (int c = 0; c < nlist; ++c)
        if ((int64_t)pivots[c] >= n) return -1;
    uint32_t *probe = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n * nprobe);
    int64_t *start = (int64_t *)calloc((size_t)nlist + 1, sizeof(int64_t));
    uint32_t *member = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    if (!probe || !start || !member) { free(probe); free(start); free(member); return -2; }
    int bad = 0;
    /* probes: the nprobe nearest pivots of every point */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const float *x = base + i * (int64_t)d;
        dkey_t top[160];
        int cnt = 0;
        for (int c = 0; c < nlist; ++c) {
            double key = (double)oracle_l2sq_f32(x, base + (int64_t)pivots[c] * d, d);
            uint32_t id = (uint32_t)c;
            if (cnt == nprobe && !dkey_less(key, id, top[nprobe - 1].key, top[nprobe - 1].id)) continue;
            int pos = cnt < nprobe ? cnt : nprobe - 1;
            while (pos > 0 && dkey_less(key, id, top[pos - 1].key, top[pos - 1].id)) {
                top[pos] = top[pos - 1];
                --pos;
            }
            top[pos].key = key;
            top[pos].id = id;
            if (cnt < nprobe) ++cnt;
        }
        for (int j = 0; j < nprobe; ++j) probe[i * nprobe + j] = top[j].id;
    }
    /* members of every cell, in id order */
    for (int64_t i = 0; i < n; ++i) start[probe[i * nprobe] + 1]++;
    for (int c = 0; c < nlist; ++c) start[c + 1] += start[c];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)nlist);
        if (!fill) bad = 2;
        else {
            for (int c = 0; c < nlist; ++c) fill[c] = start[c];
            for (int64_t i = 0; i < n; ++i) member[fill[probe[i * nprobe]]++] = (uint32_t)i;
            free(fill);
        }
    }
    /* every point: exact K nearest among the members of its probed cells */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        if (bad) continue;
        dkey_t *top = (dkey_t *)malloc(sizeof(dkey_t) * (size_t)K);
        if (!top) { bad = 2; continue; }
        int cnt = 0;
        const float *x = base + i * (int64_t)d;
        for (int j = 0; j < nprobe; ++j) {
            uint32_t c = probe[i * nprobe + j];
            for (int64_t t = start[c]; t < start[c + 1]; ++t) {
                uint32_t id = member[t];
                if ((int64_t)id == i) continue;
                double key = (double)oracle_l2sq_f32(x, base + (int64_t)id * d, d);
                if (cnt == K && !dkey_less(key, id, top[K - 1].key, top[K - 1].id)) continue;
                int pos = cnt < K ? cnt : K - 1;
                while (pos > 0 && dkey_less(key, id, top[pos - 1].key, top[pos - 1].id)) {
                    top[pos] = top[pos - 1];
                    --pos;
                }
                top[pos].key = key;
                top[pos].id = id;
                if (cnt < K) ++cnt;
            }
        }
        for (int j = 0; j < K; ++j) {
            ids[i * K + j] = j < cnt ? top[j].id : SENT;
            dists[i * K + j] = j < cnt ? (float)top[j].key : INFINITY;
        }
        free(top);
    }
    if (probes_out && !bad) memcpy(probes_out, probe, sizeof(uint32_t) * (size_t)n * nprobe);
    free(probe); free(start); free(member);
    return bad ? -2 : 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1, Search-on-Graph(G, p, q, l)                                  */
/* ------------------------------------------------------------------------ */

typedef struct { float dist; uint32_t id; int checked; } pent_t;

static int pent_cmp(const void *a, const void *b)
{
    const pent_t *x = (const pent_t *)a, *y = (const pent_t *)b;
    if (x->dist < y->dist) return -1;
    if (x->dist > y->dist) return 1;
    if (x->id < y->id) return -1;
    if (x->id > y->id) return 1;
    return 0;
}

/* Per-thread workspace: a visited stamp per base row, the pool and a list of
 * every visited node. */
typedef struct {
    int64_t n;
    uint32_t *stamp;
    uint32_t cur;
    pent_t *pool;       /* capacity L + R */
    int pool_cap;
    pent_t *vis;        /* every node whose distance was computed */
    int64_t vis_cnt, vis_cap;
} ws_t;

static int ws_init(ws_t *w, int64_t n, int cap)
{
    memset(w, 0, sizeof(*w));
    w->n = n;
    w->stamp = (uint32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
    w->pool = (pent_t *)malloc(sizeof(pent_t) * (size_t)cap);
    w->pool_cap = cap;
    w->vis_cap = 1024;
    w->vis = (pent_t *)malloc(sizeof(pent_t) * (size_t)w->vis_cap);
    return (w->stamp && w->pool && w->vis) ? 0 : -1;
}

static void ws_free(ws_t *w)
{
    free(w->stamp); free(w->pool); free(w->vis);
    memset(w, 0, sizeof(*w));
}

static int ws_pool_reserve(ws_t *w, int cap)
{
    if (cap <= w->pool_cap) return 0;
    pent_t *p = (pent_t *)realloc(w->pool, sizeof(pent_t) * (size_t)cap);
    if (!p) return -1;
    w->pool = p; w->pool_cap = cap;
    return 0;
}

static int ws_vis_push(ws_t *w, float dist, uint32_t id)
{
    if (w->vis_cnt == w->vis_cap) {
        int64_t nc = w->vis_cap * 2;
        pent_t *p = (pent_t *)realloc(w->vis, sizeof(pent_t) * (size_t)nc);
        if (!p) return -1;
        w->vis = p; w->vis_cap = nc;
    }
    w->vis[w->vis_cnt].dist = dist;
    w->vis[w->vis_cnt].id = id;
    w->vis[w->vis_cnt].checked = 0;
    w->vis_cnt++;
    return 0;
}

/*
 * One search (Algorithm 1), started at `start` (Sec. 3.5: always the
 * navigating node for search on an NSG).
 *
 * Steps, in the paper's order:
 *   pool <- {start} (unchecked); visited <- {start}
 *   loop: i <- first unchecked entry of the pool; stop when there is none
 *         mark it checked
 *         for every neighbour u of pool[i] in row order, up to the sentinel:
 *             if u is not visited: visit it (compute its distance), add to S
 *         sort S ascending by (distance, id), keep its first L entries
 *   return the first k entries of the pool
 *
 * Readings where the printed algorithm is silent or ambiguous:
 *   - termination: the printed loop condition would never end when the pool
 *     holds fewer than l entries and all are checked; the search stops as
 *     soon as no unchecked entry remains.
 *   - duplicates: "visited" means the distance has been computed (Sec. 3.4,
 *     step iii); a node is added at most once.
 *   - ties and truncation use the (distance, id) key.
 *   - k > |pool|: missing results are (SENT, +inf).
 * `stop_hop` >= 0 makes the search stop right after that many expansions
 * (an expansion budget: the learned early stop, and the pool state read for
 * its features).
 * When `keep_visited` is set every visited node is appended to w->vis.
 * Returns the final pool size (>= 1).
 */
static int search_core(const float *base, int d, const uint32_t *graph, int R,
                       uint32_t start, const float *q, int L, ws_t *w,
                       int64_t *hops_out, int64_t *ndist_out, int64_t *nedges_out,
                       int keep_visited, int64_t stop_hop,
                       uint32_t *trace, int64_t trace_cap,
                       const uint32_t *init, int init_n)
{
    int64_t hops = 0, ndist = 0, nedges = 0;
    w->cur++;
    if (w->cur == 0) {                      /* stamp wrap-around */
        memset(w->stamp, 0, sizeof(uint32_t) * (size_t)w->n);
        w->cur = 1;
    }
    w->vis_cnt = 0;
    ws_pool_reserve(w, (L > init_n ? L : init_n) + R);
    pent_t *pool = w->pool;
    int size = 0;
    /* S.add(p): the start node, or (random initialization) every distinct
     * node of `init`, sorted and cut to L */
    const uint32_t *ini = init_n > 0 ? init : &start;
    const int nini = init_n > 0 ? init_n : 1;
    for (int j = 0; j < nini; ++j) {
        uint32_t u = ini[j];
        if (u >= (uint64_t)w->n || w->stamp[u] == w->cur) continue;
        w->stamp[u] = w->cur;
        pool[size].dist = oracle_l2sq_f32(q, base + (int64_t)u * d, d);
        pool[size].id = u;
        pool[size].checked = 0;
        ndist++;
        if (keep_visited) ws_vis_push(w, pool[size].dist, u);
        size++;
    }
    qsort(pool, (size_t)size, sizeof(pent_t), pent_cmp);
    if (size > L) size = L;

    for (;;) {
        if (stop_hop >= 0 && hops >= stop_hop) break;
        int i = -1;
        for (int t = 0; t < size; ++t)
            if (!pool[t].checked) { i = t; break; }
        if (i < 0) break;
        pool[i].checked = 1;
        uint32_t v = pool[i].id;
        if (trace && hops < trace_cap) trace[hops] = v;
        hops++;
        int add = 0;
        const uint32_t *row = graph + (int64_t)v * R;
        for (int j = 0; j < R; ++j) {
            uint32_t u = row[j];
            if (u == SENT) break;
            nedges++;
            if (w->stamp[u] == w->cur) continue;
            w->stamp[u] = w->cur;
            float du = oracle_l2sq_f32(q, base + (int64_t)u * d, d);
            ndist++;
            if (keep_visited) ws_vis_push(w, du, u);
            pool[size + add].dist = du;
            pool[size + add].id = u;
            pool[size + add].checked = 0;
            add++;
        }
        size += add;
        qsort(pool, (size_t)size, sizeof(pent_t), pent_cmp);
        if (size > L) size = L;
    }
    if (hops_out) *hops_out = hops;
    if (ndist_out) *ndist_out = ndist;
    if (nedges_out) *nedges_out = nedges;
    return size;
}

/*
 * Batched Algorithm 1 over nq queries, each from `start`, with per-query k and
 * L when k_arr / L_arr are non-NULL (else the scalars k, L).  out_ids /
 * out_dist are [nq][k_stride]; entries past k_i are left untouched; result
 * slots past the pool size hold (SENT, +inf).  hops/ndist may be NULL.
 * pool_ids/pool_dist ([nq][pool_stride], optional) receive the final pool.
 * max_hops_arr (optional): per-query expansion budget (the learned early
 * stop); a query stops after that many expansions; values <= 0: no budget.
 * nedges (optional): per query, the neighbour entries read (valid row
 * prefixes of the expanded nodes, visited or not).
 * init_ids (optional, [nq][init_n]): the initial pool of each query is the
 * set of these nodes instead of {start} (random initialization, the search
 * of the NSG-Naive baseline, Sec. 4.1.2; random starts, Sec. 4.1.3).
 * Growing the pool to hold them: the pool holds max(L, init_n) + R entries.
 * threads <= 0 uses the OpenMP default.
 */
int oracle_search_batch(const float *base, int64_t n, int d,
                        const uint32_t *graph, int R, uint32_t start,
                        const float *queries, int64_t nq,
                        int k, int L, const int32_t *k_arr, const int32_t *L_arr,
                        int k_stride, uint32_t *out_ids, float *out_dist,
                        int64_t *hops, int64_t *ndist,
                        uint32_t *pool_ids, float *pool_dist, int pool_stride,
                        const int32_t *max_hops_arr, int64_t *nedges,
                        const uint32_t *init_ids, int init_n, int threads)
{
    if (n < 1 || d < 1 || R < 1 || start >= (uint64_t)n || nq < 0) return -1;
    int maxL = L;
    if (L_arr) { maxL = 1; for (int64_t i = 0; i < nq; ++i) if (L_arr[i] > maxL) maxL = L_arr[i]; }
    if (init_ids && init_n > maxL) maxL = init_n;
    int bad = 0;
    int nth = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel num_threads(nth)
    {
        ws_t w;
        if (ws_init(&w, n, maxL + R) != 0) bad = 1;
#pragma omp for schedule(dynamic, 1)
        for (int64_t qi = 0; qi < nq; ++qi) {
            if (bad) continue;
            int kk = k_arr ? k_arr[qi] : k;
            int LL = L_arr ? L_arr[qi] : L;
            int64_t budget = (max_hops_arr && max_hops_arr[qi] > 0) ? max_hops_arr[qi] : -1;
            int64_t h = 0, nd = 0, ne = 0;
            int size = search_core(base, d, graph, R, start, queries + qi * (int64_t)d,
                                   LL, &w, &h, &nd, &ne, 0, budget, NULL, 0,
                                   init_ids ? init_ids + qi * (int64_t)init_n : NULL, init_ids ? init_n : 0);
            for (int j = 0; j < kk; ++j) {
                out_ids[qi * k_stride + j] = j < size ? w.pool[j].id : SENT;
                out_dist[qi * k_stride + j] = j < size ? w.pool[j].dist : INFINITY;
            }
            if (pool_ids)
                for (int j = 0; j < pool_stride; ++j) {
                    pool_ids[qi * pool_stride + j] = j < size ? w.pool[j].id : SENT;
                    pool_dist[qi * pool_stride + j] = j < size ? w.pool[j].dist : INFINITY;
                }
            if (hops) hops[qi] = h;
            if (ndist) ndist[qi] = nd;
            if (nedges) nedges[qi] = ne;
        }
        ws_free(&w);
    }
    return bad ? -2 : 0;
}

/*
 * One search with full diagnostics: the pool after `stop_hop` expansions (or
 * the final pool when stop_hop < 0), the checked flag of each pool entry, the
 * expansion order and the list of visited nodes with their distances.
 * Returns the pool size, or a negative value on error.
 */
int oracle_search_one(const float *base, int64_t n, int d,
                      const uint32_t *graph, int R, uint32_t start,
                      const float *q, int L, int64_t stop_hop,
                      uint32_t *pool_ids, float *pool_dist, int32_t *pool_checked,
                      uint32_t *trace, int64_t trace_cap,
                      uint32_t *vis_ids, float *vis_dist, int64_t vis_cap,
                      int64_t *stats /* hops, ndist, n_visited */)
{
    if (n < 1 || d < 1 || R < 1 || start >= (uint64_t)n || L < 1) return -1;
    ws_t w;
    if (ws_init(&w, n, L + R) != 0) { ws_free(&w); return -2; }
    int64_t h = 0, nd = 0;
    int size = search_core(base, d, graph, R, start, q, L, &w, &h, &nd, NULL, 1,
                           stop_hop, trace, trace_cap, NULL, 0);
    for (int j = 0; j < size; ++j) {
        if (pool_ids) pool_ids[j] = w.pool[j].id;
        if (pool_dist) pool_dist[j] = w.pool[j].dist;
        if (pool_checked) pool_checked[j] = w.pool[j].checked;
    }
    for (int64_t j = 0; j < w.vis_cnt && j < vis_cap; ++j) {
        if (vis_ids) vis_ids[j] = w.vis[j].id;
        if (vis_dist) vis_dist[j] = w.vis[j].dist;
    }
    if (stats) { stats[0] = h; stats[1] = nd; stats[2] = w.vis_cnt; }
    ws_free(&w);
    return size;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2, NSGbuild(G, l, m)                                            */
/* ------------------------------------------------------------------------ */

/* Centroid of the data set (Algorithm 2 first step; Sec. 3.4 step ii-1):
 * accumulated in FP64, rounded to FP32. */
int oracle_centroid(const float *base, int64_t n, int d, float *c)
{
    if (n < 1 || d < 1) return -1;
    for (int j = 0; j < d; ++j) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += (double)base[i * (int64_t)d + j];
        c[j] = (float)(s / (double)n);
    }
    return 0;
}

/* Navigating node (Algorithm 2 lines for centroid / random node / search;
 * Sec. 3.4 step ii): Algorithm 1 on the kNN graph from `rand_start` with the
 * centroid as query and pool size Lb; the first pool entry.  The random node
 * is an input (the caller draws it). */
int oracle_navigating_node(const float *base, int64_t n, int d,
                           const uint32_t *knn, int K, uint32_t rand_start,
                           int Lb, uint32_t *nav)
{
    if (n < 1 || d < 1 || K < 1 || rand_start >= (uint64_t)n || Lb < 1) return -1;
    float *c = (float *)malloc(sizeof(float) * (size_t)d);
    if (!c) return -2;
    oracle_centroid(base, n, d, c);
    ws_t w;
    if (ws_init(&w, n, Lb + K) != 0) { ws_free(&w); free(c); return -2; }
    search_core(base, d, knn, K, rand_start, c, Lb, &w, NULL, NULL, NULL, 0, -1, NULL, 0, NULL, 0);
    *nav = w.pool[0].id;
    ws_free(&w);
    free(c);
    return 0;
}

/*
 * MRNG edge selection over a candidate list already sorted by (distance to v,
 * id) (Algorithm 2 selection loop; Sec. 3.3 construction; Def. MRNG).
 * The first candidate is always kept (NNG is a subgraph of MRNG).  A later
 * candidate p is rejected when some already selected r satisfies
 * delta(p, r) < delta(v, p): then r lies in the open lune of v and p (r
 * precedes p so delta(v, r) <= delta(v, p)), i.e. vp is the longest edge of
 * triangle v p r; the printed conflict test is garbled and this is its
 * reading.  Equality is not a conflict (isosceles case broken by the (dist,
 * id) order of the candidates).  Stops at m selected edges.
 * Returns the number selected.
 */
static int mrng_select(const float *base, int d, const pent_t *E, int64_t ne,
                       int m, uint32_t *out)
{
    int cnt = 0;
    for (int64_t t = 0; t < ne && cnt < m; ++t) {
        const float *p = base + (int64_t)E[t].id * d;
        int conflict = 0;
        for (int s = 0; s < cnt; ++s) {
            float dpr = oracle_l2sq_f32(p, base + (int64_t)out[s] * d, d);
            if (dpr < E[t].dist) { conflict = 1; break; }
        }
        if (!conflict) out[cnt++] = E[t].id;
    }
    return cnt;
}

/*
 * Search-collect-select for one node v (Algorithm 2 body of the per-node
 * loop; Sec. 3.4 step iii; Fig. 5):
 *   E <- every node visited by Algorithm 1 on the kNN graph from nav with v
 *        as query and pool size Lb ("visited" = distance computed: Sec. 3.4
 *        step iii-2 and Fig. 5 say visited, the algorithm listing says
 *        checked; the superset is taken)
 *   E <- E + all K kNN neighbours of v; v itself and duplicates removed
 *   sort E by (distance to v, id); keep the first C (C <= 0: no cap)
 *   select at most m edges with the MRNG rule.
 * Writes the row (sentinel padded to m) and returns its length.
 */
static int collect_select(const float *base, int64_t n, int d,
                          const uint32_t *knn, int K, uint32_t nav, int Lb,
                          int C, int m, uint32_t v, ws_t *w, uint32_t *row)
{
    const float *qv = base + (int64_t)v * d;
    search_core(base, d, knn, K, nav, qv, Lb, w, NULL, NULL, NULL, 1, -1, NULL, 0, NULL, 0);
    /* the visited stamp marks exactly the visited ids; add unvisited kNN ids */
    for (int j = 0; j < K; ++j) {
        uint32_t u = knn[(int64_t)v * K + j];
        if (u == SENT || u >= (uint64_t)n) continue;
        if (w->stamp[u] == w->cur) continue;
        w->stamp[u] = w->cur;
        ws_vis_push(w, oracle_l2sq_f32(qv, base + (int64_t)u * d, d), u);
    }
    /* remove v */
    int64_t ne = 0;
    for (int64_t t = 0; t < w->vis_cnt; ++t)
        if (w->vis[t].id != v) w->vis[ne++] = w->vis[t];
    qsort(w->vis, (size_t)ne, sizeof(pent_t), pent_cmp);
    if (C > 0 && ne > C) ne = C;
    int cnt = mrng_select(base, d, w->vis, ne, m, row);
    for (int j = cnt; j < m; ++j) row[j] = SENT;
    return cnt;
}

/*
 * NSG-Naive (the baseline of Sec. 4.1.2): the MRNG edge selection applied to
 * each node's own kNN list only — candidates = the K kNN neighbours of v
 * (self and sentinels skipped), sorted by (distance to v, id) — with at most
 * m edges; no navigating node, no search-collect, no connectivity repair.
 * graph_out [n][m] sentinel padded.
 */
int oracle_build_naive(const float *base, int64_t n, int d, const uint32_t *knn, int K, int m,
                       uint32_t *graph_out)
{
    if (n < 1 || d < 1 || K < 1 || m < 1) return -1;
    int bad = 0;
#pragma omp parallel
    {
        pent_t *E = (pent_t *)malloc(sizeof(pent_t) * (size_t)K);
        if (!E) bad = 1;
#pragma omp for schedule(dynamic, 64)
        for (int64_t v = 0; v < n; ++v) {
            if (!E) continue;
            int ne = 0;
            for (int j = 0; j < K; ++j) {
                uint32_t u = knn[v * K + j];
                if (u == SENT || u >= (uint64_t)n || u == (uint32_t)v) continue;
                int dup = 0;
                for (int t = 0; t < ne; ++t) dup |= E[t].id == u;
                if (dup) continue;
                E[ne].id = u;
                E[ne].dist = oracle_l2sq_f32(base + v * d, base + (int64_t)u * d, d);
                E[ne].checked = 0;
                ne++;
            }
            qsort(E, (size_t)ne, sizeof(pent_t), pent_cmp);
            uint32_t *row = graph_out + v * m;
            int cnt = mrng_select(base, d, E, ne, m, row);
            for (int j = cnt; j < m; ++j) row[j] = SENT;
        }
        free(E);
    }
    return bad ? -2 : 0;
}

/* Exposed per-node step for tests. */
int oracle_collect_select(const float *base, int64_t n, int d,
                          const uint32_t *knn, int K, uint32_t nav, int Lb,
                          int C, int m, uint32_t v, uint32_t *row)
{
    if (n < 1 || d < 1 || K < 1 || nav >= (uint64_t)n || v >= (uint64_t)n || m < 1) return -1;
    ws_t w;
    if (ws_init(&w, n, Lb + K) != 0) { ws_free(&w); return -2; }
    int cnt = collect_select(base, n, d, knn, K, nav, Lb, C, m, v, &w, row);
    ws_free(&w);
    return cnt;
}

/* Iterative DFS over graph from root, marking reached[] (Algorithm 2 tree
 * spanning).  The stack holds at most n entries. */
static void dfs_mark(const uint32_t *graph, int m, uint32_t root,
                     unsigned char *reached, uint32_t *stack)
{
    int64_t top = 0;
    if (reached[root]) return;
    reached[root] = 1;
    stack[top++] = root;
    while (top > 0) {
        uint32_t v = stack[--top];
        const uint32_t *row = graph + (int64_t)v * m;
        for (int j = 0; j < m; ++j) {
            uint32_t u = row[j];
            if (u == SENT) break;
            if (!reached[u]) { reached[u] = 1; stack[top++] = u; }
        }
    }
}

/*
 * Connectivity repair (Algorithm 2 final loop; Sec. 3.4 step iv):
 * span a DFS tree from nav; while a node is not reached, take the smallest
 * unreached id u, search the current graph from nav for u with pool size Lb
 * (Algorithm 1), link the first pool entry w whose out-degree is below m
 * (w -> u, so that nav reaches u; the direction is unstated and this is the
 * reading), and continue the DFS from u.  If no pool entry has room, the
 * nearest reached node with room is found by a full scan.  Returns the number
 * of edges added, or -3 when no reached node has room.
 */
int oracle_repair(const float *base, int64_t n, int d, uint32_t *graph, int m,
                  uint32_t nav, int Lb)
{
    unsigned char *reached = (unsigned char *)calloc((size_t)n, 1);
    uint32_t *stack = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    int *deg = (int *)malloc(sizeof(int) * (size_t)n);
    ws_t w;
    if (!reached || !stack || !deg || ws_init(&w, n, Lb + m) != 0) {
        free(reached); free(stack); free(deg); return -2;
    }
    for (int64_t v = 0; v < n; ++v) {
        int c = 0;
        while (c < m && graph[v * m + c] != SENT) ++c;
        deg[v] = c;
    }
    dfs_mark(graph, m, nav, reached, stack);
    int64_t added = 0;
    int64_t scan = 0;
    int err = 0;
    for (;;) {
        while (scan < n && reached[scan]) ++scan;
        if (scan >= n) break;
        uint32_t u = (uint32_t)scan;
        const float *qu = base + (int64_t)u * d;
        int size = search_core(base, d, graph, m, nav, qu, Lb, &w, NULL, NULL, NULL, 0,
                               -1, NULL, 0, NULL, 0);
        int64_t wsel = -1;
        for (int t = 0; t < size; ++t) {
            uint32_t c = w.pool[t].id;
            if (reached[c] && deg[c] < m) { wsel = c; break; }
        }
        if (wsel < 0) {
            float best = INFINITY;
            for (int64_t c = 0; c < n; ++c) {
                if (!reached[c] || deg[c] >= m) continue;
                float dc = oracle_l2sq_f32(qu, base + c * d, d);
                if (wsel < 0 || dc < best) { best = dc; wsel = c; }
            }
        }
        if (wsel < 0) { err = -3; break; }
        graph[wsel * m + deg[wsel]] = u;
        deg[wsel]++;
        added++;
        dfs_mark(graph, m, u, reached, stack);
    }
    ws_free(&w);
    free(reached); free(stack); free(deg);
    return err ? err : (int)added;
}

/*
 * Full Algorithm 2 from an exact or approximate kNN graph knn[n][K]:
 * navigating node, per-node search-collect-select (independent per node, so
 * run in parallel), then connectivity repair.  graph_out is [n][m].
 * stats (optional): [0] = edges added by the repair.
 * Returns 0 or a negative error.
 */
int oracle_build_nsg(const float *base, int64_t n, int d, const uint32_t *knn,
                     int K, int Lb, int C, int m, uint32_t rand_start,
                     uint32_t *graph_out, uint32_t *nav_out, int64_t *stats,
                     int threads)
{
    if (n < 2 || d < 1 || K < 1 || Lb < 1 || m < 1 || rand_start >= (uint64_t)n) return -1;
    uint32_t nav;
    int rc = oracle_navigating_node(base, n, d, knn, K, rand_start, Lb, &nav);
    if (rc) return rc;
    int bad = 0;
    int nth = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel num_threads(nth)
    {
        ws_t w;
        if (ws_init(&w, n, Lb + K) != 0) bad = 1;
#pragma omp for schedule(dynamic, 64)
        for (int64_t v = 0; v < n; ++v) {
            if (bad) continue;
            collect_select(base, n, d, knn, K, nav, Lb, C, m, (uint32_t)v, &w,
                           graph_out + v * m);
        }
        ws_free(&w);
    }
    if (bad) return -2;
    int added = oracle_repair(base, n, d, graph_out, m, nav, Lb);
    if (added < 0) return added;
    if (stats) stats[0] = added;
    *nav_out = nav;
    return 0;
}

/*
 * Naive MRNG construction (Sec. 3.3, "MRNG Construction"): for each p, rank
 * all other nodes by (distance to p, id); keep the closest; then walk the rest
 * in order and keep q unless pq is the longest edge of triangle pqr for some
 * kept r, i.e. unless delta(q, r) < delta(p, q).  prec selects FP64 or FP32
 * distances.  out is [n][n-1] (sentinel padded), deg[n] the row lengths.
 */
int oracle_mrng_naive(const float *base, int64_t n, int d, int prec,
                      uint32_t *out, int32_t *deg)
{
    if (n < 2 || d < 1 || (prec != 32 && prec != 64)) return -1;
    int64_t w = n - 1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < n; ++p) {
        dkey_t *E = (dkey_t *)malloc(sizeof(dkey_t) * (size_t)w);
        if (!E) { bad = 1; continue; }
        int64_t ne = 0;
        const float *xp = base + p * d;
        for (int64_t q = 0; q < n; ++q) {
            if (q == p) continue;
            const float *xq = base + q * d;
            E[ne].key = prec == 64 ? oracle_l2sq_f64(xp, xq, d) : (double)oracle_l2sq_f32(xp, xq, d);
            E[ne].id = (uint32_t)q;
            ne++;
        }
        /* insertion sort by (key, id): plain and obviously ordered */
        for (int64_t a = 1; a < ne; ++a) {
            dkey_t t = E[a];
            int64_t b = a;
            while (b > 0 && dkey_less(t.key, t.id, E[b - 1].key, E[b - 1].id)) { E[b] = E[b - 1]; --b; }
            E[b] = t;
        }
        uint32_t *row = out + p * w;
        int cnt = 0;
        for (int64_t t = 0; t < ne; ++t) {
            const float *xq = base + (int64_t)E[t].id * d;
            int keep = 1;
            for (int s = 0; s < cnt; ++s) {
                const float *xr = base + (int64_t)row[s] * d;
                double dqr = prec == 64 ? oracle_l2sq_f64(xq, xr, d) : (double)oracle_l2sq_f32(xq, xr, d);
                if (dqr < E[t].key) { keep = 0; break; }
            }
            if (keep) row[cnt++] = E[t].id;
        }
        for (int64_t j = cnt; j < w; ++j) row[j] = SENT;
        deg[p] = cnt;
        free(E);
    }
    return bad ? -2 : 0;
}

/* ------------------------------------------------------------------------ */
/* Reduced-precision storage (not in the paper): per-dimension FP32 scale,   */
/* encode by round-to-nearest-even with saturation, decode = s_d * value.    */
/* ------------------------------------------------------------------------ */

/*
 * Generic binary floating-point format with `eb` exponent bits and `mb`
 * mantissa bits, exponent bias 2^(eb-1)-1, subnormals, value of a code
 * computed from its fields.  `max_finite` is the largest finite magnitude.
 * For IEEE binary16 (eb=5, mb=10) and bfloat16 (eb=8, mb=7) the all-ones
 * exponent is inf/NaN; for OCP FP8 E4M3 (eb=4, mb=3) only S.1111.111 is NaN
 * and the rest of the top binade is finite (max 448).
 */
typedef struct { int eb, mb, ocp_e4m3; } fmt_t;

static double fmt_decode(fmt_t f, uint32_t code)
{
    int bits = 1 + f.eb + f.mb;
    uint32_t sign = (code >> (bits - 1)) & 1u;
    uint32_t e = (code >> f.mb) & ((1u << f.eb) - 1u);
    uint32_t m = code & ((1u << f.mb) - 1u);
    int bias = (1 << (f.eb - 1)) - 1;
    uint32_t emax = (1u << f.eb) - 1u;
    double v;
    if (!f.ocp_e4m3 && e == emax) {
        v = m ? NAN : INFINITY;
    } else if (f.ocp_e4m3 && e == emax && m == (1u << f.mb) - 1u) {
        v = NAN;
    } else if (e == 0) {
        v = ldexp((double)m, 1 - bias - f.mb);
    } else {
        v = ldexp((double)((1u << f.mb) | m), (int)e - bias - f.mb);
    }
    return sign ? -v : v;
}

static double fmt_max_finite(fmt_t f)
{
    int bias = (1 << (f.eb - 1)) - 1;
    if (f.ocp_e4m3) /* top binade, mantissa 110 */
        return ldexp((double)((1u << f.mb) | ((1u << f.mb) - 2u)), ((1 << f.eb) - 1) - bias - f.mb);
    return ldexp((double)((1u << (f.mb + 1)) - 1u), ((1 << f.eb) - 2) - bias - f.mb);
}

/*
 * Round-to-nearest-even encode with saturation to the largest finite value.
 * Works in FP64 on the exact FP32 input: find the quantum (spacing of
 * representable values) at the input's binade, round x/quantum to the nearest
 * integer with ties to even, rebuild the code from the rounded magnitude.
 */
static uint32_t fmt_encode(fmt_t f, float xf)
{
    int bits = 1 + f.eb + f.mb;
    uint32_t sign = signbit(xf) ? 1u : 0u;
    double x = fabs((double)xf);
    int bias = (1 << (f.eb - 1)) - 1;
    if (isnan(xf)) {
        if (f.ocp_e4m3) return (sign << (bits - 1)) | 0x7Fu;
        return (sign << (bits - 1)) | (((1u << f.eb) - 1u) << f.mb) | (1u << (f.mb - 1));
    }
    double maxf = fmt_max_finite(f);
    if (x >= maxf) { /* saturate (covers +inf) */
        x = maxf;
    }
    int emin = 1 - bias;                    /* exponent of the smallest normal */
    int ex;
    if (x == 0.0) return sign << (bits - 1);
    frexp(x, &ex);                          /* x = fr * 2^ex, fr in [0.5, 1) */
    int e = ex - 1;                         /* x in [2^e, 2^(e+1)) */
    if (e < emin) e = emin;                 /* subnormal range shares the quantum */
    double quantum = ldexp(1.0, e - f.mb);
    double r = x / quantum;                 /* exact: power-of-two division */
    double ri = nearbyint(r);               /* default rounding mode: ties to even */
    double mag = ri * quantum;
    if (mag > maxf) mag = maxf;             /* rounding up past the top saturates */
    /* rebuild the code from mag */
    uint32_t code;
    if (mag < ldexp(1.0, emin)) {
        code = (uint32_t)(mag / ldexp(1.0, emin - f.mb));
    } else {
        int ex2;
        frexp(mag, &ex2);
        int e2 = ex2 - 1;
        uint32_t m = (uint32_t)(mag / ldexp(1.0, e2 - f.mb)) - (1u << f.mb);
        code = ((uint32_t)(e2 + bias) << f.mb) | m;
    }
    return (sign << (bits - 1)) | code;
}

static fmt_t fmt_of(int dtype)
{
    fmt_t f = {0, 0, 0};
    if (dtype == 1) { f.eb = 8; f.mb = 7; }          /* bfloat16 */
    else if (dtype == 2) { f.eb = 5; f.mb = 10; }    /* IEEE binary16 */
    else if (dtype == 3) { f.eb = 4; f.mb = 3; f.ocp_e4m3 = 1; } /* OCP E4M3 */
    return f;
}

/* Decode codes -> float (no scale).  dtype 1 bf16, 2 f16, 3 e4m3. */
int oracle_decode(int dtype, const void *codes, int64_t cnt, float *out)
{
    if (dtype < 1 || dtype > 3) return -1;
    fmt_t f = fmt_of(dtype);
    for (int64_t i = 0; i < cnt; ++i) {
        uint32_t c = dtype == 3 ? ((const uint8_t *)codes)[i] : ((const uint16_t *)codes)[i];
        out[i] = (float)fmt_decode(f, c);
    }
    return 0;
}

/* Encode floats -> codes (no scale), RNE with saturation. */
int oracle_encode(int dtype, const float *x, int64_t cnt, void *codes)
{
    if (dtype < 1 || dtype > 3) return -1;
    fmt_t f = fmt_of(dtype);
    for (int64_t i = 0; i < cnt; ++i) {
        uint32_t c = fmt_encode(f, x[i]);
        if (dtype == 3) ((uint8_t *)codes)[i] = (uint8_t)c;
        else ((uint16_t *)codes)[i] = (uint16_t)c;
    }
    return 0;
}

/*
 * Per-dimension scales: s_j = max_i |x_ij| / M with M = 448 for E4M3 and
 * M = 1 for FP16 / BF16 (reading: every reduced format carries per-dimension
 * FP32 scales); s_j = 1 when the column is all zero.
 */
int oracle_scales(int dtype, const float *base, int64_t n, int d, float *scales)
{
    if (dtype < 1 || dtype > 3 || n < 1 || d < 1) return -1;
    float M = dtype == 3 ? 448.0f : 1.0f;
    for (int j = 0; j < d; ++j) {
        float mx = 0.0f;
        for (int64_t i = 0; i < n; ++i) {
            float a = fabsf(base[i * d + j]);
            if (a > mx) mx = a;
        }
        scales[j] = mx > 0.0f ? mx / M : 1.0f;
    }
    return 0;
}

/* Quantise the base: code = enc(x / s_j) (FP32 division), and the decoded
 * rows xt = fl32(s_j * dec(code)) that reduced-precision search works on. */
int oracle_quantize(int dtype, const float *base, int64_t n, int d,
                    const float *scales, void *codes, float *decoded)
{
    if (dtype < 1 || dtype > 3 || n < 0 || d < 1) return -1;
    fmt_t f = fmt_of(dtype);
    for (int64_t i = 0; i < n; ++i)
        for (int j = 0; j < d; ++j) {
            float y = base[i * d + j] / scales[j];
            uint32_t c = fmt_encode(f, y);
            if (codes) {
                if (dtype == 3) ((uint8_t *)codes)[i * d + j] = (uint8_t)c;
                else ((uint16_t *)codes)[i * d + j] = (uint16_t)c;
            }
            if (decoded) {
                float v = (float)fmt_decode(f, c);
                decoded[i * d + j] = scales[j] * v;
            }
        }
    return 0;
}

/*
 * Re-rank (reduced-precision extension): exact FP32 squared distances from
 * the FP32 base for every entry of a final pool, re-sorted by (distance, id),
 * first k emitted (SENT/+inf padded).
 */
int oracle_rerank(const float *base, int d, const float *queries, int64_t nq,
                  const uint32_t *pool_ids, int pool_stride, int k,
                  uint32_t *out_ids, float *out_dist)
{
    if (d < 1 || k < 1 || pool_stride < 1) return -1;
    for (int64_t qi = 0; qi < nq; ++qi) {
        pent_t *tmp = (pent_t *)malloc(sizeof(pent_t) * (size_t)pool_stride);
        if (!tmp) return -2;
        int cnt = 0;
        for (int j = 0; j < pool_stride; ++j) {
            uint32_t id = pool_ids[qi * pool_stride + j];
            if (id == SENT) continue;
            tmp[cnt].id = id;
            tmp[cnt].dist = oracle_l2sq_f32(queries + qi * d, base + (int64_t)id * d, d);
            tmp[cnt].checked = 0;
            cnt++;
        }
        qsort(tmp, (size_t)cnt, sizeof(pent_t), pent_cmp);
        for (int j = 0; j < k; ++j) {
            out_ids[qi * k + j] = j < cnt ? tmp[j].id : SENT;
            out_dist[qi * k + j] = j < cnt ? tmp[j].dist : INFINITY;
        }
        free(tmp);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Learned early termination (not in the paper): a 3-layer perceptron        */
/* in -> h -> h -> 1 with ReLU, FP64 forward, MSE loss and backward, Adam.   */
/* Parameter layout (row-major): W1[h][in], b1[h], W2[h][h], b2[h], W3[h],   */
/* b3[1].                                                                    */
/* ------------------------------------------------------------------------ */

int64_t oracle_mlp_nparams(int in, int h)
{
    return (int64_t)h * in + h + (int64_t)h * h + h + h + 1;
}

/*
 * Forward pass for B rows of X[B][in]; yhat[B].  If y and grad are non-NULL,
 * also the loss (1/B) * sum (yhat - y)^2 is returned and its gradient with
 * respect to every parameter is written to grad (same layout as params).
 * Plain per-sample backpropagation in FP64.
 */
double oracle_mlp_loss_grad(const double *params, int in, int h,
                            const double *X, const double *y, int64_t B,
                            double *yhat, double *grad)
{
    const double *W1 = params;
    const double *b1 = W1 + (int64_t)h * in;
    const double *W2 = b1 + h;
    const double *b2 = W2 + (int64_t)h * h;
    const double *W3 = b2 + h;
    const double *b3 = W3 + h;
    int64_t np = oracle_mlp_nparams(in, h);
    if (grad) memset(grad, 0, sizeof(double) * (size_t)np);
    double *gW1 = grad, *gb1 = grad ? gW1 + (int64_t)h * in : NULL;
    double *gW2 = grad ? gb1 + h : NULL, *gb2 = grad ? gW2 + (int64_t)h * h : NULL;
    double *gW3 = grad ? gb2 + h : NULL, *gb3 = grad ? gW3 + h : NULL;
    double *z1 = (double *)malloc(sizeof(double) * (size_t)h * 4);
    double *a1 = z1 + h, *z2 = a1 + h, *a2 = z2 + h;
    double *d1 = (double *)malloc(sizeof(double) * (size_t)h * 2);
    double *d2 = d1 + h;
    double loss = 0.0;
    for (int64_t b = 0; b < B; ++b) {
        const double *x = X + b * in;
        for (int i = 0; i < h; ++i) {
            double s = b1[i];
            for (int j = 0; j < in; ++j) s += W1[(int64_t)i * in + j] * x[j];
            z1[i] = s;
            a1[i] = s > 0.0 ? s : 0.0;
        }
        for (int i = 0; i < h; ++i) {
            double s = b2[i];
            for (int j = 0; j < h; ++j) s += W2[(int64_t)i * h + j] * a1[j];
            z2[i] = s;
            a2[i] = s > 0.0 ? s : 0.0;
        }
        double o = b3[0];
        for (int j = 0; j < h; ++j) o += W3[j] * a2[j];
        if (yhat) yhat[b] = o;
        if (y && grad) {
            double e = o - y[b];
            loss += e * e;
            double go = 2.0 * e / (double)B;          /* d loss / d o */
            gb3[0] += go;
            for (int j = 0; j < h; ++j) {
                gW3[j] += go * a2[j];
                d2[j] = z2[j] > 0.0 ? go * W3[j] : 0.0; /* d loss / d z2 */
            }
            for (int i = 0; i < h; ++i) {
                gb2[i] += d2[i];
                for (int j = 0; j < h; ++j) gW2[(int64_t)i * h + j] += d2[i] * a1[j];
            }
            for (int j = 0; j < h; ++j) {
                double s = 0.0;
                for (int i = 0; i < h; ++i) s += W2[(int64_t)i * h + j] * d2[i];
                d1[j] = z1[j] > 0.0 ? s : 0.0;       /* d loss / d z1 */
            }
            for (int i = 0; i < h; ++i) {
                gb1[i] += d1[i];
                for (int j = 0; j < in; ++j) gW1[(int64_t)i * in + j] += d1[i] * x[j];
            }
        } else if (y) {
            double e = o - y[b];
            loss += e * e;
        }
    }
    free(z1); free(d1);
    return B > 0 ? loss / (double)B : 0.0;
}

/*
 * One Adam step (Kingma & Ba) over np parameters at step t (1-based):
 * m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
 * p <- p - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
 */
int oracle_adam_step(double *params, const double *grad, double *m, double *v,
                     int64_t np, int64_t t, double lr, double b1, double b2, double eps)
{
    if (t < 1) return -1;
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < np; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
        v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        params[i] -= lr * mh / (sqrt(vh) + eps);
    }
    return 0;
}
