"""CPU oracle for NSG search — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct C (``nsg_oracle.c``) behind ctypes.  Only the
test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1707_00143_amd``) and never imports it.

Each wrapper cites the passage of the paper it follows; the C source states
every reading taken where the paper is silent or garbled.

Parity status per function (see the tests named):
  knn             pinned: NumPy FP64 brute force (test_oracle_knn)
  search          pinned: exhaustive-L / complete-graph special cases equal
                  exact kNN; hand-traced golden example; Theorem 1+3 greedy
                  walk on exact MRNG; pool invariant (test_oracle_search)
  mrng_naive      pinned: the MRNG definition checked pair by pair with
                  open lunes in FP64 (test_oracle_build)
  build_nsg       pinned: degree bound, reachability, NN-percentage, the
                  pairwise rule, MRNG equivalence with uncapped candidates
  encode/decode   pinned: NumPy float16, torch bfloat16 / float8_e4m3fn
                  (test_oracle_precision)
  mlp             pinned: central finite differences and torch FP64 autograd
                  (test_oracle_mlp)
  stop_features   pinned: hand-worked state with literal expected values
                  (test_oracle_mlp)
  search_sharded  pinned: one shard = the plain search; exhaustive pools in
  / merge_topk    every shard = exact kNN of the whole base; hand merge
                  with ties and padding (test_oracle_shards)
  build_naive     pinned: with every other node as candidates and no degree
                  cap it is the naive MRNG; rows are subsets of the kNN rows
                  obeying the pairwise rule (test_oracle_ablations)
  search init_ids pinned: a set holding every node = exhaustive pool (exact
                  kNN); a one-node set = the search started there
                  (test_oracle_ablations)
  rerank          pinned: hand case with a tie and padding; a pool holding
                  the exact top-k returns it (integer data, exact distances);
                  per-query stride (test_oracle_rerank)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nsg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
SENT = 0xFFFFFFFF

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle (gcc -O2 -ffp-contract=off, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
            "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _get():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, u32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_uint32, ctypes.c_double
        sig = {
            "oracle_l2sq_f32": (ctypes.c_float, [P, P, i32]),
            "oracle_l2sq_f64": (f64, [P, P, i32]),
            "oracle_knn": (i32, [P, i64, i32, P, i64, i32, i32, i32, P, P]),
            "oracle_search_batch": (i32, [P, i64, i32, P, i32, u32, P, i64, i32, i32, P, P,
                                          i32, P, P, P, P, P, P, i32, P, P, P, i32, i32]),
            "oracle_build_naive": (i32, [P, i64, i32, P, i32, i32, P]),
            "oracle_knn_ivf": (i32, [P, i64, i32, P, i32, i32, i32, P, P, P]),
            "oracle_search_one": (i32, [P, i64, i32, P, i32, u32, P, i32, i64, P, P, P,
                                        P, i64, P, P, i64, P]),
            "oracle_centroid": (i32, [P, i64, i32, P]),
            "oracle_navigating_node": (i32, [P, i64, i32, P, i32, u32, i32, P]),
            "oracle_collect_select": (i32, [P, i64, i32, P, i32, u32, i32, i32, i32, u32, P]),
            "oracle_repair": (i32, [P, i64, i32, P, i32, u32, i32]),
            "oracle_build_nsg": (i32, [P, i64, i32, P, i32, i32, i32, i32, u32, P, P, P, i32]),
            "oracle_mrng_naive": (i32, [P, i64, i32, i32, P, P]),
            "oracle_decode": (i32, [i32, P, i64, P]),
            "oracle_encode": (i32, [i32, P, i64, P]),
            "oracle_scales": (i32, [i32, P, i64, i32, P]),
            "oracle_quantize": (i32, [i32, P, i64, i32, P, P, P]),
            "oracle_rerank": (i32, [P, i32, P, i64, P, i32, i32, P, P]),
            "oracle_mlp_nparams": (i64, [i32, i32]),
            "oracle_mlp_loss_grad": (f64, [P, i32, i32, P, P, i64, P, P]),
            "oracle_adam_step": (i32, [P, P, P, P, i64, i64, f64, f64, f64, f64]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")
    return rc


# --------------------------------------------------------------------------
# distances and exact kNN (Sec. 2.1 K-NNS; Sec. 4.1.2 serial scan)
# --------------------------------------------------------------------------

def l2sq_f32(a, b) -> float:
    a, b = _f32(a), _f32(b)
    return float(_get().oracle_l2sq_f32(_p(a), _p(b), a.shape[-1]))


def knn(base, queries, k, prec=64, exclude_self=False):
    """Exact kNN ordered by (squared distance, id); FP64 keys by default."""
    base, queries = _f32(base), _f32(queries)
    n, d = base.shape
    nq = queries.shape[0]
    ids = np.empty((nq, k), np.uint32)
    dist = np.empty((nq, k), np.float64)
    _check(_get().oracle_knn(_p(base), n, d, _p(queries), nq, k, prec,
                             1 if exclude_self else 0, _p(ids), _p(dist)), "knn")
    return ids, dist


def knn_graph(base, K):
    """Exact kNN graph: each row ordered by (FP32 squared distance, id), self
    excluded (Algorithm 2 input, step i of Sec. 3.4, exact here)."""
    ids, _ = knn(base, base, K, prec=32, exclude_self=True)
    return ids


# --------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------

def search(base, graph, start, queries, k, L, k_arr=None, L_arr=None, pool_stride=0,
           max_hops=None, threads=0, nedges=None, init_ids=None):
    """Batched Algorithm 1 from `start`.  Returns (ids, dist, hops, ndist[, pool_ids,
    pool_dist]).  With per-query k_arr / L_arr the outputs are [nq][max k].
    max_hops: optional per-query expansion budget (<= 0: none).  nedges: an
    optional int64 [nq] array that receives the neighbour entries each query
    read (the valid row prefixes of its expanded nodes).  init_ids: optional
    [nq][m] node ids; each query's initial pool is that set (random
    initialization) instead of {start}."""
    base, graph, queries = _f32(base), _u32(graph), _f32(queries)
    n, d = base.shape
    R = graph.shape[1]
    nq = queries.shape[0]
    k_arr_c = None if k_arr is None else np.ascontiguousarray(k_arr, np.int32)
    L_arr_c = None if L_arr is None else np.ascontiguousarray(L_arr, np.int32)
    kst = int(k_arr_c.max()) if k_arr_c is not None and nq else k
    ids = np.full((nq, kst), SENT, np.uint32)
    dist = np.full((nq, kst), np.inf, np.float32)
    hops = np.zeros(nq, np.int64)
    nd = np.zeros(nq, np.int64)
    pids = pd = None
    if pool_stride:
        pids = np.empty((nq, pool_stride), np.uint32)
        pd = np.empty((nq, pool_stride), np.float32)
    mh = None if max_hops is None else np.ascontiguousarray(np.broadcast_to(max_hops, (nq,)), np.int32)
    ini, ini_n = None, 0
    if init_ids is not None:
        ini = np.ascontiguousarray(init_ids, np.uint32)
        assert ini.ndim == 2 and ini.shape[0] == nq
        ini_n = ini.shape[1]
    ne = None
    if nedges is not None:
        assert nedges.dtype == np.int64 and nedges.shape == (nq,) and nedges.flags.c_contiguous
        ne = nedges
    _check(_get().oracle_search_batch(
        _p(base), n, d, _p(graph), R, int(start), _p(queries), nq, int(k), int(L),
        _p(k_arr_c), _p(L_arr_c), kst, _p(ids), _p(dist), _p(hops), _p(nd),
        _p(pids), _p(pd), int(pool_stride), _p(mh), _p(ne), _p(ini), ini_n, int(threads)), "search")
    if pool_stride:
        return ids, dist, hops, nd, pids, pd
    return ids, dist, hops, nd


def search_one(base, graph, start, q, L, stop_hop=-1, trace_cap=4096, vis_cap=1 << 20):
    """One Algorithm 1 run with diagnostics: dict with pool ids/dist/checked,
    expansion trace, visited list, hops, ndist."""
    base, graph, q = _f32(base), _u32(graph), _f32(q)
    n, d = base.shape
    R = graph.shape[1]
    pids = np.empty(L + R, np.uint32)
    pdist = np.empty(L + R, np.float32)
    pchk = np.empty(L + R, np.int32)
    trace = np.empty(trace_cap, np.uint32)
    vid = np.empty(vis_cap, np.uint32)
    vdist = np.empty(vis_cap, np.float32)
    stats = np.zeros(3, np.int64)
    size = _check(_get().oracle_search_one(
        _p(base), n, d, _p(graph), R, int(start), _p(q), int(L), int(stop_hop),
        _p(pids), _p(pdist), _p(pchk), _p(trace), trace_cap, _p(vid), _p(vdist), vis_cap,
        _p(stats)), "search_one")
    h, ndist, nv = (int(x) for x in stats)
    return dict(pool_ids=pids[:size].copy(), pool_dist=pdist[:size].copy(),
                pool_checked=pchk[:size].astype(bool), trace=trace[:min(h, trace_cap)].copy(),
                vis_ids=vid[:min(nv, vis_cap)].copy(), vis_dist=vdist[:min(nv, vis_cap)].copy(),
                hops=h, ndist=ndist)


def merge_topk(ids, dist, k):
    """Top k of the union of per-shard result lists: ids/dist [nq][S][k_s]
    (global ids, SENT/+inf padding), ordered by (distance, id); the plain
    definition of the merge (a sort of the concatenation), padded with
    (SENT, +inf) when fewer than k results exist."""
    ids = np.asarray(ids, np.uint32)
    dist = np.asarray(dist, np.float32)
    nq = ids.shape[0]
    out_i = np.full((nq, k), SENT, np.uint32)
    out_d = np.full((nq, k), np.inf, np.float32)
    for q in range(nq):
        ii, dd = ids[q].ravel(), dist[q].ravel()
        ok = ii != SENT
        ii, dd = ii[ok], dd[ok]
        order = np.lexsort((ii, dd))[:k]
        out_i[q, :len(order)] = ii[order]
        out_d[q, :len(order)] = dd[order]
    return out_i, out_d


def search_sharded(base, offsets, graph, navs, queries, k, L, threads=0, walk_rows=None):
    """The partitioned scheme of the paper's large-scale experiments (one
    sub-NSG per subset, every query searched in every subset, the per-subset
    results merged; Sec. 4.2 "Search On DEEP100M", Sec. 4.3): shard s holds
    base rows offsets[s] .. offsets[s+1] - 1 and its own graph rows (local
    ids, same rows of `graph`) and navigating node navs[s] (local id).
    Algorithm 1 runs in each shard at pool size L; its top k (mapped to
    global ids) are merged by merge_topk.  With walk_rows (decoded
    reduced-precision rows [n][d]) each shard's walk runs on them and its
    final pool is re-ranked on `base` (rerank) before the shard's top k is
    taken.  Returns (ids, dist, per-shard ids [nq][S][k], per-shard dist)."""
    base, graph, queries = _f32(base), _u32(graph), _f32(queries)
    S = len(offsets) - 1
    nq = queries.shape[0]
    sid = np.full((nq, S, k), SENT, np.uint32)
    sd = np.full((nq, S, k), np.inf, np.float32)
    for s in range(S):
        a, b = int(offsets[s]), int(offsets[s + 1])
        if walk_rows is None:
            ids, dist, _, _ = search(base[a:b], graph[a:b], int(navs[s]), queries, k, L, threads=threads)
        else:
            _, _, _, _, pids, _ = search(_f32(walk_rows)[a:b], graph[a:b], int(navs[s]), queries, k, L,
                                         pool_stride=L, threads=threads)
            ids, dist = rerank(base[a:b], queries, pids, k)
        ok = ids != SENT
        sid[:, s] = np.where(ok, ids + np.uint32(a), SENT)
        sd[:, s] = dist
    out_i, out_d = merge_topk(sid, sd, k)
    return out_i, out_d, sid, sd


# --------------------------------------------------------------------------
# Algorithm 2 and the naive MRNG
# --------------------------------------------------------------------------

def centroid(base):
    base = _f32(base)
    c = np.empty(base.shape[1], np.float32)
    _check(_get().oracle_centroid(_p(base), base.shape[0], base.shape[1], _p(c)), "centroid")
    return c


def navigating_node(base, knn_g, rand_start, Lb):
    base, knn_g = _f32(base), _u32(knn_g)
    nav = np.zeros(1, np.uint32)
    _check(_get().oracle_navigating_node(_p(base), base.shape[0], base.shape[1], _p(knn_g),
                                         knn_g.shape[1], int(rand_start), int(Lb), _p(nav)),
           "navigating_node")
    return int(nav[0])


def collect_select(base, knn_g, nav, Lb, C, m, v):
    base, knn_g = _f32(base), _u32(knn_g)
    row = np.empty(m, np.uint32)
    cnt = _check(_get().oracle_collect_select(_p(base), base.shape[0], base.shape[1],
                                              _p(knn_g), knn_g.shape[1], int(nav), int(Lb),
                                              int(C), int(m), int(v), _p(row)), "collect_select")
    return row[:cnt].copy()


def repair(base, graph, nav, Lb):
    """Connectivity repair in place; returns the number of edges added."""
    base = _f32(base)
    assert graph.dtype == np.uint32 and graph.flags.c_contiguous
    return _check(_get().oracle_repair(_p(base), base.shape[0], base.shape[1], _p(graph),
                                       graph.shape[1], int(nav), int(Lb)), "repair")


def build_nsg(base, knn_g, Lb, C, m, rand_start, threads=0):
    """Algorithm 2.  Returns (graph [n][m] uint32 sentinel-padded, nav, repair_edges)."""
    base, knn_g = _f32(base), _u32(knn_g)
    n, d = base.shape
    g = np.empty((n, m), np.uint32)
    nav = np.zeros(1, np.uint32)
    stats = np.zeros(4, np.int64)
    _check(_get().oracle_build_nsg(_p(base), n, d, _p(knn_g), knn_g.shape[1], int(Lb), int(C),
                                   int(m), int(rand_start), _p(g), _p(nav), _p(stats),
                                   int(threads)), "build_nsg")
    return g, int(nav[0]), int(stats[0])


def knn_ivf(base, pivots, nprobe, K, return_probes=False):
    """Approximate kNN graph by an inverted file over the pivot points
    base[pivots]: row i = the K nearest (FP32 key, id) among the other points
    whose cell (nearest pivot) is one of i's nprobe nearest pivots.  Returns
    (ids [n][K] uint32, dists [n][K] float32[, probes [n][nprobe]])."""
    base, pivots = _f32(base), _u32(pivots)
    n, d = base.shape
    ids = np.empty((n, K), np.uint32)
    dist = np.empty((n, K), np.float32)
    pr = np.empty((n, nprobe), np.uint32)
    _check(_get().oracle_knn_ivf(_p(base), n, d, _p(pivots), len(pivots), int(nprobe), int(K), _p(ids), _p(dist),
                                 _p(pr)), "knn_ivf")
    return (ids, dist, pr) if return_probes else (ids, dist)


def build_naive(base, knn_g, m):
    """NSG-Naive (Sec. 4.1.2): MRNG edge selection on each node's kNN list
    only, at most m edges, no navigating node, no repair.  Returns [n][m]
    uint32, sentinel padded."""
    base, knn_g = _f32(base), _u32(knn_g)
    n, d = base.shape
    g = np.empty((n, m), np.uint32)
    _check(_get().oracle_build_naive(_p(base), n, d, _p(knn_g), knn_g.shape[1], int(m), _p(g)), "build_naive")
    return g


def mrng_naive(base, prec=64):
    """Naive MRNG (Sec. 3.3).  Returns list of rows (np.uint32 arrays)."""
    base = _f32(base)
    n, d = base.shape
    out = np.empty((n, n - 1), np.uint32)
    deg = np.empty(n, np.int32)
    _check(_get().oracle_mrng_naive(_p(base), n, d, prec, _p(out), _p(deg)), "mrng_naive")
    return [out[i, :deg[i]].copy() for i in range(n)]


# --------------------------------------------------------------------------
# reduced precision (not in the paper)
# --------------------------------------------------------------------------

DTYPES = {"bf16": 1, "f16": 2, "e4m3": 3}


def _code_dtype(dt):
    return np.uint8 if dt == 3 else np.uint16


def decode(dtype, codes):
    dt = DTYPES[dtype]
    codes = np.ascontiguousarray(codes, dtype=_code_dtype(dt))
    out = np.empty(codes.shape, np.float32)
    _check(_get().oracle_decode(dt, _p(codes), codes.size, _p(out)), "decode")
    return out


def encode(dtype, x):
    dt = DTYPES[dtype]
    x = _f32(x)
    out = np.empty(x.shape, _code_dtype(dt))
    _check(_get().oracle_encode(dt, _p(x), x.size, _p(out)), "encode")
    return out


def scales(dtype, base):
    base = _f32(base)
    s = np.empty(base.shape[1], np.float32)
    _check(_get().oracle_scales(DTYPES[dtype], _p(base), base.shape[0], base.shape[1], _p(s)),
           "scales")
    return s


def quantize(dtype, base, sc):
    """Returns (codes [n][d], decoded rows fl32(s_j * dec(code)) [n][d])."""
    dt = DTYPES[dtype]
    base, sc = _f32(base), _f32(sc)
    codes = np.empty(base.shape, _code_dtype(dt))
    dec = np.empty(base.shape, np.float32)
    _check(_get().oracle_quantize(dt, _p(base), base.shape[0], base.shape[1], _p(sc), _p(codes),
                                  _p(dec)), "quantize")
    return codes, dec


def rerank(base, queries, pool_ids, k):
    base, queries, pool_ids = _f32(base), _f32(queries), _u32(pool_ids)
    nq = queries.shape[0]
    ids = np.empty((nq, k), np.uint32)
    dist = np.empty((nq, k), np.float32)
    _check(_get().oracle_rerank(_p(base), base.shape[1], _p(queries), nq, _p(pool_ids),
                                pool_ids.shape[1], int(k), _p(ids), _p(dist)), "rerank")
    return ids, dist


# --------------------------------------------------------------------------
# MLP for the learned early stop (not in the paper)
# --------------------------------------------------------------------------

def mlp_nparams(n_in, h):
    return int(_get().oracle_mlp_nparams(n_in, h))


def mlp_loss_grad(params, X, y, n_in, h):
    """FP64 forward + MSE + backward.  Returns (loss, grad, yhat)."""
    params = np.ascontiguousarray(params, np.float64)
    X = np.ascontiguousarray(X, np.float64)
    B = X.shape[0]
    yhat = np.empty(B, np.float64)
    grad = None
    yy = None
    if y is not None:
        yy = np.ascontiguousarray(y, np.float64)
        grad = np.empty_like(params)
    loss = _get().oracle_mlp_loss_grad(_p(params), n_in, h, _p(X), _p(yy), B, _p(yhat), _p(grad))
    return float(loss), grad, yhat


def adam_step(params, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place FP64 Adam step on float64 arrays."""
    for a in (params, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _check(_get().oracle_adam_step(_p(params), _p(grad), _p(m), _p(v), params.size, int(t),
                                   lr, b1, b2, eps), "adam")


FEATURE_RANKS = (1, 2, 4, 9, 14, 19, 29, 39, 59, 83)


def stop_features(pool_dist, d_start, nedges, hops):
    """Early-stop features of a search state (FP64; not in the paper, the
    library's own definition).  pool_dist: the sorted pool distances after
    `hops` expansions; d_start: distance to the start node; nedges: valid
    neighbour entries read by those expansions.  d_r is the distance at rank
    min(r, size - 1).  Returns 15 values: ln(1 + d_0), d_0 / d_9 (1 if
    d_9 = 0), ln(1 + d_start), ln(1 + d_0) - ln(1 + d_start), then
    ln(1 + d_r) - ln(1 + d_0) for r in FEATURE_RANKS, then nedges / hops."""
    import math
    d = [float(x) for x in pool_dist]
    at = lambda r: d[min(r, len(d) - 1)]
    l0 = math.log1p(at(0))
    f = [l0, at(0) / at(9) if at(9) > 0 else 1.0, math.log1p(d_start), l0 - math.log1p(d_start)]
    f += [math.log1p(at(r)) - l0 for r in FEATURE_RANKS]
    f.append(nedges / hops if hops > 0 else 0.0)
    return np.asarray(f, np.float64)


def stop_query_inputs(q, pool_dist, hops):
    """Inputs of the query form of the early stop (the library's own
    definition, FP64): the query's d values, then ln(1 + d_0), d_0 / d_9
    (1 if d_9 = 0; d_r at rank min(r, size - 1)) and the expansion count."""
    f = stop_features(pool_dist, 0.0, 0, hops)
    return np.concatenate([np.asarray(q, np.float64), [f[0], f[1], float(hops)]])


def _fp16(a):
    """Round to FP16, nearest even, through FP32 (as values held in FP32 are)."""
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float16).astype(np.float64)


def mlp_forward_fp16(params, X, n_in, h):
    """The network with FP16 inference (the early stop's query form): the
    inputs X [B][n_in] (already z-scored), the weights W1, W2, W3 and the
    hidden activations after each ReLU are rounded to FP16; every product and
    sum is taken in FP64; the biases b1, b2, b3 are used as given.  Params
    layout W1[h][n_in], b1[h], W2[h][h], b2[h], W3[h], b3.  Returns yhat [B]."""
    P = np.asarray(params, np.float64)
    o = 0
    W1 = P[o:o + h * n_in].reshape(h, n_in); o += h * n_in
    b1 = P[o:o + h]; o += h
    W2 = P[o:o + h * h].reshape(h, h); o += h * h
    b2 = P[o:o + h]; o += h
    W3 = P[o:o + h]; o += h
    b3 = P[o]
    x = _fp16(np.atleast_2d(X))
    a1 = _fp16(np.maximum(x @ _fp16(W1).T + b1, 0.0))
    a2 = _fp16(np.maximum(a1 @ _fp16(W2).T + b2, 0.0))
    return a2 @ _fp16(W3) + b3


def recall_at_k(found_ids, gt_ids, k):
    """precision(R') = |R' ∩ R| / K (Sec. 2.1 Eq. 1), per query; padding is a miss."""
    found_ids = np.asarray(found_ids)[:, :k]
    gt_ids = np.asarray(gt_ids)[:, :k]
    out = np.empty(found_ids.shape[0])
    for i in range(found_ids.shape[0]):
        f = set(int(x) for x in found_ids[i] if int(x) != SENT)
        out[i] = len(f & set(int(x) for x in gt_ids[i])) / k
    return out
