"""Pins of the oracle's partitioned search (one sub-NSG per subset, every
query searched in every subset, per-subset top k merged; the paper's scheme
for DEEP100M and the Taobao sets)."""
import numpy as np

import datagen
import oracle

SENT = 0xFFFFFFFF


def test_merge_hand_case_ties_and_padding():
    # two queries, three shards of two results each
    ids = np.uint32([[[4, 9], [2, SENT], [7, 1]],
                     [[SENT, SENT], [SENT, SENT], [5, SENT]]])
    dist = np.float32([[[1.0, 3.0], [2.0, np.inf], [3.0, 3.0]],
                       [[np.inf, np.inf], [np.inf, np.inf], [0.5, np.inf]]])
    i, d = oracle.merge_topk(ids, dist, 4)
    # the three results at 3.0 are ordered by id: 1, 7, 9
    assert i[0].tolist() == [4, 2, 1, 7] and d[0].tolist() == [1.0, 2.0, 3.0, 3.0]
    assert i[1].tolist() == [5, SENT, SENT, SENT] and d[1][0] == 0.5 and np.isinf(d[1][1:]).all()


def _shards(X, S, K=16, Lb=30, C=100, R=12):
    n = len(X)
    offs = np.linspace(0, n, S + 1).astype(np.int64)
    G = np.full((n, R), SENT, np.uint32)
    navs = []
    for s in range(S):
        a, b = offs[s], offs[s + 1]
        knn = oracle.knn_graph(X[a:b], K)
        g, nav, _ = oracle.build_nsg(X[a:b], knn, Lb, C, R, 0)
        G[a:b] = g
        navs.append(nav)
    return offs, G, np.array(navs)


def test_one_shard_is_the_plain_search():
    w = datagen.scaled(datagen.TINY, 1500, 20)
    X, Q = datagen.base(w), datagen.queries(w)
    offs, G, navs = _shards(X, 1)
    a, ad, _, _ = oracle.search_sharded(X, offs, G, navs, Q, 10, 25)
    b, bd, _, _ = oracle.search(X, G, int(navs[0]), Q, 10, 25)
    assert (a == b).all() and (ad == bd).all()


def test_exhaustive_pools_in_every_shard_give_exact_knn():
    """With a pool as large as every shard (each shard's search visits all of
    it, so each returns its exact top k), the merged result is the exact top
    k of the whole base: every global top-k point is in its shard's top k."""
    w = datagen.scaled(datagen.TINY, 900, 15)
    X, Q = datagen.base(w), datagen.queries(w)
    offs, G, navs = _shards(X, 3)
    k = 10
    ids, dist, sid, _ = oracle.search_sharded(X, offs, G, navs, Q, k, 300)
    gt, _ = oracle.knn(X, Q, k, prec=32)
    assert (ids == gt).all()
    # per-shard results stay inside their shard
    for s in range(3):
        v = sid[:, s][sid[:, s] != SENT].astype(np.int64)
        assert ((v >= offs[s]) & (v < offs[s + 1])).all()


def test_rerank_walk_over_exact_rows_changes_nothing():
    """Walking decoded rows that equal the FP32 rows, then re-ranking the pool
    in FP32, is the plain partitioned search (the re-rank of a pool sorted
    by the same distances keeps its first k)."""
    w = datagen.scaled(datagen.TINY, 1200, 12)
    X, Q = datagen.base(w), datagen.queries(w)
    offs, G, navs = _shards(X, 2)
    a, ad, _, _ = oracle.search_sharded(X, offs, G, navs, Q, 10, 30)
    b, bd, _, _ = oracle.search_sharded(X, offs, G, navs, Q, 10, 30, walk_rows=X.copy())
    assert (a == b).all() and (ad == bd).all()
