"""Pins of the oracle pieces behind the paper's ablations (Sec. 4.1.2
NSG-Naive baseline, Sec. 4.1.3 random starts): the NSG-Naive build (MRNG
edge selection on each node's kNN list only) and Algorithm 1 started from a
given set of nodes (random initialization)."""
import numpy as np

import datagen
import oracle

SENT = 0xFFFFFFFF


def test_naive_build_with_all_candidates_is_the_naive_mrng():
    """With K = n - 1 (every other node a candidate) and no effective degree
    cap, the selection on the kNN list is the MRNG construction of Sec. 3.3."""
    rng = np.random.default_rng(5)
    X = rng.normal(size=(60, 3)).astype(np.float32)
    n = len(X)
    knn = oracle.knn_graph(X, n - 1)
    g = oracle.build_naive(X, knn, n - 1)
    ref = oracle.mrng_naive(X, prec=32)
    for v in range(n):
        row = g[v][g[v] != SENT]
        assert row.tolist() == ref[v].tolist(), v


def test_naive_build_rows_are_kNN_subsets_with_the_pairwise_rule():
    w = datagen.scaled(datagen.TINY, 800, 4)
    X = datagen.base(w)
    K, m = 30, 12
    knn = oracle.knn_graph(X, K)
    g = oracle.build_naive(X, knn, m)
    X64 = X.astype(np.float64)
    for v in range(0, len(X), 7):
        row = [int(u) for u in g[v] if u != SENT]
        assert 1 <= len(row) <= m
        assert set(row) <= set(knn[v].tolist())
        assert row[0] == knn[v][0]                       # the nearest neighbour is always kept
        for a in range(len(row)):                        # every kept pair obeys the rule
            for b in range(a):
                dvp = ((X64[v] - X64[row[a]]) ** 2).sum()
                dpr = ((X64[row[a]] - X64[row[b]]) ** 2).sum()
                assert dpr >= dvp * (1 - 1e-6)


def test_search_from_a_node_set():
    """Initial pool = a set of nodes: a one-node set is the search started
    at that node; the set of all nodes with L = n is the exact kNN; duplicate
    ids in the set count once."""
    w = datagen.scaled(datagen.TINY, 500, 6)
    X, Q = datagen.base(w), datagen.queries(w)
    knn = oracle.knn_graph(X, 16)
    G, nav, _ = oracle.build_nsg(X, knn, 30, 100, 12, 0)
    starts = np.array([[3], [77], [401], [0], [250], [499]], np.uint32)
    a, ad, ah, and_ = oracle.search(X, G, nav, Q, 10, 20, init_ids=starts)
    for i in range(len(Q)):
        b, bd, bh, bnd = oracle.search(X, G, int(starts[i, 0]), Q[i:i + 1], 10, 20)
        assert (a[i] == b[0]).all() and ah[i] == bh[0] and and_[i] == bnd[0]
    every = np.tile(np.arange(len(X), dtype=np.uint32), (len(Q), 1))
    c, _, ch, cnd = oracle.search(X, G, nav, Q, 10, len(X), init_ids=every)
    gt, _ = oracle.knn(X, Q, 10, prec=32)
    assert (c == gt).all() and (cnd == len(X)).all()
    dup = np.array([[5, 5, 9, 5, 9]] * len(Q), np.uint32)
    d1, _, _, n1 = oracle.search(X, G, nav, Q, 10, 20, init_ids=dup)
    d2, _, _, n2 = oracle.search(X, G, nav, Q, 10, 20, init_ids=dup[:, [0, 2]])
    assert (d1 == d2).all() and (n1 == n2).all()
