"""Pins of the oracle's kNN and Algorithm 1 against facts fixed outside the
oracle: NumPy brute force, a hand-traced example, special cases that reduce to
exact kNN, and invariants that follow from Algorithm 1's definition."""
import json
import os

import numpy as np
import pytest

import oracle

SENT = oracle.SENT
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _np_knn(X, Q, k):
    d = ((Q[:, None, :].astype(np.float64) - X[None, :, :].astype(np.float64)) ** 2).sum(-1)
    idx = np.lexsort((np.broadcast_to(np.arange(X.shape[0]), d.shape), d), axis=-1)[:, :k]
    return idx, np.take_along_axis(d, idx, 1)


def test_knn_matches_numpy_fp64():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(500, 16)).astype(np.float32)
    Q = rng.normal(size=(40, 16)).astype(np.float32)
    ids, dist = oracle.knn(X, Q, 12)
    ref_ids, ref_d = _np_knn(X, Q, 12)
    assert (ids == ref_ids).all()
    np.testing.assert_allclose(dist, ref_d, rtol=1e-12)


def test_knn_ties_ordered_by_id_and_self_exclusion():
    X = np.array([[0, 0], [1, 0], [-1, 0], [0, 1], [0, -1], [5, 5]], np.float32)
    ids, dist = oracle.knn(X, X[:1], 4)
    assert list(ids[0]) == [0, 1, 2, 3]          # self first, then the four ties by id
    ids, _ = oracle.knn(X, X, 3, prec=32, exclude_self=True)
    assert list(ids[0]) == [1, 2, 3]
    assert all(ids[i, 0] != i for i in range(6))
    ids, dist = oracle.knn(X[:2], X[:1], 4)       # fewer points than k: padding
    assert list(ids[0]) == [0, 1, SENT, SENT] and np.isinf(dist[0, 2:]).all()


def test_l2_fp32_sequential():
    a = np.array([1e8, 1.0, -1e8, 3.0], np.float32)
    b = np.zeros(4, np.float32)
    # sequential FP32: 1e16 + 1 -> 1e16, + 1e16 -> 2e16, + 9 -> 2e16 (ulp 2^31)
    s = np.float32(0)
    for t in (a - b):
        s = np.float32(s + np.float32(t * t))
    assert oracle.l2sq_f32(a, b) == s


def test_golden_hand_trace():
    g = json.load(open(os.path.join(GOLD, "search_trace_2d.json")))
    X = np.array(g["points"], np.float32)
    G = np.array(g["graph"], np.uint32)
    for c in g["cases"]:
        q = np.array([c["query"]], np.float32)
        ids, dist, hops, nd = oracle.search(X, G, c["start"], q, c["k"], c["L"])
        assert list(ids[0]) == c["ids"], c["note"]
        exp = np.array([np.inf if v == "inf" else v for v in c["dist_f64"]])
        np.testing.assert_allclose(dist[0], exp, rtol=1e-6)
        assert hops[0] == c["hops"] and nd[0] == c["ndist"]
        one = oracle.search_one(X, G, c["start"], q[0], c["L"])
        assert list(one["trace"]) == c["trace"]


@pytest.mark.parametrize("d", [2, 8, 32])
def test_exhaustive_pool_equals_exact_knn(d):
    """If L >= number of nodes reachable from the start, the pool never
    truncates and the output is exact kNN over the reachable nodes."""
    rng = np.random.default_rng(d)
    n = 300
    X = rng.normal(size=(n, d)).astype(np.float32)
    Q = rng.normal(size=(20, d)).astype(np.float32)
    # random sparse graph that is strongly connected via a ring
    G = np.full((n, 6), SENT, np.uint32)
    for v in range(n):
        nb = [(v + 1) % n] + list(rng.choice(n, 4, replace=False))
        nb = [u for u in dict.fromkeys(nb) if u != v]
        G[v, :len(nb)] = nb
    ids, dist, hops, nd = oracle.search(X, G, 7, Q, 10, n)
    gt, _ = oracle.knn(X, Q, 10, prec=32)
    assert (ids == gt).all()
    assert (nd == n).all() and (hops == n).all()


def test_complete_graph_any_L_equals_exact_knn():
    rng = np.random.default_rng(3)
    n, d = 120, 5
    X = rng.normal(size=(n, d)).astype(np.float32)
    Q = rng.normal(size=(15, d)).astype(np.float32)
    G = np.array([[u for u in range(n) if u != v] for v in range(n)], np.uint32)
    gt, _ = oracle.knn(X, Q, 8, prec=32)
    for L in (8, 9, 30):
        ids, _, _, _ = oracle.search(X, G, 0, Q, 8, L)
        assert (ids == gt).all()


def test_pool_invariant_and_warmup_invariance(tiny_index):
    """Pool = the L smallest (dist, id) keys among visited nodes after the
    last merge; and for L >= t the first t expansions do not depend on L."""
    X, G, nav, Q = tiny_index["X"], tiny_index["graph"], tiny_index["nav"], tiny_index["Q"]
    for qi in range(5):
        for L in (10, 37, 100):
            r = oracle.search_one(X, G, nav, Q[qi], L)
            keys = sorted(zip(r["vis_dist"].tolist(), r["vis_ids"].tolist()))[:L]
            assert [i for _, i in keys] == r["pool_ids"].tolist()
            assert r["pool_checked"].all()             # termination: none unchecked
        traces = [oracle.search_one(X, G, nav, Q[qi], L)["trace"][:16] for L in (16, 40, 300)]
        assert all((t == traces[0]).all() for t in traces)


def test_expansion_budget_is_a_prefix_of_the_plain_search(tiny_index):
    """A budget of B expansions (the learned early stop) is the plain search
    cut after its first B expansions: its pool is, by brute force, the L
    smallest (distance, id) keys over the start and the neighbours of the
    first B nodes of the unbounded run's expansion trace; its hop count is
    min(B, the unbounded count)."""
    X, G, nav, Q = tiny_index["X"], tiny_index["graph"], tiny_index["nav"], tiny_index["Q"]
    L, k = 40, 10
    budgets = np.array([1, 2, 5, 16, 17, 30, 60, 10_000] * 2, np.int32)
    q = Q[:len(budgets)]
    ids_b, d_b, h_b, _, pids, pd = oracle.search(X, G, nav, q, k, L, pool_stride=L, max_hops=budgets)
    for i in range(len(budgets)):
        full = oracle.search_one(X, G, nav, q[i], L)
        H = int(full["hops"])
        B = min(int(budgets[i]), H)
        assert h_b[i] == B
        seen = {int(nav)}
        for v in full["trace"][:B]:
            seen.update(int(u) for u in G[v] if u != SENT)
        ids = np.fromiter(seen, np.int64)
        dd = ((X[ids].astype(np.float64) - q[i].astype(np.float64)) ** 2).sum(1)
        order = np.lexsort((ids, dd))[:L]
        want = ids[order]
        got = pids[i][pids[i] != SENT].astype(np.int64)
        # compared as sets; FP32 and FP64 may only disagree on keys within
        # 1e-5 (relative) of the L-th distance
        dL = dd[order[-1]]
        diff = set(got.tolist()) ^ set(want.tolist())
        dmap = dict(zip(ids.tolist(), dd.tolist()))
        assert all(abs(dmap[u] - dL) <= 1e-5 * dL for u in diff), (i, diff)
        assert len(got) == len(want)
        assert np.all(np.diff(pd[i][:len(got)]) >= 0)
    # no budget (or one above the natural count) equals the plain search
    ids_p, _, h_p, _ = oracle.search(X, G, nav, q, k, L)
    big = budgets >= 10_000
    assert (ids_b[big] == ids_p[big]).all() and (h_b[big] == h_p[big]).all()


def test_per_query_k_and_L(tiny_index):
    X, G, nav, Q = tiny_index["X"], tiny_index["graph"], tiny_index["nav"], tiny_index["Q"]
    k = np.array([1, 10, 100, 10, 1], np.int32)
    L = np.array([10, 50, 20, 300, 11], np.int32)
    ids, dist, hops, _ = oracle.search(X, G, nav, Q[:5], 0, 0, k_arr=k, L_arr=L)
    for i in range(5):
        one, od, oh, _ = oracle.search(X, G, nav, Q[i:i + 1], int(k[i]), int(L[i]))
        assert (ids[i, :k[i]] == one[0]).all() and hops[i] == oh[0]
    # k=100 with L=20: only 20 results, the rest padded
    assert (ids[2, 20:100] == SENT).all() and np.isinf(dist[2, 20:100]).all()


def test_counts_distance_evaluations_and_edges_read(tiny_index):
    """The per-query counts the rooflines credit: distance evaluations =
    distinct nodes whose distance was computed (the start node plus every
    first-time neighbour of the expanded nodes), neighbour entries read =
    the valid row prefixes of the expanded nodes, both rebuilt here from the
    expansion trace and the graph."""
    X, G, nav, Q = tiny_index["X"], tiny_index["graph"], tiny_index["nav"], tiny_index["Q"]
    L, k, nq = 40, 10, 12
    ne = np.zeros(nq, np.int64)
    _, _, hops, nd = oracle.search(X, G, nav, Q[:nq], k, L, nedges=ne)
    for i in range(nq):
        tr = oracle.search_one(X, G, nav, Q[i], L)["trace"]
        assert len(tr) == hops[i]
        rows = [G[v][G[v] != SENT] for v in tr]
        assert ne[i] == sum(len(r) for r in rows)
        assert nd[i] == len({int(nav)} | {int(u) for r in rows for u in r})
