"""Pins of the oracle's NSG build (Algorithm 2) and naive MRNG (Sec. 3.3)
against the MRNG definition, Theorems 1 and 3, and the construction
guarantees (degree bound, reachability from the navigating node)."""
import numpy as np
import pytest

import oracle

SENT = oracle.SENT


def _reachable(G, root):
    n = G.shape[0]
    seen = np.zeros(n, bool)
    seen[root] = True
    stack = [root]
    while stack:
        v = stack.pop()
        for u in G[v]:
            if u == SENT:
                break
            if not seen[u]:
                seen[u] = True
                stack.append(int(u))
    return seen


def _mrng_definition_holds(X, rows):
    """Def. MRNG with open lunes, FP64: p->q is an edge iff no r with
    delta(p,r) < delta(p,q) and delta(q,r) < delta(p,q) has p->r an edge."""
    Xd = X.astype(np.float64)
    D = ((Xd[:, None] - Xd[None]) ** 2).sum(-1)
    n = X.shape[0]
    for p in range(n):
        edges = set(int(u) for u in rows[p])
        for q in range(n):
            if q == p:
                continue
            lune = [r for r in range(n) if r not in (p, q) and D[p, r] < D[p, q] and D[q, r] < D[p, q]]
            should = all(r not in edges for r in lune)
            if should != (q in edges):
                return False
    return True


@pytest.mark.parametrize("d", [2, 3, 8])
def test_naive_mrng_satisfies_definition(d):
    rng = np.random.default_rng(10 + d)
    X = rng.normal(size=(70, d)).astype(np.float32)
    rows = oracle.mrng_naive(X, prec=64)
    assert _mrng_definition_holds(X, rows)


@pytest.mark.parametrize("d", [2, 3, 8])
def test_mrng_nng_subset_and_60_degrees(d):
    rng = np.random.default_rng(20 + d)
    X = rng.normal(size=(80, d)).astype(np.float32)
    rows = oracle.mrng_naive(X, prec=64)
    Xd = X.astype(np.float64)
    D = ((Xd[:, None] - Xd[None]) ** 2).sum(-1)
    np.fill_diagonal(D, np.inf)
    for p in range(80):
        assert int(np.argmin(D[p])) in set(rows[p].tolist())          # NNG in MRNG
        r = rows[p]
        for i in range(len(r)):                                       # Lemma 2: angle >= 60 deg
            for j in range(i + 1, len(r)):
                a, b = Xd[r[i]] - Xd[p], Xd[r[j]] - Xd[p]
                cos = a @ b / np.sqrt((a @ a) * (b @ b))
                assert cos <= 0.5 + 1e-9


@pytest.mark.parametrize("d", [2, 3, 8])
def test_theorem_1_and_3_greedy_reaches_every_node(d):
    """An MRNG is an MSNET (Thm 3), on which Algorithm 1 with l=1 reaches any
    q in S from any start (Thm 1)."""
    rng = np.random.default_rng(30 + d)
    n = 60
    X = rng.normal(size=(n, d)).astype(np.float32)
    rows = oracle.mrng_naive(X, prec=64)
    G = np.full((n, n - 1), SENT, np.uint32)
    for v in range(n):
        G[v, :len(rows[v])] = rows[v]
    for p in range(n):
        ids, dist, _, _ = oracle.search(X, G, p, X, 1, 1)
        assert (ids[:, 0] == np.arange(n)).all()
        assert (dist[:, 0] == 0).all()


def test_select_with_all_candidates_is_naive_mrng():
    """Step (iii) with E = S minus v, no cap C and m = n-1 reproduces the naive
    MRNG row exactly (same FP32 distances)."""
    rng = np.random.default_rng(5)
    n, d = 50, 4
    X = rng.normal(size=(n, d)).astype(np.float32)
    full = oracle.knn_graph(X, n - 1)           # every other node, (dist, id) ordered
    rows = oracle.mrng_naive(X, prec=32)
    for v in range(n):
        row = oracle.collect_select(X, full, 0, 5, 0, n - 1, v)
        assert row.tolist() == rows[v].tolist()


def test_navigating_node_is_centroid_nn_when_pool_covers_all():
    rng = np.random.default_rng(6)
    X = rng.normal(size=(200, 6)).astype(np.float32)
    knn = oracle.knn_graph(X, 10)
    c = oracle.centroid(X)
    np.testing.assert_allclose(c, X.astype(np.float64).mean(0), rtol=1e-6, atol=1e-7)
    nav = oracle.navigating_node(X, knn, 17, 200)
    # reachable-from-start restricted exact NN (the kNN graph may be disconnected)
    reach = _reachable(knn, 17)
    cand = np.where(reach)[0]
    dd = ((X[cand].astype(np.float64) - c.astype(np.float64)) ** 2).sum(1)
    assert nav == cand[np.argmin(dd)]


def test_build_guarantees(tiny_index):
    X, knn, G, nav = tiny_index["X"], tiny_index["knn"], tiny_index["graph"], tiny_index["nav"]
    w = tiny_index["w"]
    assert G.shape == (w.n, w.R)
    valid = G != SENT
    # valid prefix then sentinels
    assert (np.diff(valid.astype(np.int8), axis=1) <= 0).all()
    assert (G[valid] < w.n).all()
    assert all(len(set(r[r != SENT].tolist())) == int((r != SENT).sum()) for r in G)
    assert not any(v in G[v] for v in range(w.n))                     # no self loops
    assert _reachable(G, nav).all()                                   # connectivity (DFS repair)
    # NN-percentage = 100 % with an exact kNN graph: v's nearest neighbour is
    # the first candidate and is always selected (NNG in MRNG)
    assert (G[:, 0] == knn[:, 0]).all()


def test_build_rows_follow_selection_rule(tiny_index):
    """For pre-repair rows: every selected pair (r before p) satisfies
    delta(p,r) >= delta(v,p), and every rejected candidate before the row
    filled had a selected conflicting node."""
    X, knn, nav, w = tiny_index["X"], tiny_index["knn"], tiny_index["nav"], tiny_index["w"]
    rng = np.random.default_rng(0)
    for v in rng.choice(w.n, 25, replace=False):
        row = oracle.collect_select(X, knn, nav, w.Lb, w.C, w.R, int(v))
        one = oracle.search_one(X, knn, nav, X[v], w.Lb)
        cand = dict(zip(one["vis_ids"].tolist(), one["vis_dist"].tolist()))
        for u in knn[v]:
            cand.setdefault(int(u), oracle.l2sq_f32(X[v], X[u]))
        cand.pop(int(v), None)
        E = sorted(((dd, u) for u, dd in cand.items()))[:w.C]
        sel = row.tolist()
        assert sel[0] == E[0][1]
        pos = {u: i for i, (_, u) in enumerate(E)}
        assert all(pos[a] < pos[b] for a, b in zip(sel, sel[1:]))     # selection order
        last = pos[sel[-1]]
        chosen = []
        for dd, p in E[:last + 1] if len(sel) == w.R else E:
            conflict = any(oracle.l2sq_f32(X[p], X[r]) < dd for r in chosen)
            if p in sel:
                assert not conflict
                chosen.append(p)
            else:
                assert conflict
        assert chosen == sel
