"""Pins of the oracle's inverted-file approximate kNN graph (the replaceable
kNN-graph step of the build; the paper names nn-descent and, on the GPU for
DEEP100M, Faiss): a worked 1-D case, the exact kNN graph when every cell is
probed or there is one cell, and an independent NumPy FP64 restatement."""
import numpy as np

import datagen
import oracle

SENT = 0xFFFFFFFF


def test_worked_1d_case():
    """Points 0, 1, 2, 10, 11, 12 (ids 0..5); pivots are points 0 and 3, so
    cells {0, 1, 2} and {3, 4, 5}."""
    X = np.array([[0], [1], [2], [10], [11], [12]], np.float32)
    piv = np.array([0, 3], np.uint32)
    ids, dist, pr = oracle.knn_ivf(X, piv, 1, 2, return_probes=True)
    assert pr[:, 0].tolist() == [0, 0, 0, 1, 1, 1]
    assert ids[2].tolist() == [1, 0] and dist[2].tolist() == [1.0, 4.0]
    assert ids[4].tolist() == [3, 5]                  # equal distances: by id
    ids, dist = oracle.knn_ivf(X, piv, 1, 3)
    assert ids[0].tolist() == [1, 2, SENT] and np.isinf(dist[0, 2])   # a cell smaller than K + 1
    ids, dist = oracle.knn_ivf(X, piv, 2, 3)
    assert ids[2].tolist() == [1, 0, 3] and dist[2].tolist() == [1.0, 4.0, 64.0]


def test_all_cells_or_one_cell_is_the_exact_graph():
    w = datagen.scaled(datagen.TINY, 1500, 4)
    X = datagen.base(w)
    exact = oracle.knn_graph(X, 20)
    rng = np.random.default_rng(1)
    piv = rng.choice(len(X), 12, replace=False).astype(np.uint32)
    assert (oracle.knn_ivf(X, piv, 12, 20)[0] == exact).all()
    assert (oracle.knn_ivf(X, piv[:1], 1, 20)[0] == exact).all()


def test_matches_numpy_fp64_restatement():
    rng = np.random.default_rng(2)
    X = rng.normal(size=(2000, 16)).astype(np.float32)
    piv = rng.choice(len(X), 25, replace=False).astype(np.uint32)
    nprobe, K = 3, 10
    ids, dist, pr = oracle.knn_ivf(X, piv, nprobe, K, return_probes=True)
    X64 = X.astype(np.float64)
    dp = ((X64[:, None, :] - X64[piv][None, :, :]) ** 2).sum(-1)
    probes = np.lexsort((np.broadcast_to(np.arange(len(piv)), dp.shape), dp), axis=1)[:, :nprobe]
    cell = probes[:, 0]
    assert (pr == probes).mean() > 0.999
    differ = 0
    for i in range(len(X)):
        cand = np.where(np.isin(cell, probes[i]))[0]
        cand = cand[cand != i]
        dd = ((X64[cand] - X64[i]) ** 2).sum(1)
        order = np.lexsort((cand, dd))[:K]
        want = cand[order]
        got = ids[i]
        assert set(got.tolist()) <= set(cand.tolist()) | {SENT}
        assert np.all(np.diff(dist[i]) >= 0)
        if not (got == want).all():
            differ += 1
            # only FP32 near-ties may reorder: the K-th distances agree closely
            assert abs(dd[order][-1] - float(dist[i, -1])) <= 1e-5 * dd[order][-1]
    assert differ <= len(X) // 200
