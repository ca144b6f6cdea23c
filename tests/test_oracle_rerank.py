"""Pins of the oracle's re-rank (reduced-precision extension: exact FP32
distances for every final pool entry, re-sorted by (distance, id), first k).

Integer coordinates keep every squared distance exact in FP32, so the
expected orders below are fixed by integer arithmetic alone."""
import numpy as np

import oracle

SENT = 0xFFFFFFFF


def test_rerank_hand_case_tie_and_padding():
    # 2-d points; query at the origin.  Squared distances:
    # id0 (3,4) 25, id1 (0,5) 25, id2 (1,1) 2, id3 (6,0) 36, id4 (2,0) 4
    base = np.float32([[3, 4], [0, 5], [1, 1], [6, 0], [2, 0]])
    q = np.float32([[0, 0]])
    pool = np.uint32([[3, SENT, 1, 0, 4, 2, SENT]])   # scrambled, SENT holes
    ids, dist = oracle.rerank(base, q, pool, 7)
    # ties at 25 ordered by id (0 before 1); five real entries, then padding
    assert ids[0].tolist() == [2, 4, 0, 1, 3, SENT, SENT]
    assert dist[0, :5].tolist() == [2.0, 4.0, 25.0, 25.0, 36.0]
    assert np.isinf(dist[0, 5:]).all()
    ids3, dist3 = oracle.rerank(base, q, pool, 3)
    assert ids3[0].tolist() == [2, 4, 0] and dist3[0].tolist() == [2.0, 4.0, 25.0]


def test_rerank_of_a_pool_holding_the_exact_top_k_is_the_exact_top_k():
    rng = np.random.default_rng(11)
    n, d, nq, k, stride = 400, 6, 25, 10, 40
    base = rng.integers(-20, 21, (n, d)).astype(np.float32)
    Q = rng.integers(-20, 21, (nq, d)).astype(np.float32)
    b64, q64 = base.astype(np.int64), Q.astype(np.int64)
    d2 = ((q64[:, None, :] - b64[None, :, :]) ** 2).sum(-1)          # exact integers
    order = np.lexsort((np.broadcast_to(np.arange(n), d2.shape), d2), axis=1)
    pool = np.full((nq, stride), SENT, np.uint32)
    for i in range(nq):
        others = rng.choice(order[i, k:], 20, replace=False)         # plus non-members
        members = np.concatenate([order[i, :k], others])
        rng.shuffle(members)
        pool[i, :len(members)] = members                              # rest stays padding
    ids, dist = oracle.rerank(base, Q, pool, k)
    for i in range(nq):
        assert ids[i].tolist() == order[i, :k].tolist(), i
        assert dist[i].tolist() == d2[i, order[i, :k]].astype(np.float32).tolist(), i


def test_rerank_rows_are_independent_of_stride_and_neighbours():
    # each query's row is read at its own stride offset: swapping two pool
    # rows swaps the outputs, and a query whose pool is all padding gets
    # padding only
    base = np.float32([[0, 0], [1, 0], [0, 2], [3, 0]])
    Q = np.float32([[0, 0], [3, 0], [9, 9]])
    pool = np.uint32([[1, 2, SENT, 0], [0, 3, 1, SENT], [SENT, SENT, SENT, SENT]])
    ids, dist = oracle.rerank(base, Q, pool, 2)
    assert ids.tolist() == [[0, 1], [3, 1], [SENT, SENT]]
    assert dist[:2].tolist() == [[0.0, 1.0], [0.0, 4.0]]
    ids2, _ = oracle.rerank(base, Q[[1, 0]], pool[[1, 0]], 2)
    assert ids2.tolist() == [[3, 1], [0, 1]]
