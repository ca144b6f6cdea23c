"""GPU parity at the sizes the benchmark runs: the SIFT-like 1M x 128 workload
(10,000 queries; graph built on the GPU: exact 100-NN graph, Algorithm 2 with
R=50, l=40, C=500) in the launch configurations the benchmark times (the
default persistent launch and the autotuned one); the uneven-batch workload
(DEEP-like 1M x 96) through a captured HIP graph; the 960-d precision
workload (200k x 960).  The oracle's Algorithm 1 runs on a sample of the
queries over the same graph; properties that hold at any size are checked on
every query."""
import numpy as np
import pytest

import datagen
import oracle
from parity import compare
from stop_model import random_stop_model

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SAMPLE = slice(0, None, 40)   # 250 of the 10,000 test queries


def _np(t):
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def full():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_00143_amd as nsg
    dev = torch.device("cuda:0")
    w = datagen.SIFT1M_LIKE
    X = datagen.base(w)
    Q = datagen.queries(w)
    print(f"full-size fixture: {w.name}, base {X.shape}, queries {Q.shape}", flush=True)
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    knn, _ = nsg.knn_bruteforce(Xd, Xd, w.K, exclude_self=True)
    graph, nav, _ = nsg.build(Xd, knn, w.Lb, w.C, w.R, datagen.random_node(w))
    del knn
    torch.cuda.synchronize()
    G = _np(graph).view(np.uint32)
    yield dict(nsg=nsg, X=X, Q=Q, Xd=Xd, Qd=Qd, graph=graph, G=G, nav=nav)


def _properties(ids, dist):
    """Every row sorted by (distance, id), no repeated id, padding last."""
    ids = ids.astype(np.int64)
    for i in range(ids.shape[0]):
        row = ids[i][ids[i] != 0xFFFFFFFF]
        d = dist[i][:len(row)]
        assert len(set(row.tolist())) == len(row), i
        keys = list(zip(d.tolist(), row.tolist()))
        assert keys == sorted(keys), i


@pytest.mark.parametrize("launch", ["default", "autotuned"])
def test_full_size_fp32_sampled_parity(full, launch):
    nsg, X, Q, G, nav = full["nsg"], full["X"], full["Q"], full["G"], full["nav"]
    ix = nsg.load_index(full["Xd"], full["graph"], nav, "f32")
    k, L = 10, 84
    if launch == "default":
        ids, dist = nsg.search(ix, full["Qd"], k, L)
    else:
        opts, _ = nsg.autotune(ix, full["Qd"], k, L)
        ids, dist = nsg.search_batched(ix, full["Qd"], k_scalar=k, L_scalar=L, opts=opts)
    ids, dist = _np(ids).view(np.uint32), _np(dist)
    _properties(ids, dist)
    o_ids, _, _, _ = oracle.search(X, G, nav, Q[SAMPLE], k, L, threads=16)
    r = compare(X, Q[SAMPLE], ids[SAMPLE], dist[SAMPLE], o_ids)
    assert r["ok"], {a: b for a, b in r.items() if a != "bad"}
    ix.close()


def test_full_size_fp32_k100_large_pool(full):
    """k = 100 at L = 300 (the sweep's large end), sampled."""
    nsg, X, Q, G, nav = full["nsg"], full["X"], full["Q"], full["G"], full["nav"]
    ix = nsg.load_index(full["Xd"], full["graph"], nav, "f32")
    ids, dist = nsg.search(ix, full["Qd"], 100, 300)
    ids, dist = _np(ids).view(np.uint32), _np(dist)
    _properties(ids, dist)
    s = slice(0, None, 160)
    o_ids, _, _, _ = oracle.search(X, G, nav, Q[s], 100, 300, threads=16)
    r = compare(X, Q[s], ids[s], dist[s], o_ids)
    assert r["ok"], {a: b for a, b in r.items() if a != "bad"}
    ix.close()


def test_full_size_fp16_sampled_parity(full):
    """FP16 storage: the walk equals the oracle's Algorithm 1 over the
    oracle's decoded rows; the re-ranked output equals the oracle's exact FP32
    re-rank of that pool."""
    nsg, X, Q, G, nav = full["nsg"], full["X"], full["Q"], full["G"], full["nav"]
    ix = nsg.load_index(full["Xd"], full["graph"], nav, "f16")
    k, L = 10, 84
    nq = Q.shape[0]
    dev = full["Qd"].device
    pids = torch.empty((nq, L), dtype=torch.int32, device=dev)
    pd = torch.empty((nq, L), dtype=torch.float32, device=dev)
    walk_ids, walk_d = nsg.search_batched(ix, full["Qd"], k_scalar=k, L_scalar=L,
                                          opts=dict(rerank=-1, pool_ids=pids, pool_dist=pd, pool_stride=L))
    opts, _ = nsg.autotune(ix, full["Qd"], k, L)
    ids, dist = nsg.search_batched(ix, full["Qd"], k_scalar=k, L_scalar=L, opts=opts)
    ids, dist = _np(ids).view(np.uint32), _np(dist)
    _properties(ids, dist)
    _, Xt = oracle.quantize("f16", X, oracle.scales("f16", X))
    o_ids, _, _, _, o_pids, _ = oracle.search(Xt, G, nav, Q[SAMPLE], k, L, pool_stride=L, threads=16)
    r = compare(Xt, Q[SAMPLE], _np(walk_ids).view(np.uint32)[SAMPLE], _np(walk_d)[SAMPLE], o_ids)
    assert r["ok"], {a: b for a, b in r.items() if a != "bad"}
    rr_ids, _ = oracle.rerank(X, Q[SAMPLE], o_pids, k)
    r = compare(X, Q[SAMPLE], ids[SAMPLE], dist[SAMPLE], rr_ids)
    assert r["ok"], {a: b for a, b in r.items() if a != "bad"}
    ix.close()


@pytest.mark.parametrize("L,hop", [(92, 16), (384, 32)])
def test_full_size_fp16_learned_stop_sampled_parity(full, L, hop):
    """The timed headline configuration: FP16 storage with the fused learned
    stop (the learned-stop kernel, autotuned launch, 10,000 queries) at the
    pool sizes and decision hops the benchmark uses for recall 0.95 (L = 92,
    hop 16, two 64-entry pool chunks) and 0.99 (L = 384, hop 32, six chunks).
    With the per-query budgets the kernel reports, the walk equals the
    oracle's Algorithm 1 over the decoded rows stopped after that many
    expansions, and the output equals the oracle's FP32 re-rank of that pool
    (sampled queries); every budget is a grid value at or above the hop."""
    from paper_1707_00143_amd import learned_stop as ls
    nsg, X, Q, G, nav, Qd = full["nsg"], full["X"], full["Q"], full["G"], full["nav"], full["Qd"]
    ix = nsg.load_index(full["Xd"], full["graph"], nav, "f16")
    k, nq, dev = 10, Q.shape[0], Qd.device
    P, mean, istd = random_stop_model(nsg, ix, Qd, 21, L=L, hop=hop, center=None)
    ls.install(ix, P, mean, istd, 1.0, hop=hop)
    tune, _ = nsg.autotune(ix, Qd, k, L, learned_stop=1)
    Bu = torch.zeros(nq, dtype=torch.int32, device=dev)
    ids, dist = nsg.search_batched(ix, Qd, k_scalar=k, L_scalar=L, opts=dict(tune, learned_stop=1, budget=Bu))
    Bw = torch.zeros(nq, dtype=torch.int32, device=dev)
    walk_ids, walk_d = nsg.search_batched(ix, Qd, k_scalar=k, L_scalar=L,
                                          opts=dict(tune, learned_stop=1, budget=Bw, rerank=-1))
    Bu, Bw = _np(Bu), _np(Bw)
    assert (Bu == Bw).all()
    assert set(Bu.tolist()) <= set(ls.GRID) and Bu.min() >= hop
    assert len(set(Bu.tolist())) > 3, np.unique(Bu)
    ids, dist = _np(ids).view(np.uint32), _np(dist)
    _properties(ids, dist)
    _, Xt = oracle.quantize("f16", X, oracle.scales("f16", X))
    o_ids, _, o_hops, _, o_pids, _ = oracle.search(Xt, G, nav, Q[SAMPLE], k, L, pool_stride=L,
                                                   max_hops=Bu[SAMPLE], threads=16)
    cut = (o_hops == Bu[SAMPLE]).mean()
    print(f"L={L} hop={hop}: budgets {np.unique(Bu).tolist()}; {cut * 100:.0f}% of sampled queries stopped "
          f"by their budget")
    assert 0.05 < cut < 0.95
    r = compare(Xt, Q[SAMPLE], _np(walk_ids).view(np.uint32)[SAMPLE], _np(walk_d)[SAMPLE], o_ids)
    assert r["ok"], {a: b for a, b in r.items() if a != "bad"}
    rr_ids, _ = oracle.rerank(X, Q[SAMPLE], o_pids, k)
    r = compare(X, Q[SAMPLE], ids[SAMPLE], dist[SAMPLE], rr_ids)
    assert r["ok"], {a: b for a, b in r.items() if a != "bad"}
    ix.close()


def test_full_size_ground_truth_sampled_exact(full):
    """The benchmark's ground truth (matrix-core brute force, all 10,000 test
    queries, k = 100, the launch the benchmark makes) equals the exact kNN
    definition in FP64 on 160 sampled queries: same id sets up to near-ties
    at the k-th distance, distances within 1e-5 of FP64; recall counts from
    nsg_recall_hits equal the plain count of common ids."""
    nsg, X, Q, Qd = full["nsg"], full["X"], full["Q"], full["Qd"]
    truth, tdist = nsg.knn_bruteforce(full["Xd"], Qd, 100)
    s = slice(0, None, 62)
    ids, dist = _np(truth).view(np.uint32), _np(tdist)
    o_ids, _ = oracle.knn(X, Q[s], 100)
    r = compare(X, Q[s], ids[s], dist[s], o_ids)
    assert r["ok"], {a: b for a, b in r.items() if a != "bad"}
    assert r["exact"] >= 0.99 * r["nq"]
    # recall counts of a searched result against this truth, as the benchmark forms them
    ix = nsg.load_index(full["Xd"], full["graph"], full["nav"], "f32")
    found, _ = nsg.search(ix, Qd, 10, 40)
    hits = _np(nsg.recall_hits(found.view(-1, 1, 10).contiguous(), truth, 10))[:, 0]
    want = oracle.recall_at_k(_np(found).view(np.uint32), ids, 10) * 10
    assert (hits == np.round(want).astype(np.int64)).all()
    ix.close()


def _build(nsg, X, w, dev):
    Xd = torch.from_numpy(X).to(dev)
    knn, _ = nsg.knn_bruteforce(Xd, Xd, w.K, exclude_self=True)
    graph, nav, _ = nsg.build(Xd, knn, w.Lb, w.C, w.R, datagen.random_node(w))
    del knn
    torch.cuda.synchronize()
    return Xd, graph, nav


def test_uneven_stream_batch_parity():
    """The uneven-batch workload as the benchmark serves it (DEEP-like 1M x 96,
    NSG R=32, per-query k in {1,10,100} and L in [10,500], a batch of 1000
    replayed from one captured HIP graph of the autotuned persistent launch):
    two replays equal the eager call, and every query of the batch equals the
    oracle's Algorithm 1 at its own (k, L)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_00143_amd as nsg
    dev = torch.device("cuda:0")
    w = datagen.scaled(datagen.DEEP10M_LIKE, 1_000_000, 100_000)
    X = datagen.base(w)
    Q = datagen.queries(w)[:1000]
    print(f"uneven fixture: {w.name}, base {X.shape}", flush=True)
    Xd, graph, nav = _build(nsg, X, w, dev)
    G = _np(graph).view(np.uint32)
    ix = nsg.load_index(Xd, graph, nav, "f32")
    kk, LL = datagen.uneven_kL(100_000, w.seed + 5)
    kk, LL = kk[:1000], LL[:1000]
    Qd = torch.from_numpy(Q).to(dev)
    kd, Ld = torch.from_numpy(kk).to(dev), torch.from_numpy(LL).to(dev)
    best, _ = nsg.autotune(ix, Qd, 10, 255, trials=1)
    opts = dict(best, persistent=1)
    eager = nsg.search_batched(ix, Qd, k=kd, L=Ld, L_scalar=500, out_stride=100, opts=opts)
    g = nsg.SearchGraph(ix, Qd, k=kd, L=Ld, L_scalar=500, out_stride=100, opts=opts)
    for _ in range(2):
        g.out_ids.fill_(-1)
        ids, dist = g.launch()
        torch.cuda.synchronize()
        for i in range(0, 1000, 37):
            kv = int(kk[i])
            assert torch.equal(ids[i, :kv], eager[0][i, :kv]) and torch.equal(dist[i, :kv], eager[1][i, :kv])
    ids, dist = _np(ids).view(np.uint32).copy(), _np(dist).copy()
    for i in range(1000):                   # entries past k[i] are not part of the result
        ids[i, kk[i]:] = 0xFFFFFFFF
        dist[i, kk[i]:] = np.inf
    o_ids, _, _, _ = oracle.search(X, G, nav, Q, 100, 500, k_arr=kk, L_arr=LL, threads=16)
    r = compare(X, Q, ids, dist, o_ids)
    assert r["ok"], {a: b for a, b in r.items() if a != "bad"}
    g.close()
    ix.close()


def test_uneven_stream_10M_sampled_parity():
    """The uneven-batch path at the configuration's full size (DEEP-like 10M x
    96): a batch of 1000 queries with per-query k in {1,10,100} and L in
    [10,500], replayed from a captured HIP graph of the persistent launch, on
    a seeded random 32-regular graph over all 10M rows (search parity does
    not need a good graph; this one makes every query touch rows spread over
    the whole 3.8 GB table), equals the oracle's Algorithm 1 at each query's
    (k, L) on 250 sampled queries."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_00143_amd as nsg
    dev = torch.device("cuda:0")
    w = datagen.DEEP10M_LIKE
    X = datagen.base(w)
    Q = datagen.queries(w)[:1000]
    print(f"10M uneven fixture: {w.name}, base {X.shape}", flush=True)
    n = X.shape[0]
    G = np.random.default_rng(2024).integers(0, n, size=(n, 32), dtype=np.uint32)
    nav = int(np.random.default_rng(2025).integers(0, n))
    Xd = torch.from_numpy(X).to(dev)
    ix = nsg.load_index(Xd, torch.from_numpy(G.view(np.int32)).to(dev), nav, "f32")
    kk, LL = datagen.uneven_kL(100_000, w.seed + 5)
    kk, LL = kk[:1000], LL[:1000]
    Qd = torch.from_numpy(Q).to(dev)
    kd, Ld = torch.from_numpy(kk).to(dev), torch.from_numpy(LL).to(dev)
    g = nsg.SearchGraph(ix, Qd, k=kd, L=Ld, L_scalar=500, out_stride=100, opts=dict(persistent=1))
    ids, dist = g.launch()
    torch.cuda.synchronize()
    print("10M uneven: batch searched", flush=True)
    ids, dist = _np(ids).view(np.uint32).copy(), _np(dist).copy()
    sel = np.arange(0, 1000, 4)
    for i in sel:                             # entries past k[i] are not part of the result
        ids[i, kk[i]:] = 0xFFFFFFFF
        dist[i, kk[i]:] = np.inf
    o_ids, _, _, _ = oracle.search(X, G, nav, Q[sel], 100, 500, k_arr=kk[sel], L_arr=LL[sel], threads=16)
    r = compare(X, Q[sel], ids[sel], dist[sel], o_ids)
    assert r["ok"], {a: b for a, b in r.items() if a != "bad"}
    g.close()
    ix.close()


@pytest.fixture(scope="module")
def gist():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_00143_amd as nsg
    dev = torch.device("cuda:0")
    w = datagen.scaled(datagen.GIST1M_LIKE, 200_000)
    X = datagen.base(w)
    Q = datagen.queries(w)
    print(f"precision fixture: {w.name}, base {X.shape}", flush=True)
    Xd, graph, nav = _build(nsg, X, w, dev)
    yield dict(nsg=nsg, X=X, Q=Q, Xd=Xd, Qd=torch.from_numpy(Q).to(dev), graph=graph, G=_np(graph).view(np.uint32),
               nav=nav)


@pytest.mark.parametrize("dt", ["f32", "bf16", "f16", "e4m3"])
def test_precision_workload_sampled_parity(gist, dt):
    """The 960-d precision workload at the size the benchmark reports (GIST-like
    200k x 960, NSG R=70, 1000 queries, L=250): the walk equals the oracle's
    Algorithm 1 over the oracle's decoded rows and the output equals the
    oracle's FP32 re-rank of that pool, on sampled queries."""
    nsg, X, Q, G, nav, Qd = gist["nsg"], gist["X"], gist["Q"], gist["G"], gist["nav"], gist["Qd"]
    ix = nsg.load_index(gist["Xd"], gist["graph"], nav, dt)
    k, L, nq = 10, 250, Q.shape[0]
    pids = torch.empty((nq, L), dtype=torch.int32, device=Qd.device)
    pd = torch.empty((nq, L), dtype=torch.float32, device=Qd.device)
    walk_ids, walk_d = nsg.search_batched(ix, Qd, k_scalar=k, L_scalar=L,
                                          opts=dict(rerank=-1, pool_ids=pids, pool_dist=pd, pool_stride=L))
    ids, dist = nsg.search(ix, Qd, k, L)
    ids, dist = _np(ids).view(np.uint32), _np(dist)
    _properties(ids, dist)
    s = slice(0, None, 8)
    Xt = X if dt == "f32" else oracle.quantize(dt, X, oracle.scales(dt, X))[1]
    o_ids, _, _, _, o_pids, _ = oracle.search(Xt, G, nav, Q[s], k, L, pool_stride=L, threads=16)
    r = compare(Xt, Q[s], _np(walk_ids).view(np.uint32)[s], _np(walk_d)[s], o_ids)
    assert r["ok"], {a: b for a, b in r.items() if a != "bad"}
    if dt != "f32":
        rr_ids, _ = oracle.rerank(X, Q[s], o_pids, k)
        r = compare(X, Q[s], ids[s], dist[s], rr_ids)
        assert r["ok"], {a: b for a, b in r.items() if a != "bad"}
    ix.close()


def test_precision_1M_sampled_parity():
    """The 960-d workload at the configuration's full 1M rows in every storage
    format, on a seeded random 70-regular graph (search parity does not need
    a good graph): the walk equals the oracle's Algorithm 1 over the oracle's
    decoded rows and the output the oracle's FP32 re-rank of its pool, on 64
    sampled queries at L = 100."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_00143_amd as nsg
    dev = torch.device("cuda:0")
    w = datagen.GIST1M_LIKE
    X = datagen.base(w)
    Q = datagen.queries(w)[:64]
    n = X.shape[0]
    print(f"1M precision fixture: {w.name}, base {X.shape}", flush=True)
    G = np.random.default_rng(2026).integers(0, n, size=(n, 70), dtype=np.uint32)
    nav = int(np.random.default_rng(2027).integers(0, n))
    Xd = torch.from_numpy(X).to(dev)
    Gd = torch.from_numpy(G.view(np.int32)).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    k, L = 10, 100
    for dt in ("f32", "bf16", "f16", "e4m3"):
        ix = nsg.load_index(Xd, Gd, nav, dt)
        walk_ids, walk_d = nsg.search_batched(ix, Qd, k_scalar=k, L_scalar=L, opts=dict(rerank=-1))
        ids, dist = nsg.search(ix, Qd, k, L)
        ix.close()
        Xt = X if dt == "f32" else oracle.quantize(dt, X, oracle.scales(dt, X))[1]
        o_ids, _, _, _, o_pids, _ = oracle.search(Xt, G, nav, Q, k, L, pool_stride=L, threads=16)
        r = compare(Xt, Q, _np(walk_ids).view(np.uint32), _np(walk_d), o_ids)
        assert r["ok"], (dt, {a: b for a, b in r.items() if a != "bad"})
        if dt != "f32":
            rr_ids, _ = oracle.rerank(X, Q, o_pids, k)
            r = compare(X, Q, _np(ids).view(np.uint32), _np(dist), rr_ids)
            assert r["ok"], (dt, {a: b for a, b in r.items() if a != "bad"})
        print(f"1M precision parity: {dt} ok", flush=True)
        del Xt
