"""GPU parity of the search path (nsg_search / nsg_search_batched) against the
CPU oracle's Algorithm 1 on the same seeded inputs and the same graph."""
import numpy as np
import pytest

import datagen
import oracle
from parity import compare

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def nsg():
    import paper_1707_00143_amd as m
    return m


@pytest.fixture(scope="module")
def tiny_gpu(tiny_index, nsg):
    dev = _dev()
    X, G, nav, Q = tiny_index["X"], tiny_index["graph"], tiny_index["nav"], tiny_index["Q"]
    Xd = torch.from_numpy(X).to(dev)
    Gd = torch.from_numpy(G.view(np.int32)).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    ix = nsg.load_index(Xd, Gd, nav)
    yield dict(ix=ix, Xd=Xd, Qd=Qd, **tiny_index)
    ix.close()


def _np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("L", [10, 20, 50, 100])
def test_search_parity_tiny(tiny_gpu, nsg, L):
    """FP32 parity on the tiny workload: id sets, distances within 1e-5 of FP64,
    identical hop counts on matching queries."""
    t = tiny_gpu
    k = 10
    hops = torch.zeros(len(t["Q"]), dtype=torch.int64, device=t["Qd"].device)
    nd = torch.zeros_like(hops)
    ids, dist = nsg.search_batched(t["ix"], t["Qd"], k_scalar=k, L_scalar=L,
                                   opts=dict(hops=hops, ndist=nd))
    o_ids, o_dist, o_h, o_nd = oracle.search(t["X"], t["graph"], t["nav"], t["Q"], k, L)
    r = compare(t["X"], t["Q"], _np(ids).view(np.uint32), _np(dist), o_ids, o_dist,
                gpu_hops=_np(hops), ora_hops=o_h)
    print(L, {k_: v for k_, v in r.items() if k_ != "bad"}, r["bad"][:3])
    assert r["ok"], r
    # distance evaluations: the visited filter may forget, never over-report
    assert (_np(nd) >= o_nd).all()
    # plain entry point gives the same result
    ids2, dist2 = nsg.search(t["ix"], t["Qd"], k, L)
    assert (ids2 == ids).all() and (dist2 == dist).all()


def test_search_edge_cases(tiny_gpu, nsg):
    t = tiny_gpu
    Q, Qd = t["Q"], t["Qd"]
    # k > L: padding
    ids, dist = nsg.search(t["ix"], Qd[:7], 30, 12)
    o_ids, _, _, _ = oracle.search(t["X"], t["graph"], t["nav"], Q[:7], 30, 12)
    ids = _np(ids).view(np.uint32)
    assert (ids[:, 12:] == 0xFFFFFFFF).all() and np.isinf(_np(dist)[:, 12:]).all()
    r = compare(t["X"], Q[:7], ids, _np(dist), o_ids)
    assert r["ok"], r
    # L = 1, k = 1 (greedy walk) and a ragged batch (not a multiple of the block)
    # pools of 2, 4, 6 and 8 register chunks
    for (k, L, nq) in [(1, 1, 13), (1, 512, 5), (100, 100, 33), (10, 200, 9), (10, 300, 9)]:
        ids, dist = nsg.search(t["ix"], Qd[:nq], k, L)
        o_ids, _, _, _ = oracle.search(t["X"], t["graph"], t["nav"], Q[:nq], k, L)
        r = compare(t["X"], Q[:nq], _np(ids).view(np.uint32), _np(dist), o_ids)
        assert r["ok"], (k, L, r)
    # empty batch is a no-op
    e_ids = torch.full((0, 5), 7, dtype=torch.int32, device=Qd.device)
    e_d = torch.zeros((0, 5), device=Qd.device)
    nsg.search(t["ix"], Qd[:0], 5, 10, out_ids=e_ids, out_dist=e_d)
    # bad arguments are rejected before any launch, outputs untouched
    out = torch.full((3, 5), 7, dtype=torch.int32, device=Qd.device)
    outd = torch.zeros((3, 5), device=Qd.device)
    for k, L in [(0, 10), (5, 0), (5, 513), (600, 10)]:
        with pytest.raises(nsg.NSGError):
            nsg.search(t["ix"], Qd[:3], k, L, out_ids=out, out_dist=outd)
    assert (out == 7).all()


def test_batched_uneven_and_persistent(tiny_gpu, nsg):
    """Per-query (k, L) and the persistent work-counter grid give each query
    its own plain result."""
    t = tiny_gpu
    nq = 100
    k, L = datagen.uneven_kL(nq, 123, k_choices=(1, 10, 100), L_lo=10, L_hi=300)
    kd = torch.from_numpy(k).to(t["Qd"].device)
    Ld = torch.from_numpy(L).to(t["Qd"].device)
    o_ids, o_dist, o_h, _ = oracle.search(t["X"], t["graph"], t["nav"], t["Q"][:nq], 0, 0, k_arr=k, L_arr=L)
    for persistent in (0, 1):
        hops = torch.zeros(nq, dtype=torch.int64, device=t["Qd"].device)
        ids, dist = nsg.search_batched(t["ix"], t["Qd"][:nq], k=kd, L=Ld, L_scalar=int(L.max()),
                                       out_stride=100, opts=dict(persistent=persistent, hops=hops, blocks=7))
        ids = _np(ids).view(np.uint32)
        dist = _np(dist)
        for i in range(nq):
            r = compare(t["X"], t["Q"][i:i + 1], ids[i:i + 1, :k[i]], dist[i:i + 1, :k[i]],
                        o_ids[i:i + 1, :k[i]], gpu_hops=_np(hops)[i:i + 1], ora_hops=o_h[i:i + 1])
            assert r["ok"], (persistent, i, r)


def test_out_of_range_per_query_k_and_L_are_clamped_and_counted(tiny_gpu, nsg):
    """Per-query k[i] / L[i] live on the device and are not checked on the
    host: values outside [0, out_stride] / [1, L_scalar] are clamped into
    range (the result equals the search at the clamped values) and each such
    query is counted in opts.clamped; waves_per_block above 4 is rejected."""
    t = tiny_gpu
    dev = t["Qd"].device
    nq, stride, Lmax = 12, 10, 40
    k = np.int32([10, 0, -3, 25, 10, 5, 10, 10, 10, 10, 1, 10])
    L = np.int32([40, 40, 40, 40, 0, -7, 99, 40, 20, 1, 40, 40])
    kc, Lc = np.clip(k, 0, stride), np.clip(L, 1, Lmax)
    want = int(((k != kc) | (L != Lc)).sum())
    cl = torch.zeros(1, dtype=torch.int32, device=dev)
    ids, dist = nsg.search_batched(t["ix"], t["Qd"][:nq], k=torch.from_numpy(k).to(dev),
                                   L=torch.from_numpy(L).to(dev), L_scalar=Lmax, out_stride=stride,
                                   opts=dict(clamped=cl))
    assert int(cl.item()) == want == 5
    ids = _np(ids).view(np.uint32)
    for i in range(nq):
        if kc[i] == 0:
            assert (ids[i] == 0xFFFFFFFF).all()      # k = 0 writes nothing (buffer left as filled)
            continue
        o_ids, _, _, _ = oracle.search(t["X"], t["graph"], t["nav"], t["Q"][i:i + 1], int(kc[i]), int(Lc[i]))
        r = compare(t["X"], t["Q"][i:i + 1], ids[i:i + 1, :kc[i]], _np(dist)[i:i + 1, :kc[i]], o_ids)
        assert r["ok"], (i, r)
    for bad in (5, 16):
        with pytest.raises(nsg.NSGError):
            nsg.search_batched(t["ix"], t["Qd"][:4], k_scalar=10, L_scalar=20, opts=dict(waves_per_block=bad))


def test_determinism(tiny_gpu, nsg):
    t = tiny_gpu
    a = nsg.search(t["ix"], t["Qd"], 10, 64)
    for _ in range(3):
        b = nsg.search(t["ix"], t["Qd"], 10, 64)
        assert (a[0] == b[0]).all() and (a[1] == b[1]).all()


def test_small_hash_forgets_but_results_unchanged(tiny_gpu, nsg):
    """A tiny visited filter forgets nodes: more distance evaluations, same
    results (a forgotten node is found in the pool by key or rejected)."""
    t = tiny_gpu
    nq = 50
    nd_big = torch.zeros(nq, dtype=torch.int64, device=t["Qd"].device)
    nd_small = torch.zeros_like(nd_big)
    a = nsg.search_batched(t["ix"], t["Qd"][:nq], k_scalar=10, L_scalar=100,
                           opts=dict(ndist=nd_big, hash_slots=4096))
    b = nsg.search_batched(t["ix"], t["Qd"][:nq], k_scalar=10, L_scalar=100,
                           opts=dict(ndist=nd_small, hash_slots=64))
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all()
    assert (nd_small >= nd_big).all() and (nd_small > nd_big).any()


def test_pool_output_matches_oracle_pool(tiny_gpu, nsg):
    t = tiny_gpu
    nq, L = 20, 40
    pids = torch.empty((nq, L), dtype=torch.int32, device=t["Qd"].device)
    pd = torch.empty((nq, L), dtype=torch.float32, device=t["Qd"].device)
    nsg.search_batched(t["ix"], t["Qd"][:nq], k_scalar=10, L_scalar=L,
                       opts=dict(pool_ids=pids, pool_dist=pd, pool_stride=L))
    _, _, _, _, o_pids, o_pd = oracle.search(t["X"], t["graph"], t["nav"], t["Q"][:nq], 10, L, pool_stride=L)
    r = compare(t["X"], t["Q"][:nq], _np(pids).view(np.uint32), _np(pd), o_pids)
    assert r["ok"], r


def test_graph_replay_matches_eager(tiny_gpu, nsg):
    """A batch captured as a HIP graph replays to the eager result every time,
    with eager work and synchronisation between replays, after refilling the
    bound query buffer in place."""
    t = tiny_gpu
    dev = t["Qd"].device
    nq = 64
    k, L = datagen.uneven_kL(nq, 7, k_choices=(1, 10), L_lo=10, L_hi=120)
    kd = torch.from_numpy(k).to(dev)
    Ld = torch.from_numpy(L).to(dev)
    qbuf = t["Qd"][:nq].clone()
    for persistent in (0, 1):
        g = nsg.SearchGraph(t["ix"], qbuf, k=kd, L=Ld, L_scalar=120, out_stride=10,
                            opts=dict(persistent=persistent))
        for rep in range(4):
            src = t["Qd"][(rep * 17) % 36:(rep * 17) % 36 + nq]
            qbuf.copy_(src)
            ids, dist = g.launch()
            torch.cuda.synchronize()
            e_ids, e_dist = nsg.search_batched(t["ix"], src.contiguous(), k=kd, L=Ld, L_scalar=120, out_stride=10)
            torch.cuda.synchronize()
            for i in range(nq):
                assert (ids[i, :k[i]] == e_ids[i, :k[i]]).all() and (dist[i, :k[i]] == e_dist[i, :k[i]]).all()
        g.close()


def test_autotune_returns_working_config(tiny_gpu, nsg):
    t = tiny_gpu
    best, ms = nsg.autotune(t["ix"], t["Qd"], 10, 40, trials=2)
    assert ms > 0 and best["lanes_per_row"] in (8, 16, 32, 64)
    a = nsg.search(t["ix"], t["Qd"], 10, 40)
    b = nsg.search_batched(t["ix"], t["Qd"], k_scalar=10, L_scalar=40, opts=best)
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all()


@pytest.mark.parametrize("lpr", [8, 16, 32, 64])
def test_layouts_agree(tiny_gpu, nsg, lpr):
    """Every lanes-per-row layout returns the oracle's results (summation
    order differs only within FP32 rounding)."""
    t = tiny_gpu
    ids, dist = nsg.search_batched(t["ix"], t["Qd"], k_scalar=10, L_scalar=50, opts=dict(lanes_per_row=lpr))
    o_ids, _, _, _ = oracle.search(t["X"], t["graph"], t["nav"], t["Q"], 10, 50)
    r = compare(t["X"], t["Q"], _np(ids).view(np.uint32), _np(dist), o_ids)
    assert r["ok"], r


def test_repeated_ids_and_tiny_filter_regression(tiny_gpu, nsg):
    """Rows that repeat ids, searched with a 64-slot visited filter: nodes are
    recomputed and offered twice in one merge batch; results still equal the
    oracle's (regression: a repeated key once left an unwritten pool slot)."""
    t = tiny_gpu
    G = t["graph"].copy()
    rng = np.random.default_rng(11)
    for v in range(G.shape[0]):
        row = G[v][G[v] != 0xFFFFFFFF]
        if len(row) >= 4:
            j = rng.integers(1, len(row))
            G[v, j] = row[0]                      # repeat the first id inside the row
    dev = t["Qd"].device
    ix = nsg.load_index(t["Xd"], torch.from_numpy(G.view(np.int32)).to(dev), t["nav"])
    ids, dist = nsg.search_batched(ix, t["Qd"], k_scalar=10, L_scalar=60, opts=dict(hash_slots=64))
    o_ids, _, _, _ = oracle.search(t["X"], G, t["nav"], t["Q"], 10, 60)
    r = compare(t["X"], t["Q"], _np(ids).view(np.uint32), _np(dist), o_ids)
    assert r["ok"], r
    ix.close()


@pytest.mark.parametrize("L", [200, 330, 500])
def test_large_pools_launch_invariant(tiny_gpu, nsg, L):
    """Pools held in 4, 6 and 8 register chunks: for each lanes-per-row layout,
    every visited-filter size, block shape and grid (one wave per query or the
    persistent work counter), and the counter and feature-capture variants of
    the kernel, return bit-identical ids and distances; each layout's result
    equals the oracle's Algorithm 1 (layouts differ only in FP32 summation
    order)."""
    t = tiny_gpu
    k = 50
    dev = t["Qd"].device
    nq = len(t["Q"])
    o_ids, o_dist, _, _ = oracle.search(t["X"], t["graph"], t["nav"], t["Q"], k, L)
    for lpr in (8, 16, 32):
        ref = None
        runs = [dict(hash_slots=h, waves_per_block=w, persistent=p)
                for h in (1024, 2048) for w in (1, 4) for p in (0, 1)]
        runs += [dict(hops=torch.zeros(nq, dtype=torch.int64, device=dev)),
                 dict(features=torch.empty((nq, nsg.STOP_FEATURES), dtype=torch.float32, device=dev),
                      feature_hop=16)]
        for o in runs:
            ids, dist = nsg.search_batched(t["ix"], t["Qd"], k_scalar=k, L_scalar=L,
                                           opts=dict(o, lanes_per_row=lpr))
            if ref is None:
                ref = (ids.clone(), dist.clone())
                r = compare(t["X"], t["Q"], _np(ids).view(np.uint32), _np(dist), o_ids, o_dist)
                assert r["ok"], (L, lpr, {a: b for a, b in r.items() if a != "bad"})
            else:
                same = torch.equal(ids, ref[0]) and torch.equal(dist, ref[1])
                assert same, (L, lpr, {a: b for a, b in o.items() if not isinstance(b, torch.Tensor)})


def test_persistent_batches_on_two_streams(tiny_gpu, nsg):
    """Persistent-grid batches issued on two streams at once (each stream has
    its own work counter; the calls bring none) all equal the result of one
    call on the default stream."""
    t = tiny_gpu
    nq = 100
    Q = t["Qd"][:nq].contiguous()
    ref = nsg.search_batched(t["ix"], Q, k_scalar=10, L_scalar=60, opts=dict(persistent=1))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for rep in range(3):
        for s in streams:
            with torch.cuda.stream(s):
                outs.append(nsg.search_batched(t["ix"], Q, k_scalar=10, L_scalar=60, opts=dict(persistent=1),
                                               stream=s))
    torch.cuda.synchronize()
    for ids, dist in outs:
        assert torch.equal(ids, ref[0]) and torch.equal(dist, ref[1])


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_longest_first_changes_no_result(tiny_gpu, nsg, storage):
    """Starting the queries farthest from the navigating node first (the
    longest_first option) changes the schedule only: every query's ids,
    distances and expansion count equal those of the given order, for both
    grids, uneven k / L, a captured graph, and a batch above the sorted
    limit (which runs in the given order)."""
    t = tiny_gpu
    dev = t["Qd"].device
    ix = nsg.load_index(t["Xd"], torch.from_numpy(t["graph"].view(np.int32)).to(dev), t["nav"], storage)
    nq = 300
    Q = t["Qd"][torch.arange(nq, device=dev) % t["Qd"].shape[0]].contiguous()
    k, L = datagen.uneven_kL(nq, 5, k_choices=(1, 10), L_lo=10, L_hi=120)
    kd, Ld = torch.from_numpy(k).to(dev), torch.from_numpy(L).to(dev)
    for persistent in (0, 1):
        for wpb in (1, 2):
            res = []
            for lf in (0, 1):
                hops = torch.zeros(nq, dtype=torch.int64, device=dev)
                ids, dist = nsg.search_batched(ix, Q, k=kd, L=Ld, L_scalar=120, out_stride=10,
                                               opts=dict(persistent=persistent, waves_per_block=wpb,
                                                         longest_first=lf, hops=hops))
                res.append((ids, dist, hops))
            torch.cuda.synchronize()
            for i in range(nq):
                assert torch.equal(res[0][0][i, :k[i]], res[1][0][i, :k[i]])
                assert torch.equal(res[0][1][i, :k[i]], res[1][1][i, :k[i]])
            assert torch.equal(res[0][2], res[1][2])
    g = nsg.SearchGraph(ix, Q, k=kd, L=Ld, L_scalar=120, out_stride=10, opts=dict(persistent=1, longest_first=1))
    e_ids, e_dist = nsg.search_batched(ix, Q, k=kd, L=Ld, L_scalar=120, out_stride=10)
    for _ in range(3):
        ids, dist = g.launch()
        torch.cuda.synchronize()
        for i in range(0, nq, 7):
            assert torch.equal(ids[i, :k[i]], e_ids[i, :k[i]]) and torch.equal(dist[i, :k[i]], e_dist[i, :k[i]])
    g.close()
    big = t["Qd"][torch.arange(65_537, device=dev) % t["Qd"].shape[0]].contiguous()
    a = nsg.search_batched(ix, big, k_scalar=10, L_scalar=40, opts=dict(longest_first=1))
    b = nsg.search_batched(ix, big, k_scalar=10, L_scalar=40)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    with pytest.raises(nsg.NSGError):
        nsg.search_batched(ix, Q, k_scalar=10, L_scalar=40, opts=dict(longest_first=2))
    ix.close()


def test_graphs_in_flight_on_four_streams(tiny_gpu, nsg):
    """Four captured persistent batches (each with its own buffers and work
    counter) replayed at once on four streams, batch j on stream j mod 4,
    three rounds with fresh queries copied in on each stream: every query's
    first k[i] entries equal its eager search."""
    t = tiny_gpu
    dev = t["Qd"].device
    nq, S = 25, 4
    k, L = datagen.uneven_kL(nq * 12, 11, k_choices=(1, 10), L_lo=10, L_hi=120)
    kd_all = torch.from_numpy(k).to(dev)
    Ld_all = torch.from_numpy(L).to(dev)
    Qall = t["Qd"][torch.arange(nq * 12, device=dev) % t["Qd"].shape[0]].contiguous()
    e_ids, e_dist = nsg.search_batched(t["ix"], Qall, k=kd_all, L=Ld_all, L_scalar=120, out_stride=10)
    streams = [torch.cuda.Stream() for _ in range(S)]
    slots = []
    for _ in range(S):
        q_ = torch.empty((nq, Qall.shape[1]), dtype=torch.float32, device=dev)
        k_ = torch.empty(nq, dtype=torch.int32, device=dev)
        L_ = torch.empty(nq, dtype=torch.int32, device=dev)
        slots.append((q_, k_, L_, nsg.SearchGraph(t["ix"], q_, k=k_, L=L_, L_scalar=120, out_stride=10,
                                                  opts=dict(persistent=1))))
    out_ids = torch.full((nq * 12, 10), -1, dtype=torch.int32, device=dev)
    out_dist = torch.full((nq * 12, 10), float("inf"), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    for j in range(12):
        st = streams[j % S]
        q_, k_, L_, g = slots[j % S]
        with torch.cuda.stream(st):
            rows = slice(j * nq, (j + 1) * nq)
            q_.copy_(Qall[rows])
            k_.copy_(kd_all[rows])
            L_.copy_(Ld_all[rows])
            ids, dist = g.launch(st)
            out_ids[rows].copy_(ids)
            out_dist[rows].copy_(dist)
    torch.cuda.synchronize()
    for i in range(nq * 12):
        assert torch.equal(out_ids[i, :k[i]], e_ids[i, :k[i]]) and torch.equal(out_dist[i, :k[i]], e_dist[i, :k[i]])
    for *_, g in slots:
        g.close()


@pytest.mark.parametrize("d,R", [(1024, 128), (1, 8), (37, 128), (129, 65)])
def test_extreme_shapes_match_oracle(nsg, d, R):
    """The largest dimension and out-degree the library accepts (d = 1024,
    R = 128: a neighbour row spans two 64-lane loads), the smallest dimension,
    and ragged ones, in every storage format, on a seeded random R-regular
    graph: the walk equals the oracle's Algorithm 1 over the decoded rows and
    the re-ranked output the oracle's FP32 re-rank of its pool."""
    dev = _dev()
    rng = np.random.default_rng(d * 1000 + R)
    n, nq, k, L = 3000, 24, 10, 64
    X = (rng.normal(size=(n, d)) * 3 + 1).astype(np.float32)
    Q = (rng.normal(size=(nq, d)) * 3 + 1).astype(np.float32)
    G = rng.integers(0, n, size=(n, R), dtype=np.uint32)
    G[::7, R // 2:] = 0xFFFFFFFF                       # some short rows (sentinel tails)
    nav = 11
    Xd, Qd = torch.from_numpy(X).to(dev), torch.from_numpy(Q).to(dev)
    Gd = torch.from_numpy(G.view(np.int32)).to(dev)
    for dt in ("f32", "bf16", "f16", "e4m3"):
        ix = nsg.load_index(Xd, Gd, nav, dt)
        wi, wd = nsg.search_batched(ix, Qd, k_scalar=k, L_scalar=L, opts=dict(rerank=-1))
        ids, dist = nsg.search(ix, Qd, k, L)
        ix.close()
        Xt = X if dt == "f32" else oracle.quantize(dt, X, oracle.scales(dt, X))[1]
        o_ids, _, _, _, o_pids, _ = oracle.search(Xt, G, nav, Q, k, L, pool_stride=L)
        wids = _np(wi).view(np.uint32)
        r = compare(Xt, Q, wids, _np(wd), o_ids, rtol=1e-5 if dt == "f32" else 1.0)
        assert r["ok"], (d, R, dt, {a: b for a, b in r.items() if a != "bad"})
        if dt != "f32":
            # the walk forms q_j - s_j * code_j with one rounding (a fused
            # decode), the decoded rows round s_j * code_j first: per
            # dimension the two differ by at most |x_j| * 2^-24, so the
            # squared distance by at most 2 sum_j |q_j - x_j| |x_j| 2^-24
            # (plus the FP32 sum's own rounding, 1e-5 relative)
            Q64, X64 = Q.astype(np.float64), Xt.astype(np.float64)
            wdist = _np(wd)
            for i in range(nq):
                for j, u in enumerate(wids[i]):
                    if u == 0xFFFFFFFF:
                        continue
                    t = Q64[i] - X64[u]
                    ref = float((t * t).sum())
                    bound = 1e-5 * ref + 2.0 * float((np.abs(t) * np.abs(X64[u])).sum()) * 2.0 ** -24 * 1.01
                    assert abs(float(wdist[i, j]) - ref) <= bound, (d, R, dt, i, j, float(wdist[i, j]), ref, bound)
            rr_ids, _ = oracle.rerank(X, Q, o_pids, k)
            r = compare(X, Q, _np(ids).view(np.uint32), _np(dist), rr_ids)
            assert r["ok"], (d, R, dt, {a: b for a, b in r.items() if a != "bad"})
