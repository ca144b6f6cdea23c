"""GPU parity of the partitioned search (one NSG per subset of consecutive
rows, every query searched in every subset, per-subset top k merged: the
paper's scheme for DEEP100M and the Taobao sets) against the oracle's
partitioned search over the same sub-graphs."""
import numpy as np
import pytest

import datagen
import oracle
from parity import compare

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SENT = 0xFFFFFFFF


@pytest.fixture(scope="module")
def shards(tiny_index):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_00143_amd as nsg
    X = tiny_index["X"]
    n = len(X)
    offs = np.array([0, 2600, 5000, 7400, n], np.int64)        # ragged subsets
    R = 32
    G = np.full((n, R), SENT, np.uint32)
    navs = []
    for s in range(4):
        a, b = offs[s], offs[s + 1]
        knn = oracle.knn_graph(X[a:b], 50)
        g, nav, _ = oracle.build_nsg(X[a:b], knn, 40, 300, R, 0)
        G[a:b] = g
        navs.append(nav)
    dev = torch.device("cuda:0")
    Q = np.concatenate([tiny_index["Q"], datagen.train_queries(tiny_index["w"], 1900)])
    print(f"shards fixture: {X.shape} in subsets {offs.tolist()}, {len(Q)} queries", flush=True)
    yield dict(nsg=nsg, X=X, Q=Q, offs=offs, G=G, navs=np.array(navs), dev=dev,
               Xd=torch.from_numpy(X).to(dev), Gd=torch.from_numpy(G.view(np.int32)).to(dev),
               Qd=torch.from_numpy(Q).to(dev))


@pytest.mark.parametrize("dt,k,L,nq", [("f32", 10, 40, 100), ("f32", 10, 40, 2000), ("f32", 25, 8, 37),
                                       ("f16", 10, 40, 2000), ("e4m3", 10, 60, 300)])
def test_sharded_search_matches_oracle(shards, dt, k, L, nq):
    """Merged top k equals the oracle's partitioned search (each subset's walk
    over its decoded rows, its pool re-ranked in FP32 for reduced formats):
    id sets up to near-ties, distances within 1e-5 of FP64; k > L pads each
    subset's list and the merge fills from the others; 2,000 queries x 4
    subsets run on the persistent grid."""
    nsg, X, Q = shards["nsg"], shards["X"], shards["Q"][:nq]
    sh = nsg.load_shards(shards["Xd"], shards["offs"], shards["Gd"], shards["navs"], dt)
    ids, dist = nsg.search_shards(sh, shards["Qd"][:nq].contiguous(), k, L)
    ids, dist = ids.cpu().numpy().view(np.uint32), dist.cpu().numpy()
    walk = None if dt == "f32" else oracle.quantize(dt, X, oracle.scales(dt, X))[1]
    o_ids, o_d, _, _ = oracle.search_sharded(X, shards["offs"], shards["G"], shards["navs"], Q, k, L,
                                             walk_rows=walk)
    r = compare(X, Q, ids, dist, o_ids)
    assert r["ok"], (dt, k, L, {a: b for a, b in r.items() if a != "bad"}, r["bad"][:3])
    for i in range(nq):                       # sorted by (distance, id), unique, padding last
        v = ids[i][ids[i] != SENT]
        assert len(set(v.tolist())) == len(v)
        keys = list(zip(dist[i][:len(v)].tolist(), v.tolist()))
        assert keys == sorted(keys)
    sh.close()


def test_one_subset_equals_plain_search_and_bad_graphs_rejected(shards, tiny_index):
    nsg, dev = shards["nsg"], shards["dev"]
    X, G, nav = tiny_index["X"], tiny_index["graph"], tiny_index["nav"]
    Gd = torch.from_numpy(G.view(np.int32)).to(dev)
    sh = nsg.load_shards(shards["Xd"], [0, len(X)], Gd, [nav])
    ix = nsg.load_index(shards["Xd"], Gd, nav)
    a = nsg.search_shards(sh, shards["Qd"][:100].contiguous(), 10, 30)
    b = nsg.search(ix, shards["Qd"][:100].contiguous(), 10, 30)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    sh.close()
    ix.close()
    offs = shards["offs"]
    bad = shards["G"].copy()
    bad[offs[1], 0] = offs[2] - offs[1]          # a local id beyond its subset
    with pytest.raises(nsg.NSGError):
        nsg.load_shards(shards["Xd"], offs, torch.from_numpy(bad.view(np.int32)).to(dev), shards["navs"])
    navs = shards["navs"].copy()
    navs[2] = offs[3] - offs[2]                   # navigating node outside its subset
    with pytest.raises(nsg.NSGError):
        nsg.load_shards(shards["Xd"], offs, shards["Gd"], navs)
