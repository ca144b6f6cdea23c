"""GPU parity of the pieces behind the paper's ablations: the NSG-Naive build
(MRNG edge selection on each node's kNN list only, Sec. 4.1.2) and Algorithm
1 started from a set of random nodes (random initialization on NSG-Naive,
Sec. 4.1.2; random starts on NSG, Sec. 4.1.3), against the oracle."""
import numpy as np
import pytest

import oracle
from parity import compare

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SENT = 0xFFFFFFFF


@pytest.fixture(scope="module")
def nsg():
    import paper_1707_00143_amd as m
    return m


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_naive_build_matches_oracle(nsg, tiny_index):
    dev = _dev()
    X, knn = tiny_index["X"], tiny_index["knn"]
    R = tiny_index["w"].R
    g = nsg.build_naive(torch.from_numpy(X).to(dev), torch.from_numpy(knn.view(np.int32)).to(dev), R)
    g = g.cpu().numpy().view(np.uint32)
    o = oracle.build_naive(X, knn, R)
    same = np.mean([(a == b).all() for a, b in zip(g, o)])
    print("NSG-Naive rows identical to the oracle's:", same)
    assert same >= 0.99
    valid = g != SENT
    assert (np.diff(valid.astype(np.int8), axis=1) <= 0).all() and valid[:, 0].all()
    assert all(set(g[v][valid[v]].tolist()) <= set(knn[v].tolist()) for v in range(0, len(X), 97))


@pytest.mark.parametrize("graph,init_n,L", [("naive", 40, 40), ("naive", 100, 60), ("nsg", 1, 40), ("nsg", 64, 30)])
def test_search_from_random_nodes_matches_oracle(nsg, tiny_index, graph, init_n, L):
    """Each query's pool starts as its own set of random nodes (drawn on the
    host, seeded, passed to both sides)."""
    dev = _dev()
    X, knn, Q = tiny_index["X"], tiny_index["knn"], tiny_index["Q"]
    R = tiny_index["w"].R
    if graph == "naive":
        G = oracle.build_naive(X, knn, R)
        nav = 0
    else:
        G, nav = tiny_index["graph"], tiny_index["nav"]
    rng = np.random.default_rng(17 + init_n)
    init = rng.integers(0, len(X), size=(len(Q), init_n)).astype(np.uint32)
    ix = nsg.load_index(torch.from_numpy(X).to(dev), torch.from_numpy(G.view(np.int32)).to(dev), nav)
    Qd = torch.from_numpy(Q).to(dev)
    hops = torch.zeros(len(Q), dtype=torch.int64, device=dev)
    ids, dist = nsg.search_batched(ix, Qd, k_scalar=10, L_scalar=L,
                                   opts=dict(init_ids=torch.from_numpy(init.view(np.int32)).to(dev), init_n=init_n,
                                             hops=hops))
    o_ids, _, o_h, _ = oracle.search(X, G, nav, Q, 10, L, init_ids=init)
    r = compare(X, Q, ids.cpu().numpy().view(np.uint32), dist.cpu().numpy(), o_ids,
                gpu_hops=hops.cpu().numpy(), ora_hops=o_h)
    assert r["ok"], (graph, init_n, {a: b for a, b in r.items() if a != "bad"}, r["bad"][:3])
    # the same search through the plain kernel (no statistics)
    ids2, dist2 = nsg.search_batched(ix, Qd, k_scalar=10, L_scalar=L,
                                     opts=dict(init_ids=torch.from_numpy(init.view(np.int32)).to(dev), init_n=init_n))
    assert torch.equal(ids, ids2) and torch.equal(dist, dist2)
    ix.close()
