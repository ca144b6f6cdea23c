"""nsg_search_noalloc (no device allocation; scratch in a library-held
device array) against nsg_search on the same index and queries: two calls in
a row, the second with a smaller batch, both large enough for the persistent
grid that uses the scratch counter; outputs equal nsg_search's bit for bit
and meet the oracle parity criterion on sampled queries."""
import numpy as np
import pytest

import datagen
import oracle
from parity import compare

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_noalloc_search_equals_search_on_two_calls(tiny_index):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_00143_amd as nsg
    dev = torch.device("cuda:0")
    X, G, nav = tiny_index["X"], tiny_index["graph"], tiny_index["nav"]
    Q = datagen.train_queries(tiny_index["w"], 9000)
    print(f"no-alloc search: tiny index {X.shape}, batches 9000 then 5000, k=10, L=40", flush=True)
    ix = nsg.load_index(torch.from_numpy(X).to(dev), torch.from_numpy(G.view(np.int32)).to(dev), nav, "f32")
    Qd = torch.from_numpy(Q).to(dev)
    k, L = 10, 40
    for nq in (9000, 5000):
        q = Qd[:nq].contiguous()
        ref_i, ref_d = nsg.search(ix, q, k, L)
        ids = torch.full((nq, k), 7, dtype=torch.int32, device=dev)
        dist = torch.full((nq, k), -1.0, dtype=torch.float32, device=dev)
        nsg.search_noalloc(ix, q, k, L, ids, dist)
        torch.cuda.synchronize()
        assert torch.equal(ids, ref_i) and torch.equal(dist, ref_d), nq
        s = slice(0, None, 60)
        o_ids, _, _, _ = oracle.search(X, G, nav, Q[:nq][s], k, L)
        r = compare(X, Q[:nq][s], ids.cpu().numpy().view(np.uint32)[s], dist.cpu().numpy()[s], o_ids)
        assert r["ok"], (nq, {a: b for a, b in r.items() if a != "bad"})
    ix.close()
