import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")


@pytest.fixture(scope="session")
def tiny_index():
    """The tiny workload (10k x 128, 100-component isotropic mixture) with its
    exact kNN graph and the oracle's NSG (R=50, Lb=40, C=500).  Cached on disk
    under tests/.cache so the CPU and GPU suites build it once."""
    import numpy as np

    import datagen
    import oracle

    w = datagen.TINY
    cache = os.path.join(ROOT, "tests", ".cache")
    os.makedirs(cache, exist_ok=True)
    f = os.path.join(cache, f"{w.name}_nsg.npz")
    X = datagen.base(w)
    Q = datagen.queries(w)
    if os.path.exists(f):
        z = np.load(f)
        return dict(w=w, X=X, Q=Q, knn=z["knn"], graph=z["graph"], nav=int(z["nav"]))
    knn = oracle.knn_graph(X, w.K)
    g, nav, _ = oracle.build_nsg(X, knn, w.Lb, w.C, w.R, datagen.random_node(w))
    tmp = f + ".tmp.npz"
    np.savez(tmp, knn=knn, graph=g, nav=np.int64(nav))
    os.replace(tmp, f)
    return dict(w=w, X=X, Q=Q, knn=knn, graph=g, nav=nav)
