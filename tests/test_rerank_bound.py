"""The bound behind the bounded re-rank of the reduced-storage search: the
kernel re-ranks only the prefix of its walk-sorted pool whose walk distance
is at most B(W, rho, E) (W the k-th walk distance, rho the relative bound of
a computed squared distance, E the index's bound on the distance shift
between a stored row and its FP32 row), and claims that this prefix always
holds the FP32 top k of the whole pool.  Checked here in FP64 on adversarial
pools: every computed distance carries the full error allowed in the
direction that hurts the claim, with ties, and with errors far larger than
FP32 rounding (so the check does not rest on the error being small)."""
import numpy as np
import pytest


def prefix_bound(W, rho, E):
    """B as the search kernel forms it (rerank_prefix in search_impl.hpp)."""
    a = np.sqrt(W / (1.0 - rho)) + E
    t = np.sqrt((1.0 + rho) / (1.0 - rho)) * a + E
    return (1.0 + rho) * t * t * (1.0 + 2.0 ** -12)


def adversarial_pool(rng, L, k, rho, E, ties):
    """Exact distances D, re-rank distances r (D^2 within rho), and walk
    distances w pushed up for the re-rank top k and down for the rest."""
    D = rng.uniform(1.0, 3.0, size=L) * rng.uniform(0.5, 50.0)
    if ties:
        D = np.round(D, 1)   # many equal exact distances
    r = D * D * (1.0 + rng.uniform(-rho, rho, size=L))
    ids = rng.permutation(L)
    order = np.lexsort((ids, r))          # re-rank order: (distance, id)
    top = np.zeros(L, bool)
    top[order[:k]] = True
    walk_root = np.where(top, D + E, np.maximum(D - E, 0.0))
    w = walk_root ** 2 * np.where(top, 1.0 + rho, 1.0 - rho)
    return w, ids, top


@pytest.mark.parametrize("rho,ties", [(1e-6, False), (1e-3, False), (3e-2, False), (1e-3, True)])
def test_prefix_holds_the_rerank_top_k(rho, ties):
    rng = np.random.default_rng(int(rho * 1e6) + ties)
    shorter = 0
    for trial in range(1500):
        L = int(rng.integers(2, 200))
        k = int(rng.integers(1, L + 1))
        E = float(rng.choice([0.0, rng.uniform(0.0, 0.2), rng.uniform(0.0, 5.0)]))
        w, ids, top = adversarial_pool(rng, L, k, rho, E, ties)
        walk = np.lexsort((ids, w))        # the pool as the walk leaves it: (walk distance, id)
        W = w[walk[k - 1]]
        B = prefix_bound(W, rho, E)
        in_prefix = w <= B
        assert in_prefix[top].all(), (trial, L, k, E)
        # the kernel re-ranks a prefix of the walk order: it is one
        m = int(in_prefix.sum())
        assert in_prefix[walk[:m]].all()
        shorter += m < L
    assert shorter > 100   # the bound does cut pools, not only keep them whole


def test_bound_is_monotone_and_exact_without_error():
    # no rounding and no storage error: the prefix is exactly the entries at
    # or below the k-th walk distance (up to the 2^-12 slack of B)
    W = np.array([1.0, 4.0, 100.0])
    assert np.allclose(prefix_bound(W, 0.0, 0.0), W * (1.0 + 2.0 ** -12))
    assert (np.diff(prefix_bound(np.linspace(0.0, 10.0, 50), 1e-4, 0.3)) > 0).all()
    assert (prefix_bound(4.0, 1e-4, np.linspace(0.0, 1.0, 20))[1:] > prefix_bound(4.0, 1e-4, 0.0)).all()
