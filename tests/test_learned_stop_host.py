"""Host logic of the learned early stop (labels, pool-size pick, calibration)
on synthetic traces; no GPU needed."""
import numpy as np
import pytest

ls = pytest.importorskip("paper_1707_00143_amd.learned_stop")


def test_grid():
    g = ls.GRID
    assert g[0] == 16 and g[-1] == 512 and len(g) == 21
    assert all(b > a for a, b in zip(g, g[1:]))
    r = np.array(g[1:]) / np.array(g[:-1])
    assert np.all(np.abs(r - 2 ** 0.25) < 0.05)


def test_l_hat_picks_grid_value_at_or_above():
    g = ls.GRID
    # c * 2^y exactly on a grid value picks it; just above picks the next
    assert ls.l_hat(np.log2([64.0]), 1.0, g)[0] == 64
    assert ls.l_hat(np.log2([64.01]), 1.0, g)[0] == 76
    assert ls.l_hat(np.log2([1.0]), 1.0, g)[0] == 16             # clamp low
    assert ls.l_hat(np.log2([4000.0]), 1.0, g)[0] == 512         # clamp high
    assert ls.l_hat(np.log2([10.0]), 2.0, g)[0] == 23            # c scales
    assert ls.l_hat(np.log2([20.0]), 1.0, g, k=100)[0] == 100    # k floor
    assert np.isnan(ls.l_hat(np.array([np.nan]), 1.0, g)[0])


def test_labels_smallest_exact_L_and_censoring():
    tr = ls.Traces(features=None, hits=None, grid=ls.GRID)

    class H:
        def __init__(self, a):
            self.a = a

        def cpu(self):
            return self

        def numpy(self):
            return self.a
    h = np.zeros((3, len(ls.GRID)), np.int32)
    h[0, 5:] = 10          # exact from the 6th grid value
    h[1, :] = 10           # exact at the first
    h[2, :] = 9            # never exact: censored at the top
    tr.hits = H(h)
    y, reached = ls.labels(tr, 10)
    np.testing.assert_allclose(y, np.log2([ls.GRID[5], ls.GRID[0], ls.GRID[-1]]))
    assert reached.tolist() == [True, True, False]


def test_calibrate_meets_target():
    rng = np.random.default_rng(0)
    nq, G = 2000, len(ls.GRID)
    need = rng.integers(0, G, nq)                                  # first exact column per query
    h = np.where(np.arange(G)[None, :] >= need[:, None], 10, 7)
    yhat = np.log2(np.asarray(ls.GRID)[need]) + rng.normal(0, 0.3, nq)
    c, rec, meanL = ls.calibrate(yhat, h, ls.GRID, 10, target=0.95)
    L = ls.l_hat(yhat, c, ls.GRID)
    col = np.searchsorted(ls.GRID, L)
    assert (h[np.arange(nq), col] / 10).mean() >= 0.95
    # the next smaller c on the ladder misses the target
    c2 = c / 2 ** (1 / 16)
    L2 = ls.l_hat(yhat, c2, ls.GRID)
    assert (h[np.arange(nq), np.searchsorted(ls.GRID, L2)] / 10).mean() < 0.95


def test_model_blob_layout():
    import torch
    n_in, h = 131, 64
    P = torch.arange(ls.HIDDEN * 0 + 12673, dtype=torch.float32)
    mean = torch.zeros(n_in)
    istd = torch.ones(n_in)
    b = ls.model_blob(P, mean, istd, ls.GRID)
    a = np.frombuffer(b, np.float32)
    assert a.size == 2 * n_in + 12673 + len(ls.GRID)
    assert a[2 * n_in] == 0 and a[2 * n_in + 12672] == 12672 and a[-1] == 512
