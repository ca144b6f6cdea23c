"""Host logic of the learned early stop (labels, pool-size pick, calibration)
on synthetic traces; no GPU needed."""
import numpy as np
import pytest

ls = pytest.importorskip("paper_1707_00143_amd.learned_stop")


def test_grid():
    g = ls.GRID
    assert g[0] == 16 and g[-1] == 1024 and len(g) == 25
    assert all(b > a for a, b in zip(g, g[1:]))
    r = np.array(g[1:]) / np.array(g[:-1])
    assert np.all(np.abs(r - 2 ** 0.25) < 0.05)


def test_budget_picks_grid_value_at_or_above():
    g = ls.GRID
    # c * 2^y exactly on a grid value picks it; just above picks the next
    assert ls.budget(np.log2([64.0]), 1.0, g)[0] == 64
    assert ls.budget(np.log2([64.01]), 1.0, g)[0] == 76
    assert ls.budget(np.log2([1.0]), 1.0, g)[0] == 16              # at least the decision hop
    assert ls.budget(np.log2([1e6]), 1.0, g)[0] == 1024            # the largest if none is above
    assert ls.budget(np.log2([10.0]), 2.0, g)[0] == 23             # c scales
    assert ls.budget(np.log2([20.0]), 1.0, g, hop=40)[0] == 40     # decision-hop floor
    assert np.isnan(ls.budget(np.array([np.nan]), 1.0, g)[0])


def test_labels_smallest_converged_budget_and_censoring():
    """The label is the smallest budget whose top-k equals the unbudgeted
    search's own top-k (the `same` matrix), not the exact one."""

    class H:
        def __init__(self, a):
            self.a = a

        def cpu(self):
            return self

        def numpy(self):
            return self.a
    same = np.zeros((3, len(ls.GRID)), np.int32)
    same[0, 5:] = 10       # converged from the 6th grid value
    same[1, :] = 10        # converged at the first
    same[2, :] = 9         # never within the grid: censored at the top
    hits = np.zeros_like(same)   # exact recall plays no part in the label
    tr = ls.Traces(features=None, hits=H(hits), grid=ls.GRID, same=H(same))
    y, reached = ls.labels(tr, 10)
    np.testing.assert_allclose(y, np.log2([ls.GRID[5], ls.GRID[0], ls.GRID[-1]]))
    assert reached.tolist() == [True, True, False]


def test_calibrate_meets_target():
    rng = np.random.default_rng(0)
    nq, G = 2000, len(ls.GRID)
    need = rng.integers(0, G, nq)                                  # first exact column per query
    h = np.where(np.arange(G)[None, :] >= need[:, None], 10, 7)
    yhat = np.log2(np.asarray(ls.GRID)[need]) + rng.normal(0, 0.3, nq)
    hops = np.full(nq, 300)
    c, rec, meanB, used = ls.calibrate(yhat, h, ls.GRID, 10, target=0.95, hops=hops)
    B = ls.budget(yhat, c, ls.GRID)
    col = np.searchsorted(ls.GRID, B)
    assert (h[np.arange(nq), col] / 10).mean() >= 0.95
    assert abs(meanB - B.mean()) < 1e-9 and abs(used - np.minimum(B, 300).mean()) < 1e-9
    # the next smaller c on the ladder misses the target
    c2 = c / 2 ** (1 / 16)
    B2 = ls.budget(yhat, c2, ls.GRID)
    assert (h[np.arange(nq), np.searchsorted(ls.GRID, B2)] / 10).mean() < 0.95


def test_model_blob_layout():
    import torch
    n_in, h = 15, 64
    n = n_in * h + h + h * h + h + h + 1
    assert n == 5249
    P = torch.arange(n, dtype=torch.float32)
    mean = torch.zeros(n_in)
    istd = torch.ones(n_in)
    b = ls.model_blob(P, mean, istd, ls.GRID)
    a = np.frombuffer(b, np.float32)
    assert a.size == 2 * n_in + n + len(ls.GRID)
    assert a[2 * n_in] == 0 and a[2 * n_in + n - 1] == n - 1 and a[-1] == 1024
