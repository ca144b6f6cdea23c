"""Learned early termination: traces, labels, training and calibration.

Driver around the library's kernels (an extension of the method; the paper
has no early stop).  The search keeps its pool size L and gets a per-query
expansion budget.  For every training query the plain search is run with a
budget at each value of a geometric grid (16 .. 1024 expansions in 2^(1/4)
steps); the label is log2 of the smallest budget whose top-k equals the top-k
of the unbudgeted plain search (the plain search is the reference: the label is
where the search has converged to its own answer, finite for every query).
Features are 15 scalars of the search state after the decision expansion
(16 by default; best distance, pool distance profile, distance to the start
node, neighbour entries per expansion; STOP_FEATURES in the library), the
same in every run, so one capture serves every grid point.  The network (15 -> 64 -> 64 -> 1,
ReLU) is trained with the library's forward/backward and Adam kernels on
z-scored features.  A second form takes the query itself plus three state
values (best distance, ratio of the 1st to the 10th pool distance, expansion
count; d + 3 -> 64 -> 64 -> 1) and runs with FP16 inference in the search
loop (query_inputs, kind=STOP_QUERY).  The calibration constant c is the smallest one whose
held-out mean recall meets the target when each query's budget is the grid
value at or above c * 2^y.  At search time the decision is fused into the
search loop of every query.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import (STOP_FEATURES, STOP_QUERY, STOP_SCALAR, column_stats, load_stop_model, mlp_adam, mlp_forward,
               mlp_forward_backward, recall_hits, search_batched, set_stop_checkpoints, set_stop_mode)

GRID = [int(round(16 * 2 ** (i / 4))) for i in range(25)]   # 16, 19, 23, ..., 1024 expansions
HOP = 16
HIDDEN = 64


@dataclasses.dataclass
class Traces:
    features: torch.Tensor   # [nq][STOP_FEATURES] float32 (NaN rows: search ended before the hop)
    hits: torch.Tensor       # [nq][G] int32: |top-k within budget grid[j] ∩ exact top-k|
    grid: list
    hops: torch.Tensor = None   # [nq] int64: expansions of the unbudgeted search
    same: torch.Tensor = None   # [nq][G] int32: |top-k within budget grid[j] ∩ unbudgeted top-k|


def traces(index, queries, truth, L, k=10, grid=GRID, hop=HOP, chunk=50_000):
    """Plain search at pool size L under every grid budget; features after
    expansion `hop` (captured in the run of the first budget >= hop)."""
    nq, d = queries.shape
    dev = queries.device
    feats = torch.empty((nq, STOP_FEATURES), dtype=torch.float32, device=dev)
    hits = torch.empty((nq, len(grid)), dtype=torch.int32, device=dev)
    hops = torch.empty(nq, dtype=torch.int64, device=dev)
    same = torch.empty((nq, len(grid)), dtype=torch.int32, device=dev)
    found = torch.empty((min(chunk, nq), len(grid), k), dtype=torch.int32, device=dev)
    g_feat = next((g for g, B in enumerate(grid) if B >= hop), len(grid) - 1)
    for s in range(0, nq, chunk):
        e = min(nq, s + chunk)
        q = queries[s:e]
        for g, B in enumerate(grid):
            ids = torch.empty((e - s, k), dtype=torch.int32, device=dev)
            dist = torch.empty((e - s, k), dtype=torch.float32, device=dev)
            opts = dict(max_hops=B)
            if g == g_feat:
                opts.update(features=feats[s:e], feature_hop=hop)
            search_batched(index, q, k_scalar=k, L_scalar=L, out_ids=ids, out_dist=dist, opts=opts)
            found[:e - s, g].copy_(ids)
        final, _ = search_batched(index, q, k_scalar=k, L_scalar=L, opts=dict(hops=hops[s:e]))
        hits[s:e] = recall_hits(found[:e - s].contiguous(), truth[s:e].contiguous(), k)
        same[s:e] = recall_hits(found[:e - s].contiguous(), final.contiguous(), k)
    return Traces(feats, hits, list(grid), hops, same)


def features_at(index, queries, L, hop, k=10, chunk=50_000):
    """Features after expansion `hop` of the plain search at pool size L."""
    nq = queries.shape[0]
    feats = torch.empty((nq, STOP_FEATURES), dtype=torch.float32, device=queries.device)
    for s in range(0, nq, chunk):
        e = min(nq, s + chunk)
        search_batched(index, queries[s:e], k_scalar=k, L_scalar=L,
                       opts=dict(max_hops=hop, features=feats[s:e], feature_hop=hop))
    return feats


def query_inputs(queries, features, hop=HOP):
    """Inputs of the query form: the query's d values, ln(1 + d_0), d_0 / d_9
    (features 0 and 1 of the capture) and the expansion count at the decision
    (the decision hop); NaN rows (search ended before the hop) stay NaN."""
    nq = queries.shape[0]
    h = torch.full((nq, 1), float(hop), dtype=torch.float32, device=queries.device)
    X = torch.cat([queries.float(), features[:, :2], h], 1)
    X[torch.isnan(features[:, 0])] = float("nan")
    return X.contiguous()


def labels(tr: Traces, k=10):
    """y = log2 of the smallest grid budget whose top-k is the unbudgeted
    search's (censored at the top of the grid if none is); also returns
    which queries reach it."""
    h = tr.same.cpu().numpy()
    ok = h >= k
    first = np.where(ok.any(1), ok.argmax(1), len(tr.grid) - 1)
    B = np.asarray(tr.grid)[first]
    return np.log2(B).astype(np.float32), ok.any(1)


def init_params(n_in, h, seed):
    """He-uniform weights, zero biases (layout W1, b1, W2, b2, W3, b3)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((n_in, h), (h, h), (h, 1)):
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def train(features, y, seed=0, epochs=30, batch=1024, lr=1e-3, min_steps=3000, log=None):
    """Adam on MSE of standardised targets (at least `min_steps` steps); the
    target scale and offset are folded into the output layer afterwards.
    Returns (params, mean, inv_std) as device tensors."""
    dev = features.device
    keep = ~torch.isnan(features).any(1)
    X = features[keep].contiguous()
    y = np.asarray(y, np.float32)[keep.cpu().numpy()]
    mu_y, sd_y = float(y.mean()), float(y.std()) or 1.0
    yy = torch.from_numpy((y - mu_y) / sd_y).to(dev).contiguous()
    n, n_in = X.shape
    batch = min(batch, n)
    epochs = max(epochs, -(-min_steps // max(1, n // batch)))
    mean, istd = column_stats(X)
    Xz = ((X - mean) * istd).contiguous()
    P = torch.from_numpy(init_params(n_in, HIDDEN, seed)).to(dev)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    grad = torch.empty_like(P)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(seed + 1)
    t = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(dev)
        Xp = Xz.index_select(0, perm)
        yp = yy.index_select(0, perm)
        tot = 0.0
        nb = 0
        for s in range(0, n - batch + 1, batch):
            t += 1
            mlp_forward_backward(P, n_in, HIDDEN, Xp[s:s + batch], yp[s:s + batch], grad=grad, loss=loss)
            mlp_adam(P, grad, m, v, t, lr=lr)
            if log is not None and s == 0:
                tot += float(loss.item())
                nb += 1
        if log is not None:
            log(f"  epoch {ep}: loss {tot / max(nb, 1):.4f}")
    # fold the target standardisation into W3, b3 (the last HIDDEN + 1 values)
    P[-(HIDDEN + 1):-1] *= sd_y
    P[-1] = P[-1] * sd_y + mu_y
    return P, mean, istd


def predict(P, mean, istd, features):
    Xz = ((features - mean) * istd).contiguous()
    Xz = torch.nan_to_num(Xz, nan=0.0)
    return mlp_forward(P, Xz.shape[1], HIDDEN, Xz)


def budget(yhat, c, grid, hop=HOP):
    """Expansion budget the kernel picks: smallest grid value >= c * 2^y (the
    largest if none is), at least the decision hop; NaN for a non-finite y."""
    t = c * np.exp2(np.asarray(yhat, np.float64))
    g = np.asarray(grid, np.float64)
    idx = np.searchsorted(g, t, side="left")
    idx = np.clip(idx, 0, len(g) - 1)
    B = np.maximum(g[idx], hop)
    return np.where(np.isfinite(t), B, np.nan)


def calibrate(yhat, hits, grid, k=10, target=0.95, margin=0.0, hops=None, hop=HOP):
    """Smallest c (on a 2^(1/16) ladder) whose mean held-out recall >= target
    when the decision is taken after expansion `hop`.  Returns (c, recall,
    mean budget, mean expansions) (the last needs `hops`, the unbudgeted
    expansion counts), or None."""
    yhat = np.asarray(yhat)
    h = np.asarray(hits)
    g = np.asarray(grid)
    for j in range(-64, 129):
        c = 2.0 ** (j / 16)
        B = budget(yhat, c, grid, hop)
        col = np.clip(np.searchsorted(g, B), 0, len(g) - 1)
        rec = h[np.arange(len(h)), col] / k
        if rec.mean() >= target + margin:
            used = float(np.minimum(B, hops).mean()) if hops is not None else float("nan")
            return c, float(rec.mean()), float(B.mean()), used
    return None


def budget_checkpoints(yhats, valid, c, grid, cps, hops):
    """Final budget per query with decisions at several checkpoints, as the
    kernel takes them: at checkpoint j a query that reaches expansion cps[j]
    (its unbudgeted search runs that far, valid[j]) and whose budget so far
    exceeds cps[j] (always true at the first) gets max(cps[j], grid pick of
    c * 2^yhats[j]) (no budget for a non-finite output).  inf = no budget."""
    n = len(hops)
    B = np.full(n, np.inf)
    for j, (cp, yh, ok) in enumerate(zip(cps, yhats, valid)):
        run = ok & (np.asarray(hops) >= cp)
        if j > 0:
            run &= B > cp
        Bj = budget(yh, c, grid, cp)
        B = np.where(run, np.where(np.isfinite(Bj), Bj, np.inf), B)
    return B


def calibrate_checkpoints(yhats, valid, hits, grid, cps, hops, k=10, target=0.95, margin=0.0):
    """Smallest c on the 2^(1/16) ladder whose mean held-out recall meets
    target + margin with decisions at every checkpoint.  Returns (c, recall,
    mean budget, mean expansions) or None."""
    h = np.asarray(hits)
    g = np.asarray(grid)
    hops = np.asarray(hops)
    for j in range(-64, 129):
        c = 2.0 ** (j / 16)
        B = budget_checkpoints(yhats, valid, c, grid, cps, hops)
        col = np.clip(np.searchsorted(g, np.where(np.isfinite(B), B, g[-1])), 0, len(g) - 1)
        rec = h[np.arange(len(h)), col] / k
        if rec.mean() >= target + margin:
            used = np.minimum(np.where(np.isfinite(B), B, hops), hops)
            return c, float(rec.mean()), float(np.where(np.isfinite(B), B, hops).mean()), float(used.mean())
    return None


def model_blob(P, mean, istd, grid):
    parts = [mean.cpu().numpy(), istd.cpu().numpy(), P.cpu().numpy(), np.asarray(grid, np.float32)]
    return np.concatenate([p.astype(np.float32).ravel() for p in parts]).tobytes()


def install(index, P, mean, istd, c, grid=GRID, hop=HOP, kind=STOP_SCALAR, checkpoints=None):
    n_in = mean.numel()
    load_stop_model(index, model_blob(P, mean, istd, grid), n_in, HIDDEN, hop, len(grid), kind=kind)
    if checkpoints:
        set_stop_checkpoints(index, checkpoints)
    set_stop_mode(index, True, c)
