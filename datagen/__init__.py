"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no arithmetic of the search method: it only draws vectors.
Both the CPU oracle tests and the GPU path take their inputs from here.

The paper's data sets (SIFT1M, GIST1M, DEEP, Sec. 4.1.1 Table 1 and Sec. 4.2)
are not available; these Gaussian mixtures stand in for them with the same
shapes and value ranges (SIFT-like 128-d values in [0, 255]; GIST-like 960-d;
DEEP-like unit-normalised 96-d).  Generation is NumPy PCG64 in FP64, cast to
FP32.  Components are picked uniformly.  Queries are fresh draws from the same
mixture (seed + 1 for test queries, seed + 2 for training queries).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int
    d: int
    n_query: int
    n_comp: int
    seed: int
    kind: str          # "iso" | "latent_clip" | "aniso_clip" | "norm_scaled" | "norm_scaled_latent" | "unit" | "unit_latent"
    # index parameters (Algorithm 2: K of the kNN graph, l = Lb, m = R, cap C)
    K: int = 100
    R: int = 50
    Lb: int = 40
    C: int = 500


# Tiny: 10k x 128, 100-component isotropic mixture, means U[0,100], sigma U[2,8].
TINY = Workload("tiny_10k_128", 10_000, 128, 100, 100, 1, "iso", K=100, R=50, Lb=40, C=500)
# SIFT-like: 1M x 128, 1000-component anisotropic mixture, per-dim sigma U[1,10],
# clipped to [0,255].  The component means lie on a 10-dimensional linear
# latent (128 + 5 * W z, z ~ N(0, I_10), W ~ N(0, 1/10)), so neighbouring
# components overlap and the data form one connected cloud of low intrinsic
# dimension, as descriptor data do.  (Means drawn independently U[0,255] give
# 1000 isolated islands: the exact 100-NN graph then has no edge between
# islands and a greedy search cannot cross them.)
SIFT1M_LIKE = Workload("sift1m_like_1M_128", 1_000_000, 128, 10_000, 1000, 2, "latent_clip",
                       K=100, R=50, Lb=40, C=500)
# the literal reading with independent U[0,255] means (kept for reference)
SIFT1M_ISLANDS = Workload("sift1m_islands_1M_128", 1_000_000, 128, 10_000, 1000, 2, "aniso_clip",
                          K=100, R=50, Lb=40, C=500)
# GIST-like: 1M x 960, 500 components, L2-normalised then scaled by U[0.5, 2]
# per vector.  The component means and the within-component spread live on a
# 32-dimensional linear latent (GIST1M's local intrinsic dimension is 29.1,
# Table 1), plus isotropic noise 0.1 in all 960 dimensions.  (Components
# isotropic in all 960 dimensions, kept as GIST1M_ISO, have an intrinsic
# dimension near 960.)
GIST1M_LIKE = Workload("gist1m_like_1M_960", 1_000_000, 960, 1_000, 500, 3, "norm_scaled_latent",
                       K=100, R=70, Lb=40, C=500)
GIST1M_ISO = Workload("gist1m_iso_1M_960", 1_000_000, 960, 1_000, 500, 3, "norm_scaled",
                       K=100, R=70, Lb=40, C=500)
# DEEP-like: 10M x 96 unit-normalised, 2000 components.  The component means
# and the within-component spread (sigma U[0.25, 1]) live on a 16-dimensional
# linear latent, plus isotropic noise 0.1 in all 96 dimensions, then each
# vector is normalised: one connected cloud of low intrinsic dimension.  With
# means drawn independently N(0, 1)^96 (kept as DEEP10M_ISLANDS) the tight
# components are isolated caps of the sphere and greedy search cannot cross
# between them (recall@10 0.46 at L = 200 on a 50k-point version, against
# 0.98 for this reading).
DEEP10M_LIKE = Workload("deep10m_like_10M_96", 10_000_000, 96, 100_000, 2000, 4, "unit_latent",
                        K=100, R=32, Lb=40, C=500)
DEEP10M_ISLANDS = Workload("deep10m_islands_10M_96", 10_000_000, 96, 100_000, 2000, 4, "unit",
                           K=100, R=32, Lb=40, C=500)


def scaled(w: Workload, n: int, n_query: int | None = None, name: str | None = None) -> Workload:
    """Same distribution, fewer points (for tests)."""
    return dataclasses.replace(w, n=n, n_query=n_query if n_query is not None else w.n_query,
                               name=name or f"{w.name}_n{n}")


def _mixture_params(w: Workload):
    rng = np.random.default_rng(w.seed)
    c, d = w.n_comp, w.d
    if w.kind == "iso":
        means = rng.uniform(0.0, 100.0, size=(c, d))
        sig = rng.uniform(2.0, 8.0, size=(c, 1)) * np.ones((1, d))
    elif w.kind == "aniso_clip":
        means = rng.uniform(0.0, 255.0, size=(c, d))
        sig = rng.uniform(1.0, 10.0, size=(c, d))
    elif w.kind == "latent_clip":
        m = 10
        W = rng.normal(0.0, 1.0 / np.sqrt(m), size=(d, m))
        z = rng.normal(0.0, 1.0, size=(c, m))
        means = 128.0 + 5.0 * (z @ W.T)
        sig = rng.uniform(1.0, 10.0, size=(c, d))
    elif w.kind in ("norm_scaled", "unit"):
        means = rng.normal(0.0, 1.0, size=(c, d))
        sig = rng.uniform(0.25, 1.0, size=(c, 1)) * np.ones((1, d))
    elif w.kind == "norm_scaled_latent":
        m = 32
        W = rng.normal(0.0, 1.0 / np.sqrt(m), size=(d, m))
        means = rng.normal(0.0, 1.0, size=(c, m))            # latent means
        sig = rng.uniform(0.25, 1.0, size=(c, 1)) * np.ones((1, m))
        return means, sig, W
    elif w.kind == "unit_latent":
        m = 16
        W = rng.normal(0.0, 1.0 / np.sqrt(m), size=(d, m))
        means = rng.normal(0.0, 1.0, size=(c, m))            # latent means
        sig = rng.uniform(0.25, 1.0, size=(c, 1)) * np.ones((1, m))
        return means, sig, W
    else:
        raise ValueError(w.kind)
    return means, sig, None


def _draw(w: Workload, count: int, stream_seed: int, chunk: int = 1 << 16) -> np.ndarray:
    means, sig, W = _mixture_params(w)
    rng = np.random.default_rng(stream_seed)
    out = np.empty((count, w.d), np.float32)
    for s in range(0, count, chunk):
        e = min(count, s + chunk)
        comp = rng.integers(0, w.n_comp, size=e - s)
        if W is not None:   # latent draw, embedded, plus isotropic noise
            z = means[comp] + sig[comp] * rng.standard_normal(size=(e - s, W.shape[1]))
            x = z @ W.T + 0.1 * rng.standard_normal(size=(e - s, w.d))
        else:
            x = means[comp] + sig[comp] * rng.standard_normal(size=(e - s, w.d))
        if w.kind in ("aniso_clip", "latent_clip"):
            np.clip(x, 0.0, 255.0, out=x)
        elif w.kind in ("norm_scaled", "norm_scaled_latent"):
            x /= np.maximum(np.linalg.norm(x, axis=1, keepdims=True), 1e-30)
            x *= rng.uniform(0.5, 2.0, size=(e - s, 1))
        elif w.kind in ("unit", "unit_latent"):
            x /= np.maximum(np.linalg.norm(x, axis=1, keepdims=True), 1e-30)
        out[s:e] = x
    return out


def base(w: Workload) -> np.ndarray:
    """[n][d] float32 base vectors."""
    return _draw(w, w.n, w.seed * 1000 + 7)


def queries(w: Workload, count: int | None = None) -> np.ndarray:
    """[n_query][d] float32 test queries (stream seed + 1)."""
    return _draw(w, count if count is not None else w.n_query, (w.seed + 1) * 1000 + 7)


def train_queries(w: Workload, count: int) -> np.ndarray:
    """Training queries for the learned early stop (stream seed + 2)."""
    return _draw(w, count, (w.seed + 2) * 1000 + 7)


def random_node(w: Workload, n: int | None = None) -> int:
    """The random start node that the navigating-node search begins from."""
    rng = np.random.default_rng(w.seed * 1000 + 11)
    return int(rng.integers(0, n if n is not None else w.n))


def uneven_kL(count: int, seed: int, k_choices=(1, 10, 100), L_lo=10, L_hi=500):
    """Per-query (k, L) for the batched uneven workload: k uniform over the
    choices, L uniform integer in [L_lo, L_hi] (k > L is allowed: the result
    tail is padded)."""
    rng = np.random.default_rng(seed)
    k = rng.choice(np.asarray(k_choices, np.int32), size=count).astype(np.int32)
    L = rng.integers(L_lo, L_hi + 1, size=count).astype(np.int32)
    return k, L
