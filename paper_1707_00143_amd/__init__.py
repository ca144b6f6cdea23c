"""MI355X (gfx950) search on a Navigating Spreading-out Graph.

Thin ctypes binding over ``libnsg.so`` (declared in ``include/nsg.h``).  Each
function here is the C entry point of the same name without the ``nsg_``
prefix; it only checks tensor placement/dtype, passes device pointers and the
current HIP stream, and raises ``NSGError`` with the library's message on a
non-zero status.  Every step of the computation runs in the library's HIP
kernels.  There is no CPU fallback: importing this package without the built
library raises.

Conventions: ids are ``torch.int32`` tensors holding the library's uint32 ids
(the sentinel 0xFFFFFFFF reads as -1); distances are squared l2 in FP32.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnsg.so")
SENT = -1  # 0xFFFFFFFF as int32

F32, BF16, F16, E4M3 = 0, 1, 2, 3
DTYPES = {"f32": F32, "bf16": BF16, "f16": F16, "e4m3": E4M3}


class NSGError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


STOP_FEATURES = 15   # early-stop features per query (see nsg.h)
STOP_SCALAR = 0      # network forms of the early stop (see nsg.h)
STOP_QUERY = 1


class SearchOpts(ctypes.Structure):
    _fields_ = [
        ("persistent", ctypes.c_int32),
        ("waves_per_block", ctypes.c_int32),
        ("hash_slots", ctypes.c_int32),
        ("blocks", ctypes.c_int32),
        ("learned_stop", ctypes.c_int32),
        ("rerank", ctypes.c_int32),
        ("hops", ctypes.c_void_p),
        ("ndist", ctypes.c_void_p),
        ("budget", ctypes.c_void_p),
        ("features", ctypes.c_void_p),
        ("pool_ids", ctypes.c_void_p),
        ("pool_dist", ctypes.c_void_p),
        ("pool_stride", ctypes.c_int32),
        ("feature_hop", ctypes.c_int32),
        ("nedges", ctypes.c_void_p),
        ("lanes_per_row", ctypes.c_int32),
        ("counter", ctypes.c_void_p),
        ("max_hops", ctypes.c_int32),
        ("clamped", ctypes.c_void_p),
        ("init_ids", ctypes.c_void_p),
        ("init_n", ctypes.c_int32),
        ("longest_first", ctypes.c_int32),
        ("order_scratch", ctypes.c_void_p),
    ]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1707_00143_amd/build.py "
                          "(or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_float
    sig = {
        "nsg_last_error": (ctypes.c_char_p, []),
        "nsg_load_index": (i32, [P, i64, i32, P, i32, u32, i32, P, P, ctypes.POINTER(P)]),
        "nsg_free_index": (None, [P]),
        "nsg_index_info": (i32, [P, P, P, P, P, P]),
        "nsg_search": (i32, [P, P, i64, i32, i32, P, P, P]),
        "nsg_search_noalloc": (i32, [P, P, i64, i32, i32, P, P, P]),
        "nsg_search_batched": (i32, [P, P, i64, P, P, i32, i32, i32, P, P,
                                     ctypes.POINTER(SearchOpts), P]),
        "nsg_knn_bruteforce": (i32, [P, i64, P, i64, i32, i32, i32, P, P, P]),
        "nsg_build": (i32, [P, i64, i32, P, i32, i32, i32, i32, u32, P, P, P, P]),
        "nsg_build_naive": (i32, [P, i64, i32, P, i32, i32, P, P]),
        "nsg_load_stop_model": (i32, [P, P, ctypes.c_size_t, i32, i32, i32, i32, i32]),
        "nsg_knn_ivf": (i32, [P, i64, i32, P, i32, i32, i32, P, P, P]),
        "nsg_set_stop_checkpoints": (i32, [P, P, i32]),
        "nsg_set_stop_mode": (i32, [P, i32, f32]),
        "nsg_mlp_forward_backward": (i32, [P, i32, i32, P, P, i64, P, P, P, P]),
        "nsg_mlp_adam": (i32, [P, P, P, P, i64, i64, f32, f32, f32, f32, P]),
        "nsg_mlp_forward": (i32, [P, i32, i32, P, i64, P, P]),
        "nsg_recall_hits": (i32, [P, i64, i32, i32, P, i32, P, P]),
        "nsg_column_stats": (i32, [P, i64, i32, P, P, P]),
        "nsg_load_shards": (i32, [P, i64, i32, P, i32, P, i32, P, i32, P, P, ctypes.POINTER(P)]),
        "nsg_free_shards": (None, [P]),
        "nsg_shards_info": (i32, [P, P, P]),
        "nsg_search_shards": (i32, [P, P, i64, i32, i32, P, P, P]),
        "nsg_search_graph_create": (i32, [P, P, i64, P, P, i32, i32, i32, P, P, ctypes.POINTER(SearchOpts),
                                          ctypes.POINTER(P)]),
        "nsg_search_graph_launch": (i32, [P, P]),
        "nsg_search_graph_destroy": (None, [P]),
        "nsg_autotune": (i32, [P, P, i64, i32, i32, i32, ctypes.POINTER(SearchOpts), ctypes.POINTER(f32), P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return _load().nsg_last_error().decode()


def _call(name, *args):
    rc = getattr(_load(), name)(*args)
    if rc != 0:
        raise NSGError(name, rc, last_error())
    return rc


def _dev(t, dtype, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Index:
    """A resident index (nsg_load_index).  Keeps a handle, frees on close()."""

    def __init__(self, handle, n, d, R, nav, storage):
        self._h = handle
        self.n, self.d, self.R, self.nav, self.storage = n, d, R, nav, storage

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("index is closed")
        return self._h

    def close(self):
        if self._h is not None:
            _load().nsg_free_index(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def load_index(base, graph, nav_node, storage="f32", scales=None, stream=None) -> Index:
    """nsg_load_index: base [n][d] float32, graph [n][R] int32 (uint32 bits)."""
    n, d = base.shape
    R = graph.shape[1]
    if graph.shape[0] != n:
        raise ValueError("graph rows != base rows")
    h = ctypes.c_void_p()
    st = DTYPES[storage] if isinstance(storage, str) else int(storage)
    _call("nsg_load_index", _dev(base, torch.float32, "base"), n, d, _dev(graph, torch.int32, "graph"), R,
          int(nav_node), st, _dev(scales, torch.float32, "scales"), _stream(stream), ctypes.byref(h))
    return Index(h, n, d, R, int(nav_node), st)


def free_index(index: Index):
    index.close()


def search(index: Index, queries, k, L, out_ids=None, out_dist=None, stream=None):
    """nsg_search: returns (ids int32 [nq][k], dist float32 [nq][k])."""
    nq = queries.shape[0]
    if out_ids is None:
        out_ids = torch.empty((nq, k), dtype=torch.int32, device=queries.device)
    if out_dist is None:
        out_dist = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
    _call("nsg_search", index.handle, _dev(queries, torch.float32, "queries"), nq, int(k), int(L),
          _dev(out_ids, torch.int32, "out_ids"), _dev(out_dist, torch.float32, "out_dist"), _stream(stream))
    return out_ids, out_dist


def search_noalloc(index: Index, queries, k, L, out_ids, out_dist, stream=None):
    """nsg_search_noalloc: nsg_search into caller-allocated outputs, with no
    device allocation by the library (its work counter is a library-held
    device array shared by every call on the GPU: calls must not overlap)."""
    nq = queries.shape[0]
    _call("nsg_search_noalloc", index.handle, _dev(queries, torch.float32, "queries"), nq, int(k), int(L),
          _dev(out_ids, torch.int32, "out_ids"), _dev(out_dist, torch.float32, "out_dist"), _stream(stream))
    return out_ids, out_dist


def search_batched(index: Index, queries, k=None, L=None, k_scalar=10, L_scalar=None, out_stride=None,
                   out_ids=None, out_dist=None, opts: dict | None = None, stream=None):
    """nsg_search_batched with per-query k / L (int32 device tensors or None).
    L_scalar bounds every L[i].  opts: SearchOpts field names; tensors for the
    pointer fields."""
    nq = queries.shape[0]
    if L_scalar is None:
        raise ValueError("L_scalar (the bound of every L[i]) is required")
    if out_stride is None:
        out_stride = int(k_scalar) if k is None else int(k.max().item()) if nq else 1
    if out_ids is None:
        out_ids = torch.full((nq, out_stride), SENT, dtype=torch.int32, device=queries.device)
    if out_dist is None:
        out_dist = torch.full((nq, out_stride), float("inf"), dtype=torch.float32, device=queries.device)
    o, keep = _opts(opts)
    _call("nsg_search_batched", index.handle, _dev(queries, torch.float32, "queries"), nq,
          _dev(k, torch.int32, "k"), _dev(L, torch.int32, "L"), int(k_scalar), int(L_scalar), int(out_stride),
          _dev(out_ids, torch.int32, "out_ids"), _dev(out_dist, torch.float32, "out_dist"), ctypes.byref(o),
          _stream(stream))
    return out_ids, out_dist


class Shards:
    """A resident partitioned index (nsg_load_shards): S subsets of consecutive
    rows, one NSG each.  `index` is the underlying single index (rows and the
    graph in global ids), usable with every search entry point of one graph."""

    def __init__(self, handle, offsets, storage):
        self._h = handle
        self.offsets = list(offsets)
        self.S = len(self.offsets) - 1
        self.storage = storage

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("partitioned index is closed")
        return self._h

    def close(self):
        if self._h is not None:
            _load().nsg_free_shards(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def load_shards(base, offsets, graph, navs, storage="f32", scales=None, stream=None) -> Shards:
    """nsg_load_shards: base [n][d] float32, offsets (S + 1 ints, host), graph
    [n][R] int32 holding each subset's LOCAL ids, navs (S local ids, host)."""
    n, d = base.shape
    R = graph.shape[1]
    offs = (ctypes.c_int64 * len(offsets))(*[int(o) for o in offsets])
    S = len(offsets) - 1
    nv = (ctypes.c_uint32 * S)(*[int(v) for v in navs])
    st = DTYPES[storage] if isinstance(storage, str) else int(storage)
    h = ctypes.c_void_p()
    _call("nsg_load_shards", _dev(base, torch.float32, "base"), n, d, offs, S, _dev(graph, torch.int32, "graph"), R,
          nv, st, _dev(scales, torch.float32, "scales"), _stream(stream), ctypes.byref(h))
    return Shards(h, offsets, st)


def search_shards(shards: Shards, queries, k, L, out_ids=None, out_dist=None, stream=None):
    """nsg_search_shards: every query in every subset, merged top k (global ids)."""
    nq = queries.shape[0]
    if out_ids is None:
        out_ids = torch.empty((nq, k), dtype=torch.int32, device=queries.device)
    if out_dist is None:
        out_dist = torch.empty((nq, k), dtype=torch.float32, device=queries.device)
    _call("nsg_search_shards", shards.handle, _dev(queries, torch.float32, "queries"), nq, int(k), int(L),
          _dev(out_ids, torch.int32, "out_ids"), _dev(out_dist, torch.float32, "out_dist"), _stream(stream))
    return out_ids, out_dist


def knn_bruteforce(base, queries, k, exclude_self=False, stream=None):
    """nsg_knn_bruteforce: exact kNN, (ids int32 [nq][k], dist float32 [nq][k])."""
    n, d = base.shape
    nq = queries.shape[0]
    ids = torch.empty((nq, k), dtype=torch.int32, device=base.device)
    dist = torch.empty((nq, k), dtype=torch.float32, device=base.device)
    _call("nsg_knn_bruteforce", _dev(base, torch.float32, "base"), n, _dev(queries, torch.float32, "queries"),
          nq, d, int(k), 1 if exclude_self else 0, _dev(ids, torch.int32, "ids"),
          _dev(dist, torch.float32, "dist"), _stream(stream))
    return ids, dist


def knn_ivf(base, pivots, nprobe, K, stream=None):
    """nsg_knn_ivf: approximate kNN graph by an inverted file over the pivot
    rows base[pivots] (pivots int32 device tensor).  Returns (ids int32
    [n][K], dist float32 [n][K])."""
    n, d = base.shape
    ids = torch.empty((n, K), dtype=torch.int32, device=base.device)
    dist = torch.empty((n, K), dtype=torch.float32, device=base.device)
    _call("nsg_knn_ivf", _dev(base, torch.float32, "base"), n, d, _dev(pivots, torch.int32, "pivots"),
          int(pivots.numel()), int(nprobe), int(K), _dev(ids, torch.int32, "ids"), _dev(dist, torch.float32, "dist"),
          _stream(stream))
    return ids, dist


def build(base, knn, Lb, C, R, rand_start, stream=None):
    """nsg_build (Algorithm 2): returns (graph int32 [n][R], nav, repair_edges)."""
    n, d = base.shape
    K = knn.shape[1]
    g = torch.empty((n, R), dtype=torch.int32, device=base.device)
    nav = ctypes.c_uint32()
    rep = ctypes.c_int64()
    _call("nsg_build", _dev(base, torch.float32, "base"), n, d, _dev(knn, torch.int32, "knn"), K, int(Lb),
          int(C), int(R), int(rand_start), _dev(g, torch.int32, "graph"), ctypes.byref(nav), ctypes.byref(rep),
          _stream(stream))
    return g, int(nav.value), int(rep.value)


def build_naive(base, knn, R, stream=None):
    """nsg_build_naive (the NSG-Naive baseline): returns graph int32 [n][R]."""
    n, d = base.shape
    K = knn.shape[1]
    g = torch.empty((n, R), dtype=torch.int32, device=base.device)
    _call("nsg_build_naive", _dev(base, torch.float32, "base"), n, d, _dev(knn, torch.int32, "knn"), K, int(R),
          _dev(g, torch.int32, "graph"), _stream(stream))
    return g


def load_stop_model(index: Index, blob: bytes, n_in: int, h: int, hop: int, grid_n: int, kind: int = 0):
    """nsg_load_stop_model: blob = FP32 mean, inv_std, W1, b1, W2, b2, W3, b3, grid.
    kind STOP_SCALAR (15 scalar features) or STOP_QUERY (query + 3 state values)."""
    buf = ctypes.create_string_buffer(blob, len(blob))
    _call("nsg_load_stop_model", index.handle, buf, len(blob), int(kind), int(n_in), int(h), int(hop), int(grid_n))


def set_stop_checkpoints(index: Index, hops):
    """nsg_set_stop_checkpoints: decision checkpoints (1 to 4 ascending expansion counts)."""
    arr = (ctypes.c_int32 * len(hops))(*[int(h) for h in hops])
    _call("nsg_set_stop_checkpoints", index.handle, arr, len(hops))


def set_stop_mode(index: Index, enabled: bool, calib_c: float = 1.0):
    _call("nsg_set_stop_mode", index.handle, 1 if enabled else 0, float(calib_c))


def mlp_forward_backward(params, n_in, h, X, y, yhat=None, grad=None, loss=None, stream=None):
    B = X.shape[0]
    if grad is None:
        grad = torch.empty_like(params)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=params.device)
    _call("nsg_mlp_forward_backward", _dev(params, torch.float32, "params"), int(n_in), int(h),
          _dev(X, torch.float32, "X"), _dev(y, torch.float32, "y"), B, _dev(yhat, torch.float32, "yhat"),
          _dev(grad, torch.float32, "grad"), _dev(loss, torch.float32, "loss"), _stream(stream))
    return grad, loss


def mlp_adam(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _call("nsg_mlp_adam", _dev(params, torch.float32, "params"), _dev(grad, torch.float32, "grad"),
          _dev(m, torch.float32, "m"), _dev(v, torch.float32, "v"), params.numel(), int(t), float(lr),
          float(beta1), float(beta2), float(eps), _stream(stream))


def mlp_forward(params, n_in, h, X, yhat=None, stream=None):
    B = X.shape[0]
    if yhat is None:
        yhat = torch.empty(B, dtype=torch.float32, device=X.device)
    _call("nsg_mlp_forward", _dev(params, torch.float32, "params"), int(n_in), int(h),
          _dev(X, torch.float32, "X"), B, _dev(yhat, torch.float32, "yhat"), _stream(stream))
    return yhat


def recall_hits(found, truth, k, stream=None):
    """found [nq][G][k] int32, truth [nq][kt] int32 -> hits [nq][G] int32."""
    nq, G, kk = found.shape
    if kk != k:
        raise ValueError("found's last dim must be k")
    hits = torch.empty((nq, G), dtype=torch.int32, device=found.device)
    _call("nsg_recall_hits", _dev(found, torch.int32, "found"), nq, G, int(k), _dev(truth, torch.int32, "truth"),
          truth.shape[1], _dev(hits, torch.int32, "hits"), _stream(stream))
    return hits


def _opts(opts):
    o = SearchOpts()
    keep = []
    names = {f[0] for f in SearchOpts._fields_}
    for key, val in (opts or {}).items():
        if key not in names:
            raise KeyError(f"unknown search option {key!r}")
        if isinstance(val, torch.Tensor):
            if not val.is_cuda or not val.is_contiguous():
                raise ValueError(f"opts[{key}] must be a contiguous CUDA tensor")
            keep.append(val)
            setattr(o, key, val.data_ptr())
        else:
            setattr(o, key, int(val))
    return o, keep


class SearchGraph:
    """nsg_search_graph_*: one batch captured as a HIP graph; refill the bound
    input tensors in place and call launch()."""

    def __init__(self, index, queries, k=None, L=None, k_scalar=10, L_scalar=None, out_stride=None,
                 opts: dict | None = None):
        nq = queries.shape[0]
        if out_stride is None:
            out_stride = int(k_scalar) if k is None else int(k.max().item())
        self.queries, self.k, self.L = queries, k, L
        self.out_ids = torch.full((nq, out_stride), SENT, dtype=torch.int32, device=queries.device)
        self.out_dist = torch.full((nq, out_stride), float("inf"), dtype=torch.float32, device=queries.device)
        o, self._keep = _opts(opts)
        h = ctypes.c_void_p()
        _call("nsg_search_graph_create", index.handle, _dev(queries, torch.float32, "queries"), nq,
              _dev(k, torch.int32, "k"), _dev(L, torch.int32, "L"), int(k_scalar), int(L_scalar), int(out_stride),
              _dev(self.out_ids, torch.int32, "out_ids"), _dev(self.out_dist, torch.float32, "out_dist"),
              ctypes.byref(o), ctypes.byref(h))
        self._h = h
        self._index = index

    def launch(self, stream=None):
        _call("nsg_search_graph_launch", self._h, _stream(stream))
        return self.out_ids, self.out_dist

    def close(self):
        if self._h is not None:
            _load().nsg_search_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(index, queries, k, L, trials=3, learned_stop=0, stream=None):
    """nsg_autotune: returns (opts dict for search_batched, ms per call)."""
    o = SearchOpts()
    o.learned_stop = int(learned_stop)
    ms = ctypes.c_float()
    _call("nsg_autotune", index.handle, _dev(queries, torch.float32, "queries"), queries.shape[0], int(k), int(L),
          int(trials), ctypes.byref(o), ctypes.byref(ms), _stream(stream))
    best = dict(lanes_per_row=o.lanes_per_row, hash_slots=o.hash_slots, waves_per_block=o.waves_per_block,
                persistent=o.persistent, longest_first=o.longest_first)
    return best, float(ms.value)


def column_stats(X, stream=None):
    """nsg_column_stats: (mean [in], inv_std [in]) of X [B][in]."""
    B, n_in = X.shape
    mean = torch.empty(n_in, dtype=torch.float32, device=X.device)
    istd = torch.empty(n_in, dtype=torch.float32, device=X.device)
    _call("nsg_column_stats", _dev(X, torch.float32, "X"), B, n_in, _dev(mean, torch.float32, "mean"),
          _dev(istd, torch.float32, "inv_std"), _stream(stream))
    return mean, istd


_load()
