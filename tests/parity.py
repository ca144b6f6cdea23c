"""Parity criterion between the GPU path and the CPU oracle (test helper).

A query matches when its result id set equals the oracle's.  A mismatch is
accepted only as a near-tie: every id in the symmetric difference has an FP64
squared distance within `tie` (relative) of the oracle's k-th FP64 distance.
Returned distances must be within `rtol` of the FP64 distance of the returned
id.  Hop counts must agree on matching queries when both are given.
"""
import numpy as np

SENT = 0xFFFFFFFF


def fp64_dist(X, q, ids):
    out = np.full(len(ids), np.inf)
    for j, i in enumerate(ids):
        if int(i) != SENT:
            out[j] = float(((X[int(i)].astype(np.float64) - q.astype(np.float64)) ** 2).sum())
    return out


def compare(X, Q, gpu_ids, gpu_dist, ora_ids, ora_dist=None, rtol=1e-5, tie=1e-5,
            gpu_hops=None, ora_hops=None, min_match=0.999):
    gpu_ids = np.asarray(gpu_ids).astype(np.int64).astype(np.uint32)
    ora_ids = np.asarray(ora_ids).astype(np.int64).astype(np.uint32)
    nq, k = ora_ids.shape
    exact = 0
    ties = 0
    bad = []
    max_rel = 0.0
    for i in range(nq):
        g = [int(x) for x in gpu_ids[i] if int(x) != SENT]
        o = [int(x) for x in ora_ids[i] if int(x) != SENT]
        gd = fp64_dist(X, Q[i], g)
        if len(g):
            rel = np.abs(np.asarray(gpu_dist[i][:len(g)], np.float64) - gd) / np.maximum(gd, 1e-30)
            max_rel = max(max_rel, float(rel.max()))
        if set(g) == set(o) and len(g) == len(o):
            exact += 1
            if gpu_hops is not None and ora_hops is not None and int(gpu_hops[i]) != int(ora_hops[i]):
                bad.append((i, "hops", int(gpu_hops[i]), int(ora_hops[i])))
            continue
        od = fp64_dist(X, Q[i], o)
        dk = od.max() if len(od) else 0.0
        diff = set(g) ^ set(o)
        dd = fp64_dist(X, Q[i], sorted(diff))
        if len(g) == len(o) and np.all(np.abs(dd - dk) <= tie * max(dk, 1e-30)):
            ties += 1
        else:
            bad.append((i, "ids", sorted(set(g) - set(o))[:5], sorted(set(o) - set(g))[:5]))
    return dict(nq=nq, exact=exact, ties=ties, bad=bad, max_rel=max_rel,
                ok=(exact + ties) >= min_match * nq and max_rel <= rtol and
                not any(b[1] == "hops" for b in bad))
