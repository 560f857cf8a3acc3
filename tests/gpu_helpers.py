"""Shared helpers of the GPU tests: device upload, and the tie-aware
comparison of a GPU query against the FP64 oracle on the same index."""
import numpy as np

from oracle import compare as oc
from oracle import mask_oracle as mo


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def oracle_index_from_gpu(X, index, metric="l2"):
    """FP64 oracle view of a GPU-built index (exported prototypes and
    parents of every level)."""
    L = index.info()["n_levels"]
    protos, parents = [], []
    for lev in range(1, L + 1):
        P, par = index.export_level(lev)
        protos.append(P)
        parents.append(par)
    return mo.index_from_arrays(X, protos, parents, metric)


def check_query_against_oracle(oix, X, Q, k, r, ids, dist, sel, rel=1e-5, rows=None):
    """Compare GPU (ids, dist, sel) with the oracle's descent on the same
    index.  Rows whose plain comparison fails are accepted when the GPU's
    per-level selections are nearest sets up to near-ties and the oracle's
    leaf ranking replayed on them matches.  Returns (n_checked, n_replayed,
    failures)."""
    rows = range(Q.shape[0]) if rows is None else rows
    failures = []
    n_replayed = 0
    metric = oix.metric
    for i in rows:
        o_ids, o_dist = mo.query_one(oix, Q[i], k, r)
        g_ids = ids[i:i + 1].astype(np.int64)
        g_dist = dist[i:i + 1].astype(np.float64)
        true = oc.true_distances(X, Q[i:i + 1], g_ids, metric)
        res = oc.check_knn(g_ids, g_dist, o_ids[None], o_dist[None], true, rel)
        if res.ok:
            continue
        L = oix.n_levels
        selections = [s[s >= 0] for s in sel[i]] if sel is not None else None
        if selections is None:
            failures.append((i, res.messages))
            continue
        why, r_ids, r_dist = oc.replay_query(oix, Q[i], k, r, selections, rel)
        n_replayed += 1
        if why is not None:
            failures.append((i, [why] + res.messages))
            continue
        res2 = oc.check_knn(g_ids, g_dist, r_ids[None], r_dist[None], true, rel)
        if not res2.ok:
            failures.append((i, ["after replay"] + res2.messages))
    return len(list(rows)), n_replayed, failures
