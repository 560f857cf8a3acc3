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


def check_query_against_oracle(oix, X, Q, k, r, ids, dist, sel, rel=1e-5, rows=None,
                               max_replay_frac=0.05):
    """Compare GPU (ids, dist, sel) with the oracle's descent on the same
    index.  Rows whose plain comparison fails are accepted when the GPU's
    per-level selections are nearest sets up to near-ties and the oracle's
    leaf ranking replayed on them matches.  Replays are expected only at
    near-ties: more than max(2, max_replay_frac of the rows) counts as a
    failure.  Returns (n_checked, n_replayed, failures)."""
    rows = list(range(Q.shape[0]) if rows is None else rows)
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
    limit = max(2, int(np.ceil(max_replay_frac * len(rows))))
    if n_replayed > limit:
        failures.append((-1, [f"{n_replayed} of {len(rows)} rows needed a replay (limit {limit})"]))
    return len(rows), n_replayed, failures


def check_lowp_against_oracle(oix, Q, k, beams, ids, dist, sel, rank_protos, leaf_rows,
                              factor, screened_levels=(), rows=None, rel=1e-5):
    """Precision form against the oracle on the same index, per query:
    each level's selection is a nearest set by the FP64 distance to the
    level's low-precision rows (screened levels within the expanded-form
    bound, the others within ``rel``), and the result is the FP32 re-rank of
    an R-nearest set by low-precision distance (``oc.check_lowp_query``).
    ``screened_levels``: level numbers (1 = first prototype level) scored by
    the batched GEMM.  Returns the list of (row, reason) failures."""
    L = oix.n_levels
    rows = range(Q.shape[0]) if rows is None else rows
    fails = []
    for i in rows:
        tol = []
        for depth in range(L):
            lev = L - depth  # level number of this depth
            if lev in screened_levels:
                tol.append(oc.screened_bound(Q[i], np.asarray(rank_protos[lev - 1])))
            else:
                tol.append(None)
        selections = [s[s >= 0] for s in sel[i]]
        why = oc.check_lowp_query(oix, Q[i], k, beams, selections, ids[i], dist[i],
                                  rank_protos, leaf_rows, factor, tol, rel)
        if why is not None:
            fails.append((i, why))
    return fails
