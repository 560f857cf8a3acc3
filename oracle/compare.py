"""Tie-aware comparison of another implementation's k-NN results with the
FP64 oracle, and recall against exhaustive search.

TEST INFRASTRUCTURE ONLY (see ``mask_oracle``).

The rule: every returned distance is within ``rel`` (relative) of the
oracle's float64 distance for the same id, and an exact zero stays zero; the
returned ids equal the oracle's position by position, except where the two
ids' oracle distances differ by at most ``rel`` relative (a near-tie, where
either order is correct); padded slots (id -1) match.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import mask_oracle as mo


@dataclasses.dataclass
class KnnCheck:
    n_rows: int
    bad_rows: List[int]
    max_rel_dist_err: float
    n_id_diffs: int  # positions where ids differ (all within the tie rule when ok)
    messages: List[str]

    @property
    def ok(self) -> bool:
        return not self.bad_rows


def true_distances(X: np.ndarray, Q: np.ndarray, ids: np.ndarray, metric: str = "l2") -> np.ndarray:
    """Oracle float64 reported distance of each (query, returned id); inf
    where the id is -1."""
    X64 = np.asarray(X, dtype=np.float64)
    Q64 = np.asarray(Q, dtype=np.float64)
    out = np.full(ids.shape, np.inf, dtype=np.float64)
    for i in range(ids.shape[0]):
        valid = ids[i] >= 0
        if valid.any():
            diff = X64[ids[i][valid]] - Q64[i][None, :]
            if metric == "l2":
                out[i, valid] = np.sqrt(np.einsum("ij,ij->i", diff, diff))
            else:
                out[i, valid] = np.abs(diff).sum(axis=1)
    return out


def check_knn(got_ids: np.ndarray, got_dist: np.ndarray, ref_ids: np.ndarray,
              ref_dist: np.ndarray, got_true: np.ndarray, rel: float = 1e-5,
              max_messages: int = 10) -> KnnCheck:
    """Compare rows of (ids, reported distances).  ``got_true`` holds the
    oracle's float64 distance of each returned id (``true_distances``)."""
    got_ids = np.asarray(got_ids, dtype=np.int64)
    ref_ids = np.asarray(ref_ids, dtype=np.int64)
    got_dist = np.asarray(got_dist, dtype=np.float64)
    bad, msgs = [], []
    max_err = 0.0
    n_diff = 0
    for i in range(got_ids.shape[0]):
        g, o = got_ids[i], ref_ids[i]
        reason = None
        if not np.array_equal(g < 0, o < 0):
            reason = f"padding differs: got {g.tolist()} ref {o.tolist()}"
        valid = g >= 0
        if reason is None and valid.any():
            gd, gt = got_dist[i, valid], got_true[i, valid]
            if np.unique(g[valid]).size != g[valid].size:
                reason = "duplicate ids"
            zero = gt == 0
            if reason is None and np.any(gd[zero] != 0):
                reason = "exact zero distance not reported as zero"
            nz = ~zero
            if nz.any():
                err = np.abs(gd[nz] - gt[nz]) / gt[nz]
                max_err = max(max_err, float(err.max()))
                if reason is None and err.max() > rel:
                    reason = f"distance rel err {err.max():.3g} > {rel}"
            if np.any(~np.isinf(got_dist[i, ~valid])):
                reason = reason or "padded slot has a finite distance"
        if reason is None:
            for j in np.nonzero(g != o)[0]:
                n_diff += 1
                a, b = got_true[i, j], ref_dist[i, j]
                if not (abs(a - b) <= rel * max(a, b)):
                    reason = (f"id differs at slot {j}: got {g[j]} (d={a!r}) "
                              f"ref {o[j]} (d={b!r})")
                    break
        if reason is not None:
            bad.append(i)
            if len(msgs) < max_messages:
                msgs.append(f"row {i}: {reason}")
    return KnnCheck(n_rows=got_ids.shape[0], bad_rows=bad, max_rel_dist_err=max_err,
                    n_id_diffs=n_diff, messages=msgs)


def check_selection(cand: np.ndarray, cand_dist: np.ndarray, sel: np.ndarray, r: int,
                    rel: float = 1e-5) -> Optional[str]:
    """Is ``sel`` a set of the r nearest candidates up to near-ties?  Every
    selected id must be a candidate, the count must be min(r, |cand|), and no
    unselected candidate may be nearer than a selected one by more than
    ``rel`` relative.  Returns None when acceptable, else the reason."""
    sel = np.asarray(sel, dtype=np.int64)
    m = min(r, cand.size)
    if sel.size != m:
        return f"selected {sel.size} items, expected {m}"
    if np.unique(sel).size != sel.size:
        return "duplicate selection"
    pos = {int(c): p for p, c in enumerate(cand.tolist())}
    if any(int(s) not in pos for s in sel):
        return "selected id is not a candidate"
    if m == cand.size:
        return None
    mask = np.zeros(cand.size, dtype=bool)
    mask[[pos[int(s)] for s in sel]] = True
    worst_in = cand_dist[mask].max()
    best_out = cand_dist[~mask].min()
    if worst_in > best_out and (worst_in - best_out) > rel * worst_in:
        return f"selection not nearest: worst selected {worst_in!r} > best left {best_out!r}"
    return None


def replay_query(index: "mo.OracleIndex", q: np.ndarray, k: int, r: int,
                 selections: List[np.ndarray], rel: float = 1e-5):
    """Check another implementation's per-level selections (top level
    first) against the oracle's candidates at each level, then replay the
    oracle's leaf ranking on those selections.  Returns (reason or None,
    replayed ids, replayed distances)."""
    L = index.n_levels
    cand = np.arange(index.protos[L - 1].shape[0], dtype=np.int64)
    for depth, l in enumerate(range(L - 1, -1, -1)):
        d = mo.pairwise(np.asarray(q, dtype=np.float64)[None, :], index.protos[l][cand],
                        index.metric)[0]
        why = check_selection(cand, d, selections[depth], r, rel)
        if why is not None:
            return f"level {l}: {why}", None, None
        kids = index.children(l)
        sel = np.asarray(selections[depth], dtype=np.int64)
        cand = np.concatenate([kids[p] for p in sel]) if sel.size else np.zeros(0, np.int64)
    ids, dist = mo.query_one(index, q, k, r, forced=selections)
    return None, ids, dist


def recall_at_k(got_ids: np.ndarray, true_ids: np.ndarray, true_dist: np.ndarray,
                got_true: np.ndarray, k: int, rel: float = 1e-5) -> float:
    """Mean fraction of the true k nearest found.  A returned id that is not
    in the true list still counts when its true distance ties the k-th true
    distance within ``rel``."""
    hits = 0
    total = 0
    for i in range(got_ids.shape[0]):
        truth = set(int(t) for t in true_ids[i, :k] if t >= 0)
        kth = true_dist[i, min(k, len(truth)) - 1] if truth else np.inf
        got = got_ids[i, :k]
        h = 0
        for j, g in enumerate(got):
            if g < 0:
                continue
            if int(g) in truth or got_true[i, j] <= kth * (1.0 + rel):
                h += 1
        hits += min(h, len(truth))
        total += len(truth)
    return hits / max(total, 1)
