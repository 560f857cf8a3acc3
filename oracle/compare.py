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
                    rel: float = 1e-5, abs_tol: float = 0.0) -> Optional[str]:
    """Is ``sel`` a set of the r nearest candidates up to near-ties?  Every
    selected id must be a candidate, the count must be min(r, |cand|), and no
    unselected candidate may be nearer than a selected one by more than
    max(``rel`` relative, ``abs_tol``).  Returns None when acceptable, else
    the reason."""
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
    if worst_in > best_out and (worst_in - best_out) > max(rel * worst_in, abs_tol):
        return f"selection not nearest: worst selected {worst_in!r} > best left {best_out!r}"
    return None


def replay_query(index: "mo.OracleIndex", q: np.ndarray, k: int, r,
                 selections: List[np.ndarray], rel: float = 1e-5):
    """Check another implementation's per-level selections (top level
    first) against the oracle's candidates at each level, then replay the
    oracle's leaf ranking on those selections.  ``r``: one beam, or one per
    level from the top.  Returns (reason or None, replayed ids, replayed
    distances)."""
    L = index.n_levels
    beams = [int(r)] * L if np.isscalar(r) else [int(x) for x in r]
    cand = np.arange(index.protos[L - 1].shape[0], dtype=np.int64)
    for depth, l in enumerate(range(L - 1, -1, -1)):
        d = mo.pairwise(np.asarray(q, dtype=np.float64)[None, :], index.protos[l][cand],
                        index.metric)[0]
        why = check_selection(cand, d, selections[depth], beams[depth], rel)
        if why is not None:
            return f"level {l}: {why}", None, None
        kids = index.children(l)
        sel = np.asarray(selections[depth], dtype=np.int64)
        cand = np.concatenate([kids[p] for p in sel]) if sel.size else np.zeros(0, np.int64)
    ids, dist = mo.query_one(index, q, k, beams, forced=selections)
    return None, ids, dist


def screened_bound(q: np.ndarray, rows: np.ndarray) -> float:
    """Bound on |s - delta^2(q, c)| for a screened score s = |q|^2 + |c|^2 -
    2 q.c of a bfloat16 row c against a float32 query q written as two
    bfloat16 terms (hi + lo, |q - hi - lo| <= 2^-18 |q| per entry), with
    float32 norms and float32 accumulation of the exact bfloat16 products:
    ((3d + 4) 2^-24 + 2^-18) (|q|^2 + |c|^2), doubled for slack, with the
    largest |c|^2 of ``rows``."""
    q = np.asarray(q, dtype=np.float64)
    d = q.shape[0]
    cmax = float(np.einsum("ij,ij->i", rows, rows).max()) if rows.size else 0.0
    return 2.0 * ((3 * d + 4) * 2.0 ** -24 + 2.0 ** -18) * (float(q @ q) + cmax)


def check_rerank(got_ids: np.ndarray, got_dist: np.ndarray, cand: np.ndarray,
                 d_low: np.ndarray, d_full: np.ndarray, k: int, R: int,
                 rel: float = 1e-5) -> Optional[str]:
    """Is one result row the k nearest on the full rows of a set of the R
    nearest candidates by low-precision distance?  ``d_low`` and ``d_full``
    are the squared distances of every leaf candidate; when there are no
    more than R candidates, or R <= k, every candidate is ranked on the full
    rows.  Both cuts accept near-ties within ``rel``: a candidate within
    ``rel`` of the R-th low-precision distance may be in the set or not, and
    the ranking is checked on reported (square-rooted) distances.  Returns
    None when acceptable, else the reason."""
    got_ids = np.asarray(got_ids, dtype=np.int64)
    got_dist = np.asarray(got_dist, dtype=np.float64)
    D = np.sqrt(np.asarray(d_full, dtype=np.float64))
    if cand.size > R and R > k:
        order = np.lexsort((cand, d_low))
        dR = d_low[order[R - 1]]
        sure = d_low < dR - rel * dR
        maybe = d_low <= dR + rel * dR
        n_pool = R
    else:
        sure = np.ones(cand.size, dtype=bool)
        maybe = sure
        n_pool = cand.size
    where = {int(c): j for j, c in enumerate(cand.tolist())}
    valid = got_ids >= 0
    n_ret = int(valid.sum())
    if n_ret != min(k, n_pool):
        return f"returned {n_ret} ids, expected {min(k, n_pool)}"
    if not np.all(valid[:n_ret]):
        return "padding before a returned id"
    g = got_ids[:n_ret]
    if np.unique(g).size != g.size:
        return "duplicate ids"
    if any(int(x) not in where for x in g):
        return "returned id is not a leaf candidate"
    pos = np.array([where[int(x)] for x in g], dtype=np.int64)
    if not np.all(maybe[pos]):
        return "returned id is outside the re-rank set"
    gd = got_dist[:n_ret]
    err = np.abs(gd - D[pos]) / np.maximum(D[pos], np.finfo(float).tiny)
    if np.any((D[pos] == 0) & (gd != 0)) or np.any(err[D[pos] > 0] > rel):
        return f"distance rel err {err.max():.3g} > {rel}"
    if np.any(np.diff(gd) < 0):
        return "distances not ascending"
    if np.any(~np.isinf(got_dist[n_ret:])):
        return "padded slot has a finite distance"
    if n_ret:
        kth = D[pos].max()
        left = sure.copy()
        left[pos] = False
        if np.any(D[left] < kth - rel * kth):
            j = int(np.argmin(np.where(left, D, np.inf)))
            return f"candidate {int(cand[j])} (d={D[j]!r}) is nearer than the k-th returned ({kth!r})"
    return None


def check_lowp_query(index: "mo.OracleIndex", q: np.ndarray, k: int, beams,
                     selections: List[np.ndarray], got_ids: np.ndarray, got_dist: np.ndarray,
                     rank_protos, leaf_rows: np.ndarray, factor: int,
                     abs_tol=None, rel: float = 1e-5) -> Optional[str]:
    """One query of the precision form against the oracle on the same
    index: at every level (top first) the implementation's selection must be
    a nearest set of the candidates by the FP64 distance to
    ``rank_protos[l]`` (the level's rows as the descent reads them), up to
    ``rel`` or ``abs_tol[depth]`` (None: relative only); then the result row
    must pass ``check_rerank`` on the leaf candidates of those selections
    with R = ``mo.rerank_size``.  Returns None when acceptable."""
    L = index.n_levels
    beams = [int(beams)] * L if np.isscalar(beams) else [int(x) for x in beams]
    q64 = np.asarray(q, dtype=np.float64)[None, :]
    cand = np.arange(index.protos[L - 1].shape[0], dtype=np.int64)
    for depth, l in enumerate(range(L - 1, -1, -1)):
        rows = np.asarray(rank_protos[l][cand], dtype=np.float64)
        d = mo.pairwise(q64, rows, "l2")[0]
        tol = 0.0 if abs_tol is None or abs_tol[depth] is None else float(abs_tol[depth])
        why = check_selection(cand, d, selections[depth], beams[depth], rel, tol)
        if why is not None:
            return f"level {l}: {why}"
        kids = index.children(l)
        sel = np.asarray(selections[depth], dtype=np.int64)
        cand = np.concatenate([kids[p] for p in sel]) if sel.size else np.zeros(0, np.int64)
    R = mo.rerank_size(k, beams, factor)
    d_low = mo.pairwise(q64, np.asarray(leaf_rows[cand], dtype=np.float64), "l2")[0] \
        if cand.size else np.zeros(0)
    d_full = mo.pairwise(q64, index.data[cand], "l2")[0] if cand.size else np.zeros(0)
    why = check_rerank(got_ids, got_dist, cand, d_low, d_full, k, R, rel)
    return None if why is None else f"data layer: {why}"


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
