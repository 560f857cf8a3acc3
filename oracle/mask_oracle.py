"""FP64 CPU oracle for the MASK hot path (arXiv 2208.02734).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this module; only the tests, the smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code with the HIP path: it is plain numpy in
float64, written to be checked against the paper by eye, and slow.

What it computes, by paper passage:

* ``plan_levels``      - the level schedule of Algorithm 1 (multilevel index
                         construction), floor division.
* ``splitmix64_keys``,
  ``permutation``      - the random assignment of points to groups used in
                         Section 4.2 ("randomly assigned"), made concrete as
                         the argsort of SplitMix64 outputs (Steele, Lea and
                         Flood, OOPSLA 2014).
* ``chunk_offsets``    - ``split(data, ngroups)`` of Algorithm 1: nearly
                         equal contiguous groups (first n mod C get one more).
* ``kmeanspp_seeds``   - k-means++ seeding (Section 3.1 names it), with a
                         counter-based SplitMix64 draw per step.
* ``lloyd``            - ``kmeans(nCentroids, points)`` of Algorithm 1 as
                         Lloyd iterations with the first k group members as
                         initial prototypes.
* ``build``            - Algorithm 1 itself: per-group k-means at each level,
                         bottom-up, keeping prototypes and labels.
* ``query``            - the k-NN search of Algorithm 2 and the text of
                         Section 3.3 ("Searching and data insertion"),
                         generalised from the greedy choice to a beam of the
                         r nearest prototypes at every level.
* ``point_query_one``  - the point query of Section 3.3: greedy descent,
                         then a full scan of the leaf for the nearest point
                         and for an exact match.
* ``relocate``         - one relocation step (Sections 4.1-4.2, Table 1):
                         points not found join the group of the leaf their
                         point query reached, before the index is rebuilt.
* ``insert``           - dynamic insertion (Section 3.3): greedy descent to
                         a leaf, and the local rebuild of a level-0 group
                         whose leaf grows beyond a threshold.
* ``range_query_one``  - the range search of Algorithm 3: the prototypes
                         within the radius at every level, then the points
                         within the radius under them.
* ``exact_knn``        - the k-nearest-neighbour query of the problem
                         statement (Section 1) by exhaustive search.
* ``quantize_bf16``,
  ``quantize_fp8``,
  ``query_one_lowp``   - the precision form (not in the paper): the
                         rounding of rows to bfloat16 or to OCP e4m3 with a
                         per-row scale, and the descent on such rows with an
                         oversized candidate set re-ranked on the full rows.

Readings of silent or garbled passages (each one is listed in the design doc):
the ranking key at every selection is (distance, original id), so ties go to
the lower id; squared Euclidean distance is ranked and its square root is
reported; empty prototypes keep their previous value; the L1 update is the
per-dimension lower median; only level 0 is shuffled; children of a
prototype are the items whose label is that prototype.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

# --------------------------------------------------------------------------
# Level schedule (Algorithm 1, floor division)
# --------------------------------------------------------------------------


def plan_levels(n: int, length_group: int, n_centroids: int) -> List[Tuple[int, int]]:
    """Algorithm 1: ngroups = n // lengthGroup; k-means with nCentroids in
    each group; the next level groups the ngroups*nCentroids prototypes by
    lengthGroup again; stop once fewer than one full group remains.

    Returns [(n_groups, n_centroids)] bottom-up."""
    if length_group < 1 or n_centroids < 1:
        raise ValueError("length_group and n_centroids must be positive")
    levels = []
    ngroups = n // length_group
    while ngroups >= 1:
        levels.append((ngroups, n_centroids))
        ngroups = (ngroups * n_centroids) // length_group
        if len(levels) > 64:
            raise ValueError("schedule does not shrink (n_centroids >= length_group)")
    return levels


# --------------------------------------------------------------------------
# Random assignment to groups (Section 4.2) and split (Algorithm 1)
# --------------------------------------------------------------------------

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_keys(seed: int, n: int) -> np.ndarray:
    """The (i+1)-th SplitMix64 output from state ``seed`` for i = 0..n-1:
    state_i = seed + (i+1)*gamma (mod 2^64), then the 64-bit finaliser
    z ^= z>>30; z *= M1; z ^= z>>27; z *= M2; z ^= z>>31."""
    i = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform01(seed: int, counter: int) -> float:
    """A uniform draw in [0, 1) from the SplitMix64 output at ``counter``
    (the same outputs as ``splitmix64_keys``): its top 53 bits times 2^-53."""
    z = (int(seed) + (int(counter) + 1) * 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    z ^= z >> 31
    return (z >> 11) * 2.0 ** -53


def permutation(seed: int, n: int) -> np.ndarray:
    """pi = points ordered by (key, index); the keys are distinct because the
    finaliser is a bijection and the states are distinct for n < 2^64."""
    keys = splitmix64_keys(seed, n)
    return np.argsort(keys, kind="stable").astype(np.int64)


def chunk_offsets(n_items: int, n_chunks: int) -> np.ndarray:
    """Boundaries of ``split`` into n_chunks contiguous groups whose sizes
    differ by at most one, the larger ones first."""
    if n_chunks < 1 or n_chunks > n_items:
        raise ValueError("need 1 <= n_chunks <= n_items")
    base, extra = divmod(n_items, n_chunks)
    sizes = np.full(n_chunks, base, dtype=np.int64)
    sizes[:extra] += 1
    off = np.zeros(n_chunks + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    return off


# --------------------------------------------------------------------------
# Dissimilarity delta (Section 1: Minkowski family; Euclidean in all
# experiments).  Squared L2 is returned for "l2" and ranked; L1 for "l1".
# --------------------------------------------------------------------------


def pairwise(A: np.ndarray, B: np.ndarray, metric: str = "l2", block: int = 256) -> np.ndarray:
    """delta(a_i, b_j) for all pairs, direct form in float64:
    l2 -> sum_k (a_ik - b_jk)^2, l1 -> sum_k |a_ik - b_jk|."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    out = np.empty((A.shape[0], B.shape[0]), dtype=np.float64)
    for s in range(0, A.shape[0], block):
        diff = A[s:s + block, None, :] - B[None, :, :]
        if metric == "l2":
            out[s:s + block] = np.einsum("ijk,ijk->ij", diff, diff)
        elif metric == "l1":
            out[s:s + block] = np.abs(diff).sum(axis=2)
        else:
            raise ValueError(f"unknown metric {metric!r}")
    return out


def report_distance(dsq: np.ndarray, metric: str) -> np.ndarray:
    """Value reported to the user: the Euclidean distance for l2 (square
    root of the ranked squared distance), the L1 sum as is."""
    return np.sqrt(dsq) if metric == "l2" else dsq


# --------------------------------------------------------------------------
# k-means (Lloyd) inside one group
# --------------------------------------------------------------------------


def assign(points: np.ndarray, centroids: np.ndarray, metric: str = "l2"):
    """Label of each point = index of its nearest prototype, lowest index on
    ties (numpy argmin returns the first minimum).  Also returns each point's
    distance to that prototype."""
    D = pairwise(points, centroids, metric)
    labels = np.argmin(D, axis=1)
    return labels, D[np.arange(points.shape[0]), labels]


def lower_median(values: np.ndarray) -> np.ndarray:
    """Per-column lower median: the floor((m-1)/2)-th order statistic."""
    m = values.shape[0]
    return np.sort(values, axis=0)[(m - 1) // 2]


def update(points: np.ndarray, labels: np.ndarray, centroids: np.ndarray, metric: str = "l2"):
    """New prototypes: the mean (l2) or the per-dimension lower median (l1)
    of the members; a prototype with no member keeps its previous value."""
    points = np.asarray(points, dtype=np.float64)
    new = np.array(centroids, dtype=np.float64, copy=True)
    counts = np.bincount(labels, minlength=centroids.shape[0])
    for j in range(centroids.shape[0]):
        if counts[j] == 0:
            continue
        members = points[labels == j]
        if metric == "l2":
            new[j] = members.sum(axis=0) / counts[j]
        else:
            new[j] = lower_median(members)
    return new, counts


@dataclasses.dataclass
class LloydResult:
    centroids: np.ndarray  # (k, d) float64
    labels: np.ndarray  # (m,) int64, labels of the final assignment
    inertia: np.ndarray  # (iters,) float64: I_t = sum delta(x, c^t_{a^t})


def lloyd_step(points: np.ndarray, centroids: np.ndarray, metric: str = "l2"):
    """One Lloyd iteration from C_t: assignment a^t, inertia I_t computed
    with C_t, and the updated C_{t+1}."""
    labels, dmin = assign(points, centroids, metric)
    inertia = float(dmin.sum())
    new, _ = update(points, labels, centroids, metric)
    return labels, new, inertia


KMEANSPP_LEVEL_STRIDE = 1 << 40


def kmeanspp_seeds(points: np.ndarray, k: int, seed: int, level: int, chunk: int) -> np.ndarray:
    """k-means++ seeding (Arthur and Vassilvitskii, SODA 2007), which Section
    3.1 names as the way to spread the initial prototypes: the first is a
    member drawn uniformly; every next one is member i with probability
    D(i)^2 / sum_j D(j)^2, where D(i) is the Euclidean distance of member i
    to the nearest prototype chosen so far.

    Readings (the paper gives no procedure): draw t of group ``chunk`` at
    level ``level`` is u_t = uniform01(seed, 2^40 * level + chunk * k + t);
    draw 0 picks member floor(u_0 * m); draw t picks the first member, in
    group order, whose running sum of D^2 exceeds u_t * sum D^2 (or, if
    rounding leaves none, the last member with D^2 > 0); when every D^2 is
    0 the pick is uniform as for draw 0.  D^2 in float64 direct form.
    Returns the chosen member indices."""
    X = np.asarray(points, dtype=np.float64)
    m = X.shape[0]
    tag = KMEANSPP_LEVEL_STRIDE * int(level) + int(chunk) * int(k)
    chosen = np.empty(k, dtype=np.int64)
    d2 = None
    for t in range(k):
        u = uniform01(seed, tag + t)
        pick = -1
        if t > 0:
            total = float(d2.sum())
            if total > 0.0:
                run = np.cumsum(d2)
                above = np.nonzero(run > u * total)[0]
                pick = int(above[0]) if above.size else int(np.nonzero(d2 > 0)[0][-1])
        if pick < 0:
            pick = min(int(u * m), m - 1)
        chosen[t] = pick
        diff = X - X[pick][None, :]
        d = np.einsum("ij,ij->i", diff, diff)
        d2 = d if d2 is None else np.minimum(d2, d)
    return chosen


def lloyd(points: np.ndarray, k: int, iters: int, metric: str = "l2",
          init: Optional[np.ndarray] = None) -> LloydResult:
    """kmeans(nCentroids, points) of Algorithm 1 as Lloyd's algorithm: the
    initial prototypes are the first k points of the group (cyclically when
    the group holds fewer than k), then ``iters``
    rounds of (assign, update), then a final assignment so the labels belong
    to the returned prototypes."""
    points = np.asarray(points, dtype=np.float64)
    m = points.shape[0]
    if k < 1 or m < 1:
        raise ValueError("need k >= 1 and a non-empty group")
    # A group smaller than k (relocation can leave one) starts from its
    # members taken cyclically; the repeated copies tie with the first copy,
    # lose the tie (lowest index wins) and so stay empty with their value.
    first = points[np.arange(k) % m]
    C = np.array(first if init is None else init, dtype=np.float64, copy=True)
    log = np.empty(iters, dtype=np.float64)
    for t in range(iters):
        _, C, log[t] = lloyd_step(points, C, metric)
    labels, _ = assign(points, C, metric)
    return LloydResult(centroids=C, labels=labels, inertia=log)


# --------------------------------------------------------------------------
# Algorithm 1: multilevel index construction
# --------------------------------------------------------------------------


@dataclasses.dataclass
class OracleIndex:
    """protos[l] (n_l x d, chunk-major ids: chunk c holds ids c*k_l .. c*k_l+k_l-1)
    for l = 0..L-1 (index 0 is the first centroid level above the data);
    parents[l] gives, for each item of the level below (data points for
    l = 0, in original row order; prototypes of level l-1 otherwise), the id
    of its prototype at level l."""

    data: np.ndarray  # (n, d) float64
    protos: List[np.ndarray]
    parents: List[np.ndarray]
    levels: List[Tuple[int, int]]
    metric: str
    inertia: List[np.ndarray]  # per level, (n_chunks, iters)
    _kids: Optional[List[List[np.ndarray]]] = None
    # level-0 order (original ids) and group boundaries of the build
    perm0: Optional[np.ndarray] = None
    group_off0: Optional[np.ndarray] = None

    @property
    def n_levels(self) -> int:
        return len(self.protos)

    def children(self, level: int) -> List[np.ndarray]:
        """children(p) for every prototype p of ``level``: ids of the items
        one level down whose label is p, ascending."""
        if self._kids is None:
            self._kids = [self._children(l) for l in range(self.n_levels)]
        return self._kids[level]

    def _children(self, level: int) -> List[np.ndarray]:
        par = self.parents[level]
        n_l = self.protos[level].shape[0]
        order = np.argsort(par, kind="stable")
        counts = np.bincount(par, minlength=n_l)
        off = np.zeros(n_l + 1, dtype=np.int64)
        off[1:] = np.cumsum(counts)
        return [order[off[p]:off[p + 1]] for p in range(n_l)]


def build(X: np.ndarray, levels: Sequence[Tuple[int, int]], iters: int, seed: int,
          metric: str = "l2", perm: Optional[np.ndarray] = None,
          group_off: Optional[np.ndarray] = None, init: str = "first") -> OracleIndex:
    """Algorithm 1 with explicit level sizes [(n_chunks, k)] bottom-up.

    Level 0 (the data) is permuted by ``permutation(seed, n)`` (or the given
    ``perm``) and split into n_chunks contiguous groups (or at the given
    ``group_off`` boundaries, as a relocation leaves them); every upper level
    splits the previous level's prototypes, in chunk-major id order, the same
    way without shuffling.  Each group runs ``lloyd`` independently, from
    its first k members (``init="first"``) or from ``kmeanspp_seeds`` with
    the build's seed and the level number (``init="kmeans++"``)."""
    if init not in ("first", "kmeans++"):
        raise ValueError("init must be 'first' or 'kmeans++'")
    if init == "kmeans++" and metric != "l2":
        raise ValueError("k-means++ seeding is defined for the l2 metric")
    data = np.asarray(X, dtype=np.float64)
    n = data.shape[0]
    pi = permutation(seed, n) if perm is None else np.asarray(perm, dtype=np.int64)
    items = data[pi]
    item_ids = pi  # original id of each item in the current order
    protos, parents, inertia = [], [], []
    off0 = None
    for lev, (n_chunks, k) in enumerate(levels):
        if lev == 0 and group_off is not None:
            off = np.asarray(group_off, dtype=np.int64)
            if off.shape[0] != n_chunks + 1 or off[0] != 0 or off[-1] != n or \
                    np.any(np.diff(off) < 1):
                raise ValueError("group_off must rise strictly from 0 to n")
        else:
            off = chunk_offsets(items.shape[0], n_chunks)
        if lev == 0:
            off0 = off
        P = np.empty((n_chunks * k, data.shape[1]), dtype=np.float64)
        par = np.empty(items.shape[0], dtype=np.int64)
        logs = np.empty((n_chunks, iters), dtype=np.float64)
        for c in range(n_chunks):
            pts = items[off[c]:off[c + 1]]
            start = None
            if init == "kmeans++":
                start = pts[kmeanspp_seeds(pts, k, seed, lev + 1, c)]
            res = lloyd(pts, k, iters, metric, init=start)
            P[c * k:(c + 1) * k] = res.centroids
            par[item_ids[off[c]:off[c + 1]]] = c * k + res.labels
            logs[c] = res.inertia
        protos.append(P)
        parents.append(par)
        inertia.append(logs)
        items = P
        item_ids = np.arange(P.shape[0], dtype=np.int64)
    return OracleIndex(data=data, protos=protos, parents=parents, levels=list(levels),
                       metric=metric, inertia=inertia, perm0=np.asarray(pi, dtype=np.int64),
                       group_off0=np.asarray(off0, dtype=np.int64))


def index_from_arrays(X: np.ndarray, protos: Sequence[np.ndarray], parents: Sequence[np.ndarray],
                      metric: str = "l2") -> OracleIndex:
    """Wrap prototypes and parent arrays produced elsewhere (for instance
    exported from the GPU) so that ``query`` can run on them."""
    levels = [(0, 0)] * len(protos)
    return OracleIndex(data=np.asarray(X, dtype=np.float64),
                       protos=[np.asarray(p, dtype=np.float64) for p in protos],
                       parents=[np.asarray(p, dtype=np.int64) for p in parents],
                       levels=levels, metric=metric, inertia=[])


# --------------------------------------------------------------------------
# Algorithm 2: k-NN search, with a beam of r prototypes per level
# --------------------------------------------------------------------------


def smallest(dist: np.ndarray, ids: np.ndarray, m: int) -> np.ndarray:
    """Positions of the m smallest entries ordered by (dist, id)."""
    order = np.lexsort((ids, dist))
    return order[:m]


@dataclasses.dataclass
class QueryTrace:
    selected: List[np.ndarray]  # per level, top level first: selected prototype ids
    candidates: List[np.ndarray]  # per level, top level first: candidate ids
    cand_dist: List[np.ndarray]  # the ranked distance of each candidate


def query_one(index: OracleIndex, q: np.ndarray, k: int, r: int,
              trace: bool = False, forced: Optional[List[np.ndarray]] = None):
    """Descent for one query.  Top level: rank all prototypes, keep the r
    nearest.  Each lower level: the candidates are the children of the kept
    prototypes; keep the r nearest of them (all when fewer).  Data layer: the
    candidates are the points under the kept level-1 prototypes; return the
    k nearest by (delta, original id), padded with (-1, inf).

    ``forced`` replaces the selection made at each level (top level first) so
    that the leaf result can be replayed on another implementation's choice."""
    metric = index.metric
    L = index.n_levels
    q = np.asarray(q, dtype=np.float64)[None, :]
    kids = [index.children(l) for l in range(L)]
    # r: one beam for every level, or one per level from the top level down
    beams = [int(r)] * L if np.isscalar(r) else [int(x) for x in r]
    cand = np.arange(index.protos[L - 1].shape[0], dtype=np.int64)
    tr = QueryTrace([], [], [])
    for l in range(L - 1, -1, -1):
        d = pairwise(q, index.protos[l][cand], metric)[0]
        sel = cand[smallest(d, cand, beams[L - 1 - l])]
        if forced is not None:
            sel = np.asarray(forced[L - 1 - l], dtype=np.int64)
        if trace:
            tr.selected.append(sel)
            tr.candidates.append(cand)
            tr.cand_dist.append(d)
        cand = (np.concatenate([kids[l][p] for p in sel]) if sel.size else
                np.zeros(0, dtype=np.int64))
    d = pairwise(q, index.data[cand], metric)[0] if cand.size else np.zeros(0)
    pos = smallest(d, cand, k)
    ids = np.full(k, -1, dtype=np.int64)
    dist = np.full(k, np.inf, dtype=np.float64)
    ids[:pos.size] = cand[pos]
    dist[:pos.size] = report_distance(d[pos], metric)
    if trace:
        tr.candidates.append(cand)
        tr.cand_dist.append(d)
        return ids, dist, tr
    return ids, dist


def query(index: OracleIndex, Q: np.ndarray, k: int, r: int):
    """``query_one`` for every row of Q; returns ids (nq x k) int64 and
    reported distances (nq x k) float64."""
    Q = np.asarray(Q, dtype=np.float64)
    ids = np.empty((Q.shape[0], k), dtype=np.int64)
    dist = np.empty((Q.shape[0], k), dtype=np.float64)
    for i in range(Q.shape[0]):
        ids[i], dist[i] = query_one(index, Q[i], k, r)
    return ids, dist


# --------------------------------------------------------------------------
# Precision form (not in the paper): rows held in a low precision for the
# descent, an oversized candidate set re-ranked on the full rows
# --------------------------------------------------------------------------


def quantize_bf16(X: np.ndarray) -> np.ndarray:
    """Value of every float32 entry of X rounded to bfloat16 (8 significant
    bits, round to nearest, ties to even), as float64.  Written from the
    format's definition: the 16 low bits of the float32 encoding are
    dropped after adding half of their weight, the half going up only when
    the kept part is odd."""
    x = np.ascontiguousarray(X, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    r = ((u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)) \
        << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def round_e4m3(v: np.ndarray) -> np.ndarray:
    """Nearest value of the OCP float8 e4m3 format (4 exponent bits with
    bias 7, 3 mantissa bits, largest finite value 448, subnormal step 2^-9),
    ties to even; inputs must lie in [-448, 448]."""
    v = np.asarray(v, dtype=np.float64)
    a = np.abs(v)
    # spacing of the format at |v|: 2^(e-3) in the binade [2^e, 2^(e+1)),
    # 2^-9 below the smallest normal 2^-6
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    step = np.where(a >= 2.0 ** -6, 2.0 ** (e - 3), 2.0 ** -9)
    return np.sign(v) * np.round(a / step) * step  # np.round: half to even


def quantize_fp8(X: np.ndarray):
    """FP8 rows of the precision form: per row, m = max|x| and scale s =
    m / 448 (1 for a zero row), both in float32; every entry x times the
    float32 reciprocal 448 / m (rounded to float32), clamped to [-448, 448]
    and rounded to e4m3.  Returns (codes as float64 values, s as float64);
    the row is represented as s * code."""
    x = np.asarray(X, dtype=np.float32)
    m = np.abs(x).max(axis=1)
    pos = m > 0
    s = np.where(pos, (m / np.float32(448.0)).astype(np.float32), np.float32(1.0))
    inv = np.where(pos, (np.float32(448.0) / np.where(pos, m, 1)).astype(np.float32),
                   np.float32(1.0)).astype(np.float32)
    v = (x * inv[:, None]).astype(np.float32)
    v = np.clip(v, np.float32(-448.0), np.float32(448.0))
    return round_e4m3(v), s.astype(np.float64)


def rerank_size(k: int, beams: Sequence[int], factor: int) -> int:
    """Size R of the candidate set the precision form re-ranks on the full
    rows: R0 = factor * k, or f * k * r1 for factor = -f (r1 = the last beam,
    the number of leaves probed: the "4 k r" set of the precision form at
    f = 4); R = R0 capped at 512 when R0, k and every beam are at most 512,
    else at 2048."""
    r0 = -int(factor) * int(k) * int(beams[-1]) if int(factor) < 0 else int(factor) * int(k)
    cap = 512 if max([int(k), r0] + [int(b) for b in beams]) <= 512 else 2048
    return min(r0, cap)


def query_one_lowp(index: OracleIndex, q: np.ndarray, k: int, r, rank_protos,
                   leaf_rows: np.ndarray, factor: int, forced=None, trace: bool = False):
    """Descent of the precision form for one query (L2).  At every
    prototype level the ranking uses ``rank_protos[l]`` (the level's rows in
    the precision the descent reads them in) instead of the prototypes
    themselves; the children are those of the index.  At the data layer,
    with m candidates and R = ``rerank_size(k, beams, factor)``: when m > R
    and R > k, the R nearest by distance to ``leaf_rows`` (the data rows in
    low precision, same row order as the data) are kept, ranked by (delta,
    id), and ranked again by the distance to the full rows; otherwise every
    candidate is ranked on the full rows.  Returns the k nearest as
    ``query_one`` does.  ``forced`` replaces each level's selection (top
    level first); ``trace`` also returns the leaf candidates, their
    low-precision distances and R."""
    L = index.n_levels
    q64 = np.asarray(q, dtype=np.float64)[None, :]
    kids = [index.children(l) for l in range(L)]
    beams = [int(r)] * L if np.isscalar(r) else [int(x) for x in r]
    cand = np.arange(index.protos[L - 1].shape[0], dtype=np.int64)
    for l in range(L - 1, -1, -1):
        d = pairwise(q64, np.asarray(rank_protos[l], dtype=np.float64)[cand], "l2")[0]
        sel = cand[smallest(d, cand, beams[L - 1 - l])]
        if forced is not None:
            sel = np.asarray(forced[L - 1 - l], dtype=np.int64)
        cand = (np.concatenate([kids[l][p] for p in sel]) if sel.size else
                np.zeros(0, dtype=np.int64))
    R = rerank_size(k, beams, factor)
    d_low = (pairwise(q64, np.asarray(leaf_rows, dtype=np.float64)[cand], "l2")[0]
             if cand.size else np.zeros(0))
    pool = cand
    if cand.size > R and R > k:
        pool = cand[smallest(d_low, cand, R)]
    d = pairwise(q64, index.data[pool], "l2")[0] if pool.size else np.zeros(0)
    pos = smallest(d, pool, k)
    ids = np.full(k, -1, dtype=np.int64)
    dist = np.full(k, np.inf, dtype=np.float64)
    ids[:pos.size] = pool[pos]
    dist[:pos.size] = np.sqrt(d[pos])
    if trace:
        return ids, dist, (cand, d_low, R)
    return ids, dist


# --------------------------------------------------------------------------
# Point query (Section 3.3) and relocation (Sections 4.1 and 4.2, Table 1)
# --------------------------------------------------------------------------


def point_query_one(index: OracleIndex, q: np.ndarray):
    """Point query of Section 3.3 for one query q.  At the top level the
    prototype nearest to q is chosen; at every level below, the nearest among
    the children of the prototype chosen above; the chosen level-1 prototype
    is the leaf.  A full scan of the data points of the leaf gives the answer
    (the nearest of them, ties to the lower id) and the perfect match sought
    (the lowest id of a point equal to q coordinate by coordinate, else -1).

    Returns (answer id, reported distance, leaf id, match id); answer and
    leaf are -1 (distance inf) when the leaf has no points."""
    metric = index.metric
    L = index.n_levels
    q = np.asarray(q, dtype=np.float64)
    chosen = -1
    for l in range(L - 1, -1, -1):
        if l == L - 1:
            cand = np.arange(index.protos[l].shape[0], dtype=np.int64)
        else:
            cand = index.children(l + 1)[chosen]
        if cand.size == 0:
            return -1, np.inf, -1, -1
        d = pairwise(q[None, :], index.protos[l][cand], metric)[0]
        chosen = int(cand[np.lexsort((cand, d))[0]])
    leaf = chosen
    pts = index.children(0)[leaf]
    if pts.size == 0:
        return -1, np.inf, leaf, -1
    d = pairwise(q[None, :], index.data[pts], metric)[0]
    best = int(np.lexsort((pts, d))[0])
    equal = pts[np.all(index.data[pts] == q[None, :], axis=1)]
    match = int(equal.min()) if equal.size else -1
    return int(pts[best]), float(report_distance(d[best:best + 1], metric)[0]), leaf, match


def exhaustive_point_search(index: OracleIndex):
    """The evaluation of Section 4.1: a point query for every data point.
    Returns arrays (answer, leaf, match) in data row order."""
    n = index.data.shape[0]
    ans = np.empty(n, dtype=np.int64)
    leaf = np.empty(n, dtype=np.int64)
    match = np.empty(n, dtype=np.int64)
    for i in range(n):
        ans[i], _, leaf[i], match[i] = point_query_one(index, index.data[i])
    return ans, leaf, match


def relocate(perm: np.ndarray, group_off: np.ndarray, k0: int, leaf: np.ndarray,
             wrong: np.ndarray):
    """One relocation step (Section 4.1, iterated in Table 1): a data point
    that its own point query did not find correctly (``wrong``) joins the
    level-0 group that produced the leaf the query reached (group
    leaf // k0, the level-1 prototypes being chunk-major); the index is then
    built again on the new groups.

    ``perm`` is the level-0 order the index was built with (original ids)
    and ``group_off`` its group boundaries in that order.  Readings: a group
    keeps the members that stay, in their old order, followed by the points
    that join it, in their old order; a group left empty is dropped and the
    rest keep their relative order; a point whose query reached no leaf (an
    empty prototype on its path, leaf -1) stays.  Returns the new
    (perm, group_off)."""
    perm = np.asarray(perm, dtype=np.int64)
    group_off = np.asarray(group_off, dtype=np.int64)
    n, C = perm.shape[0], group_off.shape[0] - 1
    stay = [[] for _ in range(C)]
    join = [[] for _ in range(C)]
    for g in range(C):
        for j in range(group_off[g], group_off[g + 1]):
            i = int(perm[j])
            target = int(leaf[i]) // k0 if wrong[i] and leaf[i] >= 0 else g
            if target >= C:
                raise ValueError("leaf outside level 1")
            (stay if target == g else join)[target].append(i)
    order, off = [], [0]
    for g in range(C):
        members = stay[g] + join[g]
        if members:
            order.extend(members)
            off.append(off[-1] + len(members))
    assert len(order) == n
    return np.array(order, dtype=np.int64), np.array(off, dtype=np.int64)


# --------------------------------------------------------------------------
# Dynamic insertion (Section 3.3, the data-insertion procedure and the local
# rebuild of a partition that grows too large)
# --------------------------------------------------------------------------


def insertion_leaf(index: OracleIndex, x: np.ndarray) -> int:
    """The leaf a new point joins: the nearest top-level prototype, then at
    each level the nearest child of the one chosen, down to a level-1
    prototype.  Reading: above level 1 a prototype without children is
    skipped (a path through it ends before any leaf); level-1 prototypes are
    leaves whether or not they hold points.  Ties go to the lower id."""
    metric = index.metric
    L = index.n_levels
    x = np.asarray(x, dtype=np.float64)
    cand = np.arange(index.protos[L - 1].shape[0], dtype=np.int64)
    for l in range(L - 1, -1, -1):
        if l >= 1:
            kids = index.children(l)
            cand = np.array([p for p in cand if kids[p].size > 0], dtype=np.int64)
        d = pairwise(x[None, :], index.protos[l][cand], metric)[0]
        chosen = int(cand[np.lexsort((cand, d))[0]])
        if l >= 1:
            cand = index.children(l)[chosen]
    return chosen


def insert(index: OracleIndex, X_new: np.ndarray, max_leaf: int = 0, iters: int = 0):
    """Insert the rows of X_new.  Every new point joins the leaf given by
    ``insertion_leaf`` on the index as it was before the batch (insertion
    changes no prototype, so the order within the batch does not matter)
    and takes the next id.  Then every level-0 group holding a leaf with
    more than ``max_leaf`` points (max_leaf > 0) is built again locally: its
    Lloyd iterations (``iters`` of them, then the final assignment) run
    over the group's current members, starting from the group's current
    prototypes; the levels above keep their structure.

    Readings: a new point joins the level-0 group that produced its leaf
    (leaf // k0), after that group's members, in batch order; leaf sizes are
    measured once the whole batch is placed; groups are rebuilt in
    ascending order.  Returns (new index, leaves of the new points, ids of
    the rebuilt groups)."""
    if index.perm0 is None or index.group_off0 is None:
        raise ValueError("insertion needs the level-0 groups of the build")
    X_new = np.asarray(X_new, dtype=np.float64)
    n0 = index.data.shape[0]
    k0 = index.protos[0].shape[0] // (index.group_off0.shape[0] - 1)
    leaves = np.array([insertion_leaf(index, x) for x in X_new], dtype=np.int64)
    data = np.concatenate([index.data, X_new]) if X_new.size else index.data.copy()
    parents = [p.copy() for p in index.parents]
    parents[0] = np.concatenate([parents[0], leaves])
    protos = [p.copy() for p in index.protos]
    C = index.group_off0.shape[0] - 1
    members = [list(index.perm0[index.group_off0[g]:index.group_off0[g + 1]]) for g in range(C)]
    for j, leaf in enumerate(leaves):
        members[int(leaf) // k0].append(n0 + j)
    rebuilt = []
    if max_leaf > 0:
        sizes = np.bincount(parents[0], minlength=protos[0].shape[0])
        for g in range(C):
            if sizes[g * k0:(g + 1) * k0].max() > max_leaf:
                ids = np.array(members[g], dtype=np.int64)
                res = lloyd(data[ids], k0, iters, index.metric,
                            init=protos[0][g * k0:(g + 1) * k0])
                protos[0][g * k0:(g + 1) * k0] = res.centroids
                parents[0][ids] = g * k0 + res.labels
                rebuilt.append(g)
    perm0 = np.concatenate([np.array(m, dtype=np.int64) for m in members])
    off0 = np.zeros(C + 1, dtype=np.int64)
    off0[1:] = np.cumsum([len(m) for m in members])
    new = OracleIndex(data=data, protos=protos, parents=parents, levels=list(index.levels),
                      metric=index.metric, inertia=index.inertia, perm0=perm0,
                      group_off0=off0)
    return new, leaves, rebuilt


# --------------------------------------------------------------------------
# Range search (Algorithm 3 and the range-query paragraph of Section 3.3)
# --------------------------------------------------------------------------


def range_query_one(index: OracleIndex, q: np.ndarray, radius: float, max_out: int,
                    level_cap: int):
    """Range search for one query.  At the top level, and at every level
    below among the children of the kept prototypes, keep the prototypes
    whose distance to q is at most ``radius`` (the ball of the paragraph);
    at the data layer, the points under the kept level-1 prototypes whose
    distance is at most ``radius`` are the answer.

    Readings: distances compare as squared L2 against radius^2 (delta <= r);
    at most ``level_cap`` prototypes are kept per level, the nearest by
    (distance, id), a bound the paper leaves open; the answer is ranked by
    (distance, id) and the first ``max_out`` are returned (ids, reported
    distances) together with the number of points within the radius."""
    if index.metric != "l2":
        raise ValueError("range search is written for the l2 metric")
    L = index.n_levels
    q = np.asarray(q, dtype=np.float64)[None, :]
    r2 = float(radius) ** 2
    kids = [index.children(l) for l in range(L)]
    cand = np.arange(index.protos[L - 1].shape[0], dtype=np.int64)
    for l in range(L - 1, -1, -1):
        d = pairwise(q, index.protos[l][cand], "l2")[0] if cand.size else np.zeros(0)
        inside = d <= r2
        cand_in, d_in = cand[inside], d[inside]
        sel = cand_in[smallest(d_in, cand_in, level_cap)]
        cand = (np.concatenate([kids[l][p] for p in sel]) if sel.size else
                np.zeros(0, dtype=np.int64))
    d = pairwise(q, index.data[cand], "l2")[0] if cand.size else np.zeros(0)
    inside = d <= r2
    cand_in, d_in = cand[inside], d[inside]
    pos = smallest(d_in, cand_in, max_out)
    ids = np.full(max_out, -1, dtype=np.int64)
    dist = np.full(max_out, np.inf, dtype=np.float64)
    ids[:pos.size] = cand_in[pos]
    dist[:pos.size] = np.sqrt(d_in[pos])
    return ids, dist, int(cand_in.size)


# --------------------------------------------------------------------------
# Exhaustive k-NN (problem statement, Section 1)
# --------------------------------------------------------------------------


def exact_knn(X: np.ndarray, Q: np.ndarray, k: int, metric: str = "l2",
              block: int = 1 << 16):
    """The k nearest rows of X for each query by (delta, id), exhaustively.

    l1, or small X: direct form on every pair.  l2 at scale: the expanded
    form |x|^2 + |q|^2 - 2 q.x (a float64 matrix product) screens, keeping
    every row within twice a rounding bound of the k-th screened value, and
    the kept rows are re-scored in direct form, so the result is the
    direct-form ranking."""
    X64 = np.asarray(X, dtype=np.float64)
    Q64 = np.asarray(Q, dtype=np.float64)
    n, d = X64.shape
    nq = Q64.shape[0]
    kk = min(k, n)
    ids = np.full((nq, k), -1, dtype=np.int64)
    dist = np.full((nq, k), np.inf, dtype=np.float64)
    if metric == "l1" or n * d <= (1 << 22):
        for i in range(nq):
            dd = pairwise(Q64[i:i + 1], X64, metric)[0]
            pos = smallest(dd, np.arange(n), kk)
            ids[i, :kk] = pos
            dist[i, :kk] = report_distance(dd[pos], metric)
        return ids, dist
    xn = np.einsum("ij,ij->i", X64, X64)
    xn_max = float(xn.max())
    eps = 2.0 ** -53
    for i0 in range(0, nq, 256):
        Qb = Q64[i0:i0 + 256]
        qn = np.einsum("ij,ij->i", Qb, Qb)
        # Running shortlist of (screened value, id) per query, block by block.
        best_v = np.full((Qb.shape[0], 0), np.inf)
        best_i = np.zeros((Qb.shape[0], 0), dtype=np.int64)
        bound = 4.0 * (d + 4) * eps * (qn + xn_max)  # |error| of each screened value
        for s in range(0, n, block):
            e = min(n, s + block)
            S = xn[None, s:e] + qn[:, None] - 2.0 * (Qb @ X64[s:e].T)
            v = np.concatenate([best_v, S], axis=1)
            idx = np.concatenate([best_i, np.broadcast_to(np.arange(s, e), S.shape)], axis=1)
            kth = np.partition(v, kk - 1, axis=1)[:, kk - 1]
            keep = v <= (kth + 2.0 * bound)[:, None]
            width = int(keep.sum(axis=1).max())
            nv = np.full((Qb.shape[0], width), np.inf)
            ni = np.full((Qb.shape[0], width), -1, dtype=np.int64)
            for row in range(Qb.shape[0]):
                sel = np.nonzero(keep[row])[0]
                nv[row, :sel.size] = v[row, sel]
                ni[row, :sel.size] = idx[row, sel]
            best_v, best_i = nv, ni
        for row in range(Qb.shape[0]):
            cand = best_i[row][best_i[row] >= 0]
            dd = pairwise(Qb[row:row + 1], X64[cand], "l2")[0]
            pos = smallest(dd, cand, kk)
            ids[i0 + row, :kk] = cand[pos]
            dist[i0 + row, :kk] = np.sqrt(dd[pos])
    return ids, dist


# --------------------------------------------------------------------------
# Sparse rows (Section 4.3 setting: high-dimensional, sparse, non-negative)
# --------------------------------------------------------------------------


def sparse_pairwise_l2(indptr_a, indices_a, values_a, B: np.ndarray) -> np.ndarray:
    """Squared Euclidean distance between CSR rows a_i and dense rows b_j,
    |a|^2 + |b|^2 - 2 a.b in float64 (rows are unit-norm, so there is no
    cancellation to speak of at float64)."""
    B = np.asarray(B, dtype=np.float64)
    na = indptr_a.shape[0] - 1
    out = np.empty((na, B.shape[0]), dtype=np.float64)
    bn = np.einsum("ij,ij->i", B, B)
    for i in range(na):
        cols = indices_a[indptr_a[i]:indptr_a[i + 1]]
        vals = values_a[indptr_a[i]:indptr_a[i + 1]].astype(np.float64)
        out[i] = float(vals @ vals) + bn - 2.0 * (B[:, cols] @ vals)
    return out
