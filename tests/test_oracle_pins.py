"""Pins of the FP64 oracle to facts outside itself: the paper's printed
integers, published known answers, closed forms, library routines, brute
force on tiny inputs, and invariants of Lloyd's algorithm and of the
descent.  CPU only."""
import json
import os

import numpy as np
import pytest
from scipy.cluster.vq import kmeans2
from scipy.spatial import cKDTree

import datagen
from oracle import compare as oc
from oracle import mask_oracle as mo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- schedule

def test_level_schedule_worked_examples():
    g = _golden("paper_level_schedule.json")
    for case in g["cases"]:
        lv = mo.plan_levels(case["n"], case["length_group"], case["n_centroids"])
        m = len(case["first_levels"])
        assert [list(x) for x in lv[:m]] == case["first_levels"], case["cite"]
        sizes = [c * k for c, k in lv]
        assert sizes[:m] == case["first_sizes"]
        # the top level holds at most lengthGroup prototypes
        assert sizes[-1] <= case["length_group"]


def test_level_schedule_tree_depths():
    g = _golden("paper_level_schedule.json")["depth_cases"]
    for lg, nc, depth in g["rows"]:
        assert len(mo.plan_levels(g["n"], lg, nc)) == depth, (lg, nc)


def test_level_schedule_rejects_non_shrinking():
    with pytest.raises(ValueError):
        mo.plan_levels(1000, 4, 4)


# ------------------------------------------------------------- permutation

def test_splitmix64_known_answers():
    g = _golden("splitmix64_known_answers.json")
    keys = mo.splitmix64_keys(g["state"], len(g["outputs_hex"]))
    assert [int(k) for k in keys] == [int(h, 16) for h in g["outputs_hex"]]


def test_splitmix64_matches_python_integers():
    # Arbitrary-precision Python arithmetic, masked to 64 bits, as a second
    # route to the same published definition.
    def mix(z):
        M = (1 << 64) - 1
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)
    seed = 0x1234_5678_9ABC_DEF1
    keys = mo.splitmix64_keys(seed, 50)
    for i in range(50):
        st = (seed + (i + 1) * 0x9E3779B97F4A7C15) & ((1 << 64) - 1)
        assert int(keys[i]) == mix(st)


def test_permutation_is_bijection_and_sorted_by_key():
    pi = mo.permutation(7, 10_000)
    assert np.array_equal(np.sort(pi), np.arange(10_000))
    keys = mo.splitmix64_keys(7, 10_000)
    assert np.all(keys[pi][1:] > keys[pi][:-1])


def test_chunk_offsets_match_numpy_array_split():
    for n, c in [(10, 3), (20_000, 10), (1_000_003, 100), (7, 7)]:
        parts = np.array_split(np.arange(n), c)
        off = mo.chunk_offsets(n, c)
        assert [p.size for p in parts] == np.diff(off).tolist()


# ------------------------------------------------------------------- Lloyd

def _blobs(seed, n_per, centers, sigma):
    g = np.random.default_rng(seed)
    pts = np.concatenate([c + sigma * g.standard_normal((n_per, len(c))) for c in centers])
    return pts[g.permutation(pts.shape[0])]


def test_assign_matches_brute_force_loops():
    g = np.random.default_rng(1)
    P = g.standard_normal((13, 3))
    C = g.standard_normal((5, 3))
    labels, dmin = mo.assign(P, C)
    for i in range(13):
        best, arg = None, None
        for j in range(5):
            s = 0.0
            for t in range(3):
                s += (P[i, t] - C[j, t]) ** 2
            if best is None or s < best:
                best, arg = s, j
        assert labels[i] == arg
        assert abs(dmin[i] - best) <= 1e-12 * max(best, 1)


def test_assign_tie_goes_to_lowest_index():
    P = np.array([[0.0, 0.0]])
    C = np.array([[1.0, 0.0], [-1.0, 0.0], [0.0, 1.0]])
    labels, _ = mo.assign(P, C)
    assert labels[0] == 0


def test_kmeans_one_prototype_is_the_mean():
    g = np.random.default_rng(2)
    P = g.uniform(-5, 5, (200, 7))
    res = mo.lloyd(P, 1, 3)
    np.testing.assert_allclose(res.centroids[0], P.mean(axis=0), rtol=0, atol=1e-12)
    assert np.all(res.labels == 0)


def test_kmeans_k_equals_m_is_identity():
    g = np.random.default_rng(3)
    P = g.standard_normal((12, 4))
    res = mo.lloyd(P, 12, 5)
    assert np.array_equal(res.labels, np.arange(12))
    np.testing.assert_array_equal(res.centroids, P)
    assert np.all(res.inertia == 0)


def test_kmeans_matches_scipy_kmeans2_with_given_init():
    P = _blobs(4, 40, [np.array([0, 0, 0.]), np.array([6, 0, 0.]), np.array([0, 6, 0.]),
                       np.array([0, 0, 6.])], 1.0)
    init = P[:4].copy()
    res = mo.lloyd(P, 4, 10, init=init)
    cb, lab = kmeans2(P, init.copy(), iter=10, minit="matrix")
    np.testing.assert_allclose(res.centroids, cb, rtol=0, atol=1e-10)
    assert np.array_equal(res.labels, lab)


def test_kmeans_recovers_separated_cluster_means():
    centers = [np.array([0.0, 0.0]), np.array([100.0, 0.0]), np.array([0.0, 100.0])]
    P = _blobs(5, 50, centers, 0.5)
    # one initial prototype inside each cloud
    init = np.array([P[np.argmin(((P - c) ** 2).sum(1))] for c in centers])
    res = mo.lloyd(P, 3, 4, init=init)
    for j, c in enumerate(centers):
        members = P[((P - c) ** 2).sum(1) < 100]
        np.testing.assert_allclose(res.centroids[j], members.mean(axis=0), atol=1e-12)


def test_lloyd_invariants_l2():
    g = np.random.default_rng(6)
    P = g.standard_normal((300, 5)) * g.uniform(0.2, 3, (300, 1))
    res = mo.lloyd(P, 17, 25)
    # inertia never increases
    assert np.all(np.diff(res.inertia) <= 1e-9 * res.inertia[:-1])
    # final labels are an argmin under the returned prototypes
    D = ((P[:, None, :] - res.centroids[None]) ** 2).sum(-1)
    assert np.all(D[np.arange(300), res.labels] <= D.min(axis=1))
    # inertia of step t is the sum of nearest distances under C_t
    labels, C1, I0 = mo.lloyd_step(P, P[:17])
    D0 = ((P[:, None, :] - P[None, :17]) ** 2).sum(-1)
    assert abs(I0 - D0.min(axis=1).sum()) <= 1e-9 * I0


def test_empty_prototype_keeps_its_value():
    P = np.array([[0.0], [0.1], [0.2], [10.0]])
    C = np.array([[0.0], [50.0], [10.0]])
    labels, new, _ = mo.lloyd_step(P, C)
    assert labels.tolist() == [0, 0, 0, 2]
    assert new[1, 0] == 50.0
    np.testing.assert_allclose(new[0, 0], 0.1)


def test_lower_median_minimises_l1_and_is_a_data_value():
    g = np.random.default_rng(7)
    for m in [1, 2, 3, 4, 9, 10]:
        v = g.integers(-5, 6, size=(m, 3)).astype(float)
        med = mo.lower_median(v)
        for t in range(3):
            col = sorted(v[:, t].tolist())
            assert med[t] == col[(m - 1) // 2]
            cost = lambda a: sum(abs(x - a) for x in col)  # noqa: E731
            assert cost(med[t]) <= min(cost(x) for x in col) + 1e-12


def test_lloyd_invariants_l1():
    g = np.random.default_rng(8)
    P = g.laplace(size=(200, 4))
    res = mo.lloyd(P, 9, 15, metric="l1")
    assert np.all(np.diff(res.inertia) <= 1e-9 * res.inertia[:-1])
    D = np.abs(P[:, None, :] - res.centroids[None]).sum(-1)
    assert np.all(D[np.arange(200), res.labels] <= D.min(axis=1))


# ------------------------------------------------------------ build/query

def _small_index(seed=11, n=600, d=5, levels=((6, 10), (2, 6), (1, 4)), iters=8):
    g = np.random.default_rng(seed)
    X = (g.standard_normal((n, d)) * 2 + g.integers(-8, 8, (n, 1))).astype(np.float32)
    return X, mo.build(X, list(levels), iters, seed=99)


def test_build_structure():
    X, ix = _small_index()
    assert [p.shape[0] for p in ix.protos] == [60, 12, 4]
    assert ix.parents[0].shape[0] == 600
    pi = mo.permutation(99, 600)
    off = mo.chunk_offsets(600, 6)
    for c in range(6):
        members = pi[off[c]:off[c + 1]]
        # every point of chunk c is labelled with a prototype of chunk c
        assert np.all(ix.parents[0][members] // 10 == c)
    # children partition each level
    for l in range(3):
        kids = ix.children(l)
        allk = np.sort(np.concatenate(kids))
        assert np.array_equal(allk, np.arange(ix.parents[l].shape[0]))
    assert all(np.all(np.diff(log, axis=1) <= 1e-9 * log[:, :-1]) for log in ix.inertia)


def test_probe_all_is_exact_knn():
    X, ix = _small_index()
    g = np.random.default_rng(12)
    Q = g.standard_normal((25, 5)) * 3
    ids, dist = mo.query(ix, Q, 7, r=10_000)
    tree = cKDTree(X.astype(np.float64))
    tdist, tids = tree.query(Q, k=7)
    np.testing.assert_allclose(dist, tdist, rtol=1e-12)
    # ids equal up to exact distance ties (none expected with continuous data)
    assert np.array_equal(ids, tids)


def test_one_to_one_ratio_is_exact():
    # Section 5: one centroid per data point gives exact search.
    g = np.random.default_rng(13)
    X = g.standard_normal((120, 3)).astype(np.float32)
    ix = mo.build(X, [(4, 30), (2, 60)], 3, seed=5)
    Q = g.standard_normal((10, 3))
    k = 5
    ids, dist = mo.query(ix, Q, k, r=k)
    tids, tdist = mo.exact_knn(X, Q, k)
    assert np.array_equal(ids, tids)
    np.testing.assert_allclose(dist, tdist, rtol=1e-12)


def test_greedy_descent_follows_nearest_prototype():
    X, ix = _small_index()
    q = np.array([1.0, -2.0, 0.5, 0.0, 3.0])
    ids, dist, tr = mo.query_one(ix, q, 3, 1, trace=True)
    # at each level the chosen prototype is the nearest among the candidates
    for sel, cand, d in zip(tr.selected, tr.candidates, tr.cand_dist):
        assert sel.size == 1
        assert d[list(cand).index(sel[0])] == d.min()
    # the result lies inside the chosen level-1 prototype's children
    leaf = set(ix.children(0)[tr.selected[-1][0]].tolist())
    assert set(ids[ids >= 0].tolist()) <= leaf


def test_query_pads_when_too_few_candidates():
    g = np.random.default_rng(14)
    X = g.standard_normal((40, 2)).astype(np.float32)
    ix = mo.build(X, [(2, 10), (1, 2)], 5, seed=1)
    ids, dist = mo.query(ix, g.standard_normal((3, 2)), 40, r=1)
    for row_i, row_d in zip(ids, dist):
        n_valid = (row_i >= 0).sum()
        assert n_valid < 40
        assert np.all(np.isinf(row_d[n_valid:]))
        assert np.all(row_i[n_valid:] == -1)


def test_exact_knn_screened_path_matches_kdtree():
    g = np.random.default_rng(15)
    X = (g.standard_normal((40_000, 128)) + 5).astype(np.float32)  # n*d > 2^22
    Q = (g.standard_normal((30, 128)) + 5).astype(np.float32)
    ids, dist = mo.exact_knn(X, Q, 10)
    tree = cKDTree(X.astype(np.float64))
    tdist, tids = tree.query(Q.astype(np.float64), k=10)
    assert np.array_equal(ids, tids)
    np.testing.assert_allclose(dist, tdist, rtol=1e-12)


def test_l1_query_probe_all_is_exact():
    g = np.random.default_rng(16)
    X = g.standard_normal((300, 4)).astype(np.float32)
    ix = mo.build(X, [(3, 20), (1, 6)], 5, seed=2, metric="l1")
    Q = g.standard_normal((8, 4))
    ids, dist = mo.query(ix, Q, 5, r=1000)
    tree = cKDTree(X.astype(np.float64))
    tdist, tids = tree.query(Q, k=5, p=1)
    assert np.array_equal(ids, tids)
    np.testing.assert_allclose(dist, tdist, rtol=1e-12)


def test_sparse_distance_equals_dense_on_densified_rows():
    from datagen import sample_sparse
    S = sample_sparse(30, 64, 8, seed=3)
    D = S.to_dense()
    g = np.random.default_rng(17)
    B = np.abs(g.standard_normal((5, 64)))
    got = mo.sparse_pairwise_l2(S.indptr, S.indices, S.values, B)
    ref = mo.pairwise(D, B)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------- comparator

def test_comparator_accepts_self_and_near_ties_rejects_errors():
    X, ix = _small_index()
    g = np.random.default_rng(18)
    Q = g.standard_normal((10, 5))
    ids, dist = mo.query(ix, Q, 6, r=3)
    true = oc.true_distances(X, Q, ids)
    assert oc.check_knn(ids, dist, ids, dist, true).ok
    # swap two neighbours that are far from tied -> rejected
    bad = ids.copy()
    bad[0, [0, 5]] = bad[0, [5, 0]]
    tb = oc.true_distances(X, Q, bad)
    assert not oc.check_knn(bad, tb, ids, dist, tb).ok
    # a distance off by 1e-4 relative -> rejected
    off = dist.copy()
    off[1, 2] *= 1 + 1e-4
    assert not oc.check_knn(ids, off, ids, dist, true).ok


def test_recall_counts_ties():
    true_ids = np.array([[1, 2, 3]])
    true_dist = np.array([[1.0, 2.0, 3.0]])
    got = np.array([[1, 2, 9]])
    got_true = np.array([[1.0, 2.0, 3.0]])  # id 9 ties the 3rd distance
    assert oc.recall_at_k(got, true_ids, true_dist, got_true, 3) == 1.0
    got_true2 = np.array([[1.0, 2.0, 3.5]])
    assert abs(oc.recall_at_k(got, true_ids, true_dist, got_true2, 3) - 2 / 3) < 1e-12


def test_check_selection_accepts_nearest_sets_and_near_ties_only():
    cand = np.array([10, 11, 12, 13, 14, 15])
    d = np.array([5.0, 1.0, 3.0, 2.0, 4.0, 6.0])
    # the three nearest, in any order
    assert oc.check_selection(cand, d, np.array([13, 11, 12]), 3) is None
    # leaves out a strictly nearer candidate (12 at 3.0 for 14 at 4.0)
    why = oc.check_selection(cand, d, np.array([11, 13, 14]), 3)
    assert why is not None and "not nearest" in why
    # a near-tie within 1e-6 relative may go either way
    dt = d.copy()
    dt[4] = 3.0 * (1 + 1e-6)
    assert oc.check_selection(cand, dt, np.array([11, 13, 14]), 3) is None
    # ... but not a gap of 1e-4 relative
    dt[4] = 3.0 * (1 + 1e-4)
    assert oc.check_selection(cand, dt, np.array([11, 13, 14]), 3) is not None
    # an absolute tolerance widens the tie band
    assert oc.check_selection(cand, d, np.array([11, 13, 14]), 3, abs_tol=1.5) is None
    assert oc.check_selection(cand, d, np.array([11, 13, 14]), 3, abs_tol=0.5) is not None
    # wrong count, duplicates, a non-candidate
    for bad, what in (([11, 13], "expected 3"), ([11, 11, 13], "duplicate"),
                      ([11, 13, 99], "not a candidate")):
        why = oc.check_selection(cand, d, np.array(bad), 3)
        assert why is not None and what in why
    # r at least the candidate count: every candidate, in any order
    assert oc.check_selection(cand, d, cand[::-1], 8) is None


def _tie_index():
    """Two top prototypes at the same distance from the query (the origin):
    A = (-1, 0) with leaf points near it, B = (1, 0) with leaf points near
    it.  Level 1 holds one prototype per point; the top level two."""
    pts = np.array([[-1.0, 0.1], [-1.0, -0.2], [-1.1, 0.0],
                    [1.0, 0.05], [1.2, 0.0], [0.9, -0.3]])
    lv1 = pts.copy()
    par1 = np.arange(6)
    top = np.array([[-1.0, 0.0], [1.0, 0.0]])
    par2 = np.array([0, 0, 0, 1, 1, 1])
    return pts, mo.index_from_arrays(pts, [lv1, top], [par1, par2])


def test_replay_with_own_selections_reproduces_query_one_bit_for_bit():
    X, ix = _small_index()
    g = np.random.default_rng(31)
    for _ in range(20):
        q = g.standard_normal(5) * 3
        for r in (1, 3, [2, 5, 3]):
            ids, dist, tr = mo.query_one(ix, q, 6, r, trace=True)
            why, r_ids, r_dist = oc.replay_query(ix, q, 6, r, tr.selected)
            assert why is None
            assert np.array_equal(ids, r_ids)
            assert np.array_equal(dist, r_dist)


def test_replay_follows_a_tied_selection_and_rejects_a_farther_one():
    pts, ix = _tie_index()
    q = np.zeros(2)
    ids, _, tr = mo.query_one(ix, q, 2, 1, trace=True)
    assert tr.selected[0].tolist() == [0]  # the tie goes to the lower id
    # B ties A: accepted, and the leaf set changes with it
    # (under B the nearest level-1 prototype is point 5, at 0.9)
    why, r_ids, _ = oc.replay_query(ix, q, 2, 1, [np.array([1]), np.array([5])])
    assert why is None
    assert r_ids.tolist() == [5, -1] and ids.tolist() == [0, -1]
    # move the query towards A: B is now strictly farther and is rejected
    why, _, _ = oc.replay_query(ix, np.array([-0.01, 0.0]), 2, 1,
                                [np.array([1]), np.array([5])])
    assert why is not None and why.startswith("level 1")
    # a level-0 selection that is not a child of the kept top prototype
    why, _, _ = oc.replay_query(ix, q, 2, 1, [np.array([0]), np.array([4])])
    assert why is not None and "not a candidate" in why


def test_check_rerank_takes_the_low_precision_cut_then_the_full_ranking():
    cand = np.arange(100, 108)
    d_full = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0, 8.0]) ** 2
    # low-precision order puts candidate 100 (nearest in full) last
    d_low = np.array([9.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0, 8.0]) ** 2
    k, R = 2, 4
    good_ids = np.array([101, 102])
    good_d = np.array([2.0, 3.0])
    assert oc.check_rerank(good_ids, good_d, cand, d_low, d_full, k, R) is None
    # returning 100 is wrong: it is outside the R nearest by low precision
    assert oc.check_rerank(np.array([100, 101]), np.array([1.0, 2.0]), cand, d_low,
                           d_full, k, R) is not None
    # skipping 102 (in the set, nearer than 103) is wrong
    assert oc.check_rerank(np.array([101, 103]), np.array([2.0, 4.0]), cand, d_low,
                           d_full, k, R) is not None
    # with R >= |cand| every candidate is ranked on the full rows
    assert oc.check_rerank(np.array([100, 101]), np.array([1.0, 2.0]), cand, d_low,
                           d_full, k, 8) is None
    # a candidate tied with the R-th low-precision distance may be in or out
    d_low2 = d_low.copy()
    d_low2[0] = d_low[4] * (1 + 1e-7)   # 100 ties the 4th (104)
    assert oc.check_rerank(np.array([100, 101]), np.array([1.0, 2.0]), cand, d_low2,
                           d_full, k, R) is None
    # distances off by 1e-4 relative, or not ascending
    assert oc.check_rerank(good_ids, good_d * (1 + 1e-4), cand, d_low, d_full, k, R)
    assert oc.check_rerank(good_ids[::-1], good_d[::-1], cand, d_low, d_full, k, R)


# ------------------------------------------------------------ precision form

def test_bf16_rounding_matches_torch_and_ties_to_even():
    import torch
    g = np.random.default_rng(40)
    x = (g.standard_normal(20_000) * 10.0 ** g.integers(-6, 6, 20_000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mo.quantize_bf16(x), ref)
    # halfway cases: 1 + 2^-8 lies between 1 and 1 + 2^-7 -> 1 (even);
    # 1 + 3 * 2^-8 lies between 1 + 2^-7 and 1 + 2^-6 -> 1 + 2^-6 (even)
    h = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8)], dtype=np.float32)
    assert mo.quantize_bf16(h).tolist() == [1.0, 1 + 2.0 ** -6, -1.0]


def test_e4m3_rounding_matches_torch_and_keeps_every_code():
    import torch
    # every finite e4m3 value is a fixed point
    codes = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64)
    vals = codes.numpy()
    vals = vals[np.isfinite(vals)]
    assert np.array_equal(mo.round_e4m3(vals), vals)
    assert vals.max() == 448.0 and np.min(vals[vals > 0]) == 2.0 ** -9
    g = np.random.default_rng(41)
    v = np.clip(g.standard_normal(50_000) * 10.0 ** g.integers(-4, 3, 50_000), -448, 448)
    v = v.astype(np.float32)
    ref = torch.from_numpy(v).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(mo.round_e4m3(v.astype(np.float64)), ref)
    # halfway between 1 and 1.125 goes to 1 (even), between 1.125 and 1.25 to 1.25
    assert mo.round_e4m3(np.array([1.0625, 1.1875])).tolist() == [1.0, 1.25]


def test_fp8_rows_reconstruct_within_half_a_step():
    g = np.random.default_rng(42)
    X = (g.standard_normal((300, 24)) * g.uniform(0.01, 100, (300, 1))).astype(np.float32)
    X[7] = 0.0
    code, s = mo.quantize_fp8(X)
    assert s[7] == 1.0 and np.all(code[7] == 0)
    # the largest entry of each row lands on 448
    nz = np.abs(X).max(axis=1) > 0
    assert np.all(np.abs(code[nz]).max(axis=1) == 448.0)
    # normal codes carry 3 mantissa bits: |s*code - x| <= 2^-4 |x| (+ subnormal step)
    err = np.abs(s[:, None] * code - X.astype(np.float64))
    assert np.all(err <= 2.0 ** -4 * np.abs(X) + s[:, None] * 2.0 ** -10 + 1e-30)


def test_rerank_size_caps():
    assert mo.rerank_size(10, [3, 12, 104], 4) == 40
    # a set above 512 lifts the cap to 2048
    assert mo.rerank_size(200, [3, 12, 104], 4) == 800
    assert mo.rerank_size(100, [3, 12, 104], 5) == 500
    assert mo.rerank_size(200, [3, 600, 104], 4) == 800
    assert mo.rerank_size(600, [3], 48) == 2048
    # -f: f * k * (leaves probed), the "4 k r" set
    assert mo.rerank_size(10, [3, 3, 24], -4) == 960
    assert mo.rerank_size(10, [2, 4, 12], -4) == 480
    assert mo.rerank_size(10, [4, 8, 96], -4) == 2048


def test_lowp_descent_on_exact_rows_is_the_plain_descent():
    X, ix = _small_index()
    g = np.random.default_rng(43)
    for _ in range(15):
        q = g.standard_normal(5) * 3
        for factor in (1, 2, 4, 1000):
            a = mo.query_one(ix, q, 6, [2, 4, 3])
            b = mo.query_one_lowp(ix, q, 6, [2, 4, 3], ix.protos, ix.data, factor)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_lowp_descent_preselects_by_the_low_precision_rows():
    pts, ix = _tie_index()
    q = np.array([-1.0, 0.0])
    # leaf candidates {0, 1, 2} at full distances 0.1, 0.2, 0.1; the
    # low-precision copy pushes point 0 far away
    low = pts.copy()
    low[0] = [5.0, 5.0]
    ids, dist = mo.query_one_lowp(ix, q, 1, [1, 3], ix.protos, low, 2)
    # R = 2 keeps {1, 2} by low distance; the nearest of those on the full
    # rows is point 2 (0.1)
    assert ids.tolist() == [2]
    assert abs(dist[0] - 0.1) < 1e-12
    # R = k: every candidate is ranked on the full rows (0 and 2 tie at 0.1;
    # the tie goes to the lower id)
    ids2, _ = mo.query_one_lowp(ix, q, 1, [1, 3], ix.protos, low, 1)
    assert ids2.tolist() == [0]
    ids3, _ = mo.query_one_lowp(ix, q, 2, [1, 3], ix.protos, low, 1)
    assert ids3.tolist() == [0, 2]


def test_screened_bound_covers_the_float32_expanded_form():
    import torch
    g = np.random.default_rng(44)
    for d in (16, 96, 128):
        Q = (g.uniform(-10, 10, (40, d)) + g.standard_normal((40, d))).astype(np.float32)
        C = mo.quantize_bf16((g.uniform(-10, 10, (60, d))).astype(np.float32))
        hi = mo.quantize_bf16(Q)
        lo = mo.quantize_bf16((Q - hi).astype(np.float32))
        # float32 evaluation of the expanded form on the two bfloat16 terms
        qt = torch.from_numpy(Q)
        ct = torch.from_numpy(C.astype(np.float32))
        dot = torch.from_numpy(hi.astype(np.float32)) @ ct.T + \
            torch.from_numpy(lo.astype(np.float32)) @ ct.T
        s = ((qt * qt).sum(1)[:, None] + (ct * ct).sum(1)[None, :] - 2 * dot).double().numpy()
        exact = mo.pairwise(Q.astype(np.float64), C)
        for i in range(Q.shape[0]):
            assert np.all(np.abs(s[i] - exact[i]) <= oc.screened_bound(Q[i], C))


# ------------------------------------------------------------ range search

def _ball(X, q, radius):
    """Points within radius of q from scipy's kd-tree, ranked by (d, id)."""
    tree = cKDTree(X.astype(np.float64))
    idx = np.array(sorted(tree.query_ball_point(q, radius)), dtype=np.int64)
    d = np.sqrt(((X[idx].astype(np.float64) - q) ** 2).sum(1)) if idx.size else np.zeros(0)
    order = np.lexsort((idx, d))
    return idx[order], d[order]


def test_range_search_with_every_prototype_in_the_ball_is_exhaustive():
    g = np.random.default_rng(21)
    X = g.standard_normal((400, 4)).astype(np.float32)
    ix = mo.build(X, [(4, 12), (1, 6)], 4, seed=2)
    for q in g.standard_normal((6, 4)):
        radius = 1.3
        # a radius that contains every prototype of every level: the search
        # reaches every leaf, so it answers the query exactly
        big = 50.0
        ids, dist, count = mo.range_query_one(ix, q, big, 400, 1000)
        assert count == 400
        ids, dist, count = mo.range_query_one(ix, q, radius, 400, 1000)
        b_ids, b_d = _ball(X, q, radius)
        # prototypes farther than the radius cut their points off: a subset
        assert set(ids[ids >= 0].tolist()) <= set(b_ids.tolist())
        assert count == int(np.sum(ids >= 0))


def test_range_search_on_one_to_one_index_is_exact():
    # one prototype per item at every level (the exact configuration of
    # Section 5): every point's ancestors are the point itself, so the
    # search returns exactly the ball
    g = np.random.default_rng(22)
    X = g.standard_normal((120, 3)).astype(np.float32)
    ix = mo.build(X, [(4, 30), (2, 60)], 3, seed=5)
    for q in g.standard_normal((8, 3)):
        for radius in (0.4, 0.9, 1.7):
            ids, dist, count = mo.range_query_one(ix, q, radius, 200, 1000)
            b_ids, b_d = _ball(X, q, radius)
            assert count == b_ids.size
            assert np.array_equal(ids[:count], b_ids)
            np.testing.assert_allclose(dist[:count], b_d, rtol=1e-12)
    # a data point at radius 0 finds itself
    ids, dist, count = mo.range_query_one(ix, X[17].astype(np.float64), 0.0, 5, 1000)
    assert count == 1 and ids[0] == 17 and dist[0] == 0.0


def test_range_search_is_monotone_and_capped():
    g = np.random.default_rng(23)
    X = g.standard_normal((600, 5)).astype(np.float32)
    ix = mo.build(X, [(6, 10), (1, 8)], 4, seed=3)
    q = g.standard_normal(5)
    prev = set()
    for radius in (0.5, 1.0, 1.5, 2.5, 4.0):
        ids, dist, count = mo.range_query_one(ix, q, radius, 600, 1000)
        cur = set(ids[ids >= 0].tolist())
        assert prev <= cur
        assert np.all(dist[:count] <= radius)
        prev = cur
    # the per-level cap keeps the nearest prototypes: cap 1 follows the
    # greedy path of the k-NN descent
    ids1, _, _ = mo.range_query_one(ix, q, 50.0, 600, 1)
    _, _, tr = mo.query_one(ix, q, 3, 1, trace=True)
    leaf = set(ix.children(0)[tr.selected[-1][0]].tolist())
    assert set(ids1[ids1 >= 0].tolist()) == leaf


# -------------------------------------------- point query and relocation

def test_lloyd_group_smaller_than_k_keeps_every_member():
    # a group of 3 points with k = 5: the members are the first three
    # prototypes; copies of the first two follow, lose every tie and stay
    P = np.array([[0.0, 1.0], [2.0, -1.0], [5.0, 5.0]])
    res = mo.lloyd(P, 5, 4)
    np.testing.assert_array_equal(res.centroids, P[[0, 1, 2, 0, 1]])
    np.testing.assert_array_equal(res.labels, [0, 1, 2])
    np.testing.assert_array_equal(res.inertia, np.zeros(4))


def test_point_query_on_one_to_one_level_finds_every_point():
    # one level with k = group size: the prototypes are the points, so the
    # nearest prototype of a data point is its own and the scan finds it
    g = np.random.default_rng(21)
    X = g.standard_normal((60, 2)).astype(np.float32)
    ix = mo.build(X, [(3, 20)], 3, seed=2)
    ans, leaf, match = mo.exhaustive_point_search(ix)
    assert np.array_equal(ans, np.arange(60))
    assert np.array_equal(match, np.arange(60))
    assert np.array_equal(leaf, ix.parents[0])


def test_point_query_is_the_greedy_descent_then_a_leaf_scan():
    X, ix = _small_index()
    g = np.random.default_rng(22)
    Q = np.concatenate([X[:25].astype(np.float64), g.standard_normal((15, X.shape[1]))])
    n_match = 0
    for q in Q:
        a, d, leaf, match = mo.point_query_one(ix, q)
        ids, dist, tr = mo.query_one(ix, q, 1, 1, trace=True)
        assert leaf == tr.selected[-1][0]
        assert a == ids[0] and d == dist[0]
        pts = [i for i in range(X.shape[0]) if ix.parents[0][i] == leaf]
        eq = [i for i in pts if all(float(X[i, c]) == q[c] for c in range(X.shape[1]))]
        assert match == (min(eq) if eq else -1)
        n_match += match >= 0
    assert n_match >= 1  # some data rows are found, so the match branch is exercised


def _cloud_errors(npc, overlap):
    c = datagen.eight_clouds(npc, overlap, seed=42)
    ix = mo.build(c.X, mo.plan_levels(8 * npc, 16, 8), 30, seed=1)
    ans, _, match = mo.exhaustive_point_search(ix)
    wrong = (ans < 0) | (c.labels[np.maximum(ans, 0)] != c.labels)
    return wrong.mean(), (match < 0).mean()


def test_cloud_benchmark_error_rates():
    # Section 4.2 with lengthGroup 16 and nCentroids 8 (1,600 points, seven
    # centroid levels): with well separated clouds nearly every point query
    # answers with a point of the query's own cloud (the no-overlap table
    # gives at most 0.11 %), and more overlap gives more errors.  The answer
    # is rarely the query itself: an exact-match reading of the error rate
    # would be far from the paper's figures.
    none, none_miss = _cloud_errors(200, "none")
    moderate, _ = _cloud_errors(200, "moderate")
    severe, _ = _cloud_errors(200, "severe")
    assert none <= 0.002
    assert none < moderate < severe
    assert none_miss > 0.5


def test_relocation_worked_example():
    # groups in the old order: g0 = [4, 2], g1 = [0, 5], g2 = [1, 3]; k0 = 2
    # so leaf p belongs to group p // 2.  Point 0 (wrong, leaf 1) joins g0;
    # point 2 (wrong, leaf 5) joins g2; point 5 (wrong, leaf 2) is already in
    # g1; point 3 (wrong, no leaf) stays.
    perm = np.array([4, 2, 0, 5, 1, 3])
    off = np.array([0, 2, 4, 6])
    leaf = np.array([1, 0, 5, -1, 0, 2])
    wrong = np.array([1, 0, 1, 1, 0, 1], dtype=bool)
    p2, o2 = mo.relocate(perm, off, 2, leaf, wrong)
    assert p2.tolist() == [4, 0, 5, 1, 3, 2] and o2.tolist() == [0, 2, 3, 6]
    # emptying g1 drops it
    leaf = np.array([0, 0, 0, 0, 0, 4])
    wrong = np.array([1, 0, 0, 0, 0, 1], dtype=bool)
    p3, o3 = mo.relocate(perm, off, 2, leaf, wrong)
    assert p3.tolist() == [4, 2, 0, 1, 3, 5] and o3.tolist() == [0, 3, 6]
    # nothing wrong: nothing moves
    p4, o4 = mo.relocate(perm, off, 2, leaf, np.zeros(6, dtype=bool))
    assert p4.tolist() == perm.tolist() and o4.tolist() == off.tolist()


def test_build_on_given_groups():
    # explicit group boundaries replace the split, including groups smaller
    # than k; the groups' prototypes are their own k-means
    g = np.random.default_rng(23)
    X = g.standard_normal((40, 2)).astype(np.float32)
    perm = g.permutation(40)
    off = np.array([0, 3, 20, 22, 40])
    ix = mo.build(X, [(4, 4), (2, 4)], 5, seed=0, perm=perm, group_off=off)
    for c in range(4):
        members = perm[off[c]:off[c + 1]]
        res = mo.lloyd(X[members], 4, 5)
        np.testing.assert_array_equal(ix.protos[0][4 * c:4 * c + 4], res.centroids)
        assert np.array_equal(ix.parents[0][members], 4 * c + res.labels)
    with pytest.raises(ValueError):
        mo.build(X, [(4, 4)], 5, seed=0, perm=perm, group_off=np.array([0, 3, 3, 22, 40]))


# ------------------------------------------------------- dynamic insertion

def test_insertion_skips_childless_prototypes_above_level_one():
    # level 1: prototypes at 0 and 10 (children 0, 1 and 9, 11); level 2:
    # prototype 0 at 4 holds both, prototype 1 at 5 holds nothing.  A point
    # at 5.2 is nearest to the empty one; insertion passes it by and joins
    # the nearer level-1 prototype under prototype 0, while the point query
    # (which does not skip) reaches no leaf.
    X = np.array([[0.0], [1.0], [9.0], [11.0]])
    ix = mo.index_from_arrays(X, [np.array([[0.0], [10.0]]), np.array([[4.0], [5.0]])],
                              [np.array([0, 0, 1, 1]), np.array([0, 0])])
    assert mo.insertion_leaf(ix, np.array([5.2])) == 1
    assert mo.point_query_one(ix, np.array([5.2]))[2] == -1


def _insert_case(seed=31):
    g = np.random.default_rng(seed)
    X = (g.standard_normal((400, 3)) + g.integers(-6, 6, (400, 1))).astype(np.float32)
    ix = mo.build(X, [(10, 8), (2, 10)], 6, seed=4)
    Xn = (g.standard_normal((60, 3)) * 2).astype(np.float32)
    return X, ix, Xn


def test_insertion_without_rebuild_places_points_where_their_query_leads():
    X, ix, Xn = _insert_case()
    new, leaves, rebuilt = mo.insert(ix, Xn, max_leaf=0)
    assert rebuilt == []
    # nothing moves but the new rows, which take the next ids
    for a, b in zip(new.protos, ix.protos):
        assert np.array_equal(a, b)
    assert np.array_equal(new.parents[0][:400], ix.parents[0])
    assert np.array_equal(new.parents[0][400:], leaves)
    # each new point joins the level-0 group of its leaf, after its members
    k0 = 8
    for g in range(10):
        members = new.perm0[new.group_off0[g]:new.group_off0[g + 1]]
        old = ix.perm0[ix.group_off0[g]:ix.group_off0[g + 1]]
        assert np.array_equal(members[:old.size], old)
        assert np.array_equal(members[old.size:], 400 + np.nonzero(leaves // k0 == g)[0])
    # where the point query walks the same path, it finds the inserted point
    found = 0
    for j, x in enumerate(Xn):
        a, d, leaf, match = mo.point_query_one(new, x)
        if leaf == leaves[j]:
            assert match == 400 + j and d == 0.0
            found += 1
    assert found > 40


def test_local_rebuild_is_lloyd_from_the_current_prototypes():
    X, ix, Xn = _insert_case()
    new0, leaves, _ = mo.insert(ix, Xn, max_leaf=0)
    sizes = np.bincount(new0.parents[0], minlength=80)
    limit = int(np.sort(sizes)[-3])  # a few leaves exceed it
    new, leaves2, rebuilt = mo.insert(ix, Xn, max_leaf=limit, iters=5)
    assert np.array_equal(leaves, leaves2)
    expect = sorted({p // 8 for p in np.nonzero(sizes > limit)[0]})
    assert rebuilt == expect and len(rebuilt) >= 1
    data = np.concatenate([X, Xn]).astype(np.float64)
    for g in range(10):
        sl = slice(8 * g, 8 * g + 8)
        members = new.perm0[new.group_off0[g]:new.group_off0[g + 1]]
        if g in rebuilt:
            res = mo.lloyd(data[members], 8, 5, init=ix.protos[0][sl])
            assert np.array_equal(new.protos[0][sl], res.centroids)
            assert np.array_equal(new.parents[0][members], 8 * g + res.labels)
        else:
            assert np.array_equal(new.protos[0][sl], ix.protos[0][sl])
            assert np.array_equal(new.parents[0][members], new0.parents[0][members])
    # the levels above keep their structure
    assert np.array_equal(new.protos[1], ix.protos[1])
    assert np.array_equal(new.parents[1], ix.parents[1])


# ------------------------------------------------------- k-means++ seeding

def test_uniform01_is_the_splitmix64_output():
    keys = mo.splitmix64_keys(12345, 5)
    for i in range(5):
        assert mo.uniform01(12345, i) == float(int(keys[i]) >> 11) * 2.0 ** -53
    assert 0.0 <= mo.uniform01(0, 2 ** 45) < 1.0


def test_kmeanspp_picks_distinct_members_then_repeats():
    g = np.random.default_rng(40)
    P = g.standard_normal((12, 3))
    s = mo.kmeanspp_seeds(P, 12, seed=3, level=1, chunk=0)
    assert sorted(s.tolist()) == list(range(12))  # every D^2 > 0 until chosen
    s2 = mo.kmeanspp_seeds(P[:4], 7, seed=3, level=1, chunk=0)
    assert sorted(s2[:4].tolist()) == [0, 1, 2, 3]  # then D^2 = 0 everywhere: uniform
    # identical points: every pick after the first is uniform
    same = np.ones((5, 2))
    s3 = mo.kmeanspp_seeds(same, 3, seed=9, level=2, chunk=4)
    tag = mo.KMEANSPP_LEVEL_STRIDE * 2 + 4 * 3
    assert s3.tolist() == [int(mo.uniform01(9, tag + t) * 5) for t in range(3)]


def test_kmeanspp_draws_with_probability_proportional_to_squared_distance():
    # four points on a line; over many seeds the second pick given the
    # first follows D^2 / sum D^2
    P = np.array([[0.0], [1.0], [3.0], [7.0]])
    trials = 6000
    counts = np.zeros((4, 4))
    for seed in range(trials):
        s = mo.kmeanspp_seeds(P, 2, seed=seed, level=1, chunk=0)
        counts[s[0], s[1]] += 1
    for a in range(4):
        row = counts[a]
        d2 = (P[:, 0] - P[a, 0]) ** 2
        p = d2 / d2.sum()
        nrow = row.sum()
        assert abs(nrow / trials - 0.25) < 0.03  # the first pick is uniform
        sd = np.sqrt(nrow * p * (1 - p)) + 1e-9
        assert np.all(np.abs(row - nrow * p) <= 5 * sd), (a, row, nrow * p)


def test_build_with_kmeanspp_starts_each_group_from_its_seeds():
    g = np.random.default_rng(41)
    X = (g.standard_normal((300, 2)) + g.integers(-5, 5, (300, 1))).astype(np.float32)
    ix = mo.build(X, [(3, 6), (1, 4)], 0, seed=8, init="kmeans++")
    items = X[mo.permutation(8, 300)].astype(np.float64)
    off = mo.chunk_offsets(300, 3)
    for c in range(3):
        pts = items[off[c]:off[c + 1]]
        seeds = mo.kmeanspp_seeds(pts, 6, 8, 1, c)
        np.testing.assert_array_equal(ix.protos[0][6 * c:6 * c + 6], pts[seeds])
    with pytest.raises(ValueError):
        mo.build(X, [(3, 6)], 0, seed=8, init="kmeans++", metric="l1")
