"""Parity of the HIP path with the FP64 oracle, called through the C ABI.

Tolerance (stated for the plain FP32 form): every returned distance within
1e-5 relative of the oracle's float64 distance for the same id; ids equal
position by position except where the two ids' distances are within 1e-5
relative (near-ties); k-means labels equal except where the oracle's two
nearest prototypes are within 1e-5 relative; centroids within one float32
ulp of the float64 mean rounded to float32; inertia within 1e-6 relative.
"""
import numpy as np
import pytest

import datagen
from oracle import compare as oc
from oracle import mask_oracle as mo
from tests.gpu_helpers import check_query_against_oracle, dev, host, oracle_index_from_gpu

pytestmark = pytest.mark.gpu

REL = 1e-5


@pytest.fixture(scope="module")
def pk():
    import torch
    assert torch.cuda.is_available()
    import paper_2208_02734_amd as pk
    pk.lib()  # fails loudly when the HIP library is missing
    return pk


def _mixture(n, d, n_comp, seed, nq=0):
    mix = datagen.mixture_params(seed, n_comp, d, sigma_mode="loguniform", sigma_low=0.1,
                                 sigma_high=3.0)
    X = datagen.sample_mixture(mix, n, seed + 1)
    Q = datagen.sample_mixture(mix, nq, seed + 2) if nq else None
    return X, Q


# ------------------------------------------------------------------ P2 ---

@pytest.mark.parametrize("d", [16, 10, 96, 128, 200])
def test_one_lloyd_step_matches_oracle(pk, d):
    n, C, k = 3001, 3, 50
    X, _ = _mixture(n, d, 40, seed=100 + d)
    Xd = dev(X)
    # a^0 under the first k items of each group
    _, lab0, _ = pk.mask_kmeans(Xd, C, k, 0)
    # C_1 and I_0
    cent1, _, inert = pk.mask_kmeans(Xd, C, k, 1)
    lab0, cent1, inert = host(lab0), host(cent1), host(inert)
    off = mo.chunk_offsets(n, C)
    for c in range(C):
        pts = X[off[c]:off[c + 1]].astype(np.float64)
        init = pts[:k]
        olab, onew, oin = mo.lloyd_step(pts, init)
        D = mo.pairwise(pts, init)
        glab = lab0[off[c]:off[c + 1]] - c * k
        diff = np.nonzero(glab != olab)[0]
        for i in diff:  # only near-ties may differ
            a, b = D[i, glab[i]], D[i, olab[i]]
            assert abs(a - b) <= REL * max(a, b), (c, i, a, b)
        assert diff.size <= max(2, pts.shape[0] // 1000)
        assert abs(inert[0, c] - oin) <= 1e-6 * oin
        # prototypes whose members agree: within one float32 ulp
        bad = set(glab[diff].tolist()) | set(olab[diff].tolist())
        for j in range(k):
            if j in bad:
                continue
            ref = onew[j].astype(np.float32)
            got = cent1[c * k + j]
            ulp = np.spacing(np.abs(ref)).astype(np.float32)
            assert np.all(np.abs(got - ref) <= ulp), (c, j)


def test_lloyd_iterations_invariants(pk):
    n, d, C, k, T = 20_000, 16, 10, 100, 15
    X, _ = _mixture(n, d, 50, seed=7)
    cent, lab, inert = pk.mask_kmeans(dev(X), C, k, T)
    cent, lab, inert = host(cent), host(lab), host(inert)
    # inertia never increases (float32 prototypes are the only slack)
    assert np.all(inert[1:] <= inert[:-1] * (1 + 1e-6))
    # final labels are the nearest prototypes of their group
    off = mo.chunk_offsets(n, C)
    for c in range(C):
        pts = X[off[c]:off[c + 1]]
        D = mo.pairwise(pts, cent[c * k:(c + 1) * k])
        g = lab[off[c]:off[c + 1]] - c * k
        assert np.all((g >= 0) & (g < k))
        best = D.min(axis=1)
        assert np.all(D[np.arange(pts.shape[0]), g] <= best * (1 + REL))


def test_inertia_matches_oracle_trajectory(pk):
    # on separated data the whole trajectory is reproducible
    X = _separated(5)
    init = np.ascontiguousarray(X[::200][:8])  # one starting prototype per cloud
    cent, lab, inert = pk.mask_kmeans(dev(X), 1, 8, 6, init=dev(init))
    res = mo.lloyd(X, 8, 6, init=init)
    np.testing.assert_allclose(host(inert)[:, 0], res.inertia, rtol=1e-6)
    assert np.array_equal(host(lab), res.labels)
    np.testing.assert_allclose(host(cent), res.centroids, rtol=1e-6, atol=1e-5)


# ------------------------------------------------------------------ P3 ---

def _separated(seed, n_per=200, clouds=8):
    """8 well-separated 2-D Gaussian clouds, 200 points each (the shape of
    the paper's no-overlap synthetic set, Section 4.1)."""
    g = np.random.default_rng(seed)
    ang = np.arange(clouds) * 2 * np.pi / clouds
    means = np.stack([100 * np.cos(ang), 100 * np.sin(ang)], 1)
    return np.concatenate([m + g.standard_normal((n_per, 2)) * 3 for m in means]).astype(np.float32)


def test_full_build_matches_oracle_on_separated_clouds(pk):
    # seed 5: every assignment of the oracle build has a relative gap > 1e-3
    X = _separated(5)
    levels = mo.plan_levels(1600, 16, 8)  # Algorithm 1 schedule, 7 levels
    oix = mo.build(X, levels, 10, seed=5)
    gix = pk.mask_build(dev(X), levels, iters=10, seed=5)
    for lev in range(1, len(levels) + 1):
        P, par = gix.export_level(lev)
        assert np.array_equal(par, oix.parents[lev - 1]), lev
        np.testing.assert_allclose(P, oix.protos[lev - 1], rtol=1e-5, atol=1e-4)
    gix.free()


def test_permutation_and_chunks_match_oracle(pk):
    n, C, k = 1003, 7, 5
    X, _ = _mixture(n, 8, 10, seed=3)
    gix = pk.mask_build(dev(X), [(C, k)], iters=2, seed=0xDEADBEEF12345)
    _, par = gix.export_level(1)
    pi = mo.permutation(0xDEADBEEF12345, n)
    off = mo.chunk_offsets(n, C)
    chunk_of = np.empty(n, dtype=np.int64)
    for c in range(C):
        chunk_of[pi[off[c]:off[c + 1]]] = c
    assert np.array_equal(par // k, chunk_of)


def test_user_permutation(pk):
    import torch
    n, C, k = 600, 4, 6
    X, _ = _mixture(n, 4, 6, seed=4)
    perm = np.random.default_rng(0).permutation(n).astype(np.int32)
    gix = pk.mask_build(dev(X), [(C, k)], iters=3, perm=torch.from_numpy(perm).cuda())
    _, par = gix.export_level(1)
    off = mo.chunk_offsets(n, C)
    for c in range(C):
        assert np.all(par[perm[off[c]:off[c + 1]]] // k == c)


# ------------------------------------------------------------------ P1 ---

@pytest.mark.parametrize("r,k", [(1, 1), (3, 10), (8, 10), (40, 25)])
def test_query_on_oracle_built_index(pk, r, k):
    n, d = 4000, 24
    X, Q = _mixture(n, d, 30, seed=11, nq=150)
    levels = [(8, 50), (2, 20), (1, 10)]
    oix = mo.build(X, levels, 8, seed=2)
    gix = pk.mask_import(dev(X), levels, oix.protos, oix.parents)
    ids, dist, sel = pk.mask_query(gix, dev(Q), k, r, debug=True)
    n_chk, n_rep, fails = check_query_against_oracle(oix, X, Q, k, r, host(ids), host(dist),
                                                     host(sel))
    assert not fails, fails[:3]
    gix.free()


@pytest.mark.parametrize("d", [16, 7, 128])
def test_query_on_gpu_built_index(pk, d):
    n = 6000
    X, Q = _mixture(n, d, 40, seed=20 + d, nq=120)
    levels = [(6, 100), (1, 30)]
    gix = pk.mask_build(dev(X), levels, iters=10, seed=9)
    oix = oracle_index_from_gpu(X, gix)
    for r, k in [(1, 5), (5, 10), (30, 10)]:
        ids, dist, sel = pk.mask_query(gix, dev(Q), k, r, debug=True)
        _, _, fails = check_query_against_oracle(oix, X, Q, k, r, host(ids), host(dist),
                                                 host(sel))
        assert not fails, (r, k, fails[:3])
    gix.free()


def test_probe_all_is_exact_knn(pk):
    n, d = 3000, 32
    X, Q = _mixture(n, d, 20, seed=31, nq=64)
    gix = pk.mask_build(dev(X), [(6, 50), (1, 30)], iters=5, seed=1)
    ids, dist = pk.mask_query(gix, dev(Q), 10, 512)
    tids, tdist = mo.exact_knn(X, Q, 10)
    true = oc.true_distances(X, Q, host(ids).astype(np.int64))
    res = oc.check_knn(host(ids), host(dist), tids, tdist, true, REL)
    assert res.ok, res.messages


@pytest.mark.parametrize("k", [10, 500, 1000])
def test_many_rounds_at_the_data_layer(pk, k):
    # 40,000 candidates at the data layer: the key buffer is filled and
    # selected many times, and most later rounds add few or no keys (the
    # threshold is tight), so rounds that end without a selection follow
    # each other; probing every leaf must still give the exact k nearest
    X, Q = _mixture(40_000, 16, 30, seed=71, nq=24)
    gix = pk.mask_build(dev(X), [(1, 8)], iters=3, seed=4)
    ids, dist = pk.mask_query(gix, dev(Q), k, 8)
    tids, tdist = mo.exact_knn(X, Q, k)
    true = oc.true_distances(X, Q, host(ids).astype(np.int64))
    res = oc.check_knn(host(ids), host(dist), tids, tdist, true, REL)
    assert res.ok, res.messages
    gix.free()


def test_one_to_one_ratio_is_exact(pk):
    # one prototype per item at every level (Section 5: exact search)
    n, d, k = 960, 6, 4
    X, Q = _mixture(n, d, 10, seed=41, nq=40)
    gix = pk.mask_build(dev(X), [(8, 120), (4, 240)], iters=3, seed=3)
    ids, dist = pk.mask_query(gix, dev(Q), k, k)
    tids, tdist = mo.exact_knn(X, Q, k)
    true = oc.true_distances(X, Q, host(ids).astype(np.int64))
    assert oc.check_knn(host(ids), host(dist), tids, tdist, true, REL).ok


# ---------------------------------------------------------- edge cases ---

def test_padding_when_candidates_run_out(pk):
    n = 400
    X, Q = _mixture(n, 8, 5, seed=51, nq=10)
    gix = pk.mask_build(dev(X), [(4, 50), (1, 5)], iters=3, seed=2)
    ids, dist = pk.mask_query(gix, dev(Q), 100, 1)
    ids, dist = host(ids), host(dist)
    oix = oracle_index_from_gpu(X, gix)
    for i in range(Q.shape[0]):
        nv = int((ids[i] >= 0).sum())
        assert nv < 100
        assert np.all(ids[i, nv:] == -1) and np.all(np.isinf(dist[i, nv:]))
        o_ids, _ = mo.query_one(oix, Q[i], 100, 1)
        assert int((o_ids >= 0).sum()) == nv


def test_duplicates_break_ties_by_lower_id(pk):
    g = np.random.default_rng(61)
    base = g.standard_normal((100, 5)).astype(np.float32)
    X = np.concatenate([base, base, base])  # each point three times
    Q = base[:20] + np.float32(0.01)
    gix = pk.mask_build(dev(X), [(3, 20), (1, 4)], iters=4, seed=4)
    ids, dist = pk.mask_query(gix, dev(Q), 6, 4)
    oix = oracle_index_from_gpu(X, gix)
    o_ids, o_dist = mo.query(oix, Q, 6, 4)
    true = oc.true_distances(X, Q, host(ids).astype(np.int64))
    res = oc.check_knn(host(ids), host(dist), o_ids, o_dist, true, REL)
    assert res.ok, res.messages
    # no near-ties besides the exact duplicates: the ids match position by position
    assert np.array_equal(host(ids), o_ids)
    # exactly equal distances come out in increasing id order
    ids = host(ids)
    dist = host(dist)
    for i in range(ids.shape[0]):
        for j in range(5):
            if dist[i, j] == dist[i, j + 1]:
                assert ids[i, j] < ids[i, j + 1]


def test_query_distance_zero_is_exact(pk):
    X, _ = _mixture(2000, 12, 10, seed=71)
    gix = pk.mask_build(dev(X), [(4, 40), (1, 10)], iters=5, seed=6)
    ids, dist = pk.mask_query(gix, dev(X[:50]), 1, 10)
    d = host(dist)[:, 0]
    hit = host(ids)[:, 0] == np.arange(50)
    assert np.all(d[hit] == 0.0)
    assert hit.mean() > 0.9


def test_empty_query_batch_and_bad_arguments(pk):
    import torch
    X, _ = _mixture(500, 4, 4, seed=81)
    gix = pk.mask_build(dev(X), [(2, 10)], iters=2, seed=1)
    ids, dist = pk.mask_query(gix, torch.zeros((0, 4), device="cuda"), 5, 2)
    assert ids.shape == (0, 5)
    with pytest.raises(pk.MaskError):
        pk.mask_query(gix, torch.zeros((3, 5), device="cuda"), 5, 2)  # wrong dim
    with pytest.raises(pk.MaskError):
        pk.mask_query(gix, torch.zeros((3, 4), device="cuda"), 0, 2)
    with pytest.raises(pk.MaskError):
        pk.mask_query(gix, torch.zeros((3, 4), device="cuda"), 5, 2049)


def test_single_level_index(pk):
    X, Q = _mixture(3000, 20, 15, seed=91, nq=40)
    gix = pk.mask_build(dev(X), [(1, 60)], iters=8, seed=2)
    oix = oracle_index_from_gpu(X, gix)
    ids, dist, sel = pk.mask_query(gix, dev(Q), 10, 6, debug=True)
    _, _, fails = check_query_against_oracle(oix, X, Q, 10, 6, host(ids), host(dist), host(sel))
    assert not fails, fails[:3]


def test_batch_invariance(pk):
    X, Q = _mixture(8000, 32, 30, seed=101, nq=300)
    gix = pk.mask_build(dev(X), [(8, 100), (1, 40)], iters=6, seed=3)
    ids, dist = pk.mask_query(gix, dev(Q), 10, 7)
    for lo, hi in [(0, 1), (17, 18), (50, 173), (299, 300)]:
        i2, d2 = pk.mask_query(gix, dev(Q[lo:hi]), 10, 7)
        assert np.array_equal(host(i2), host(ids)[lo:hi])
        assert np.array_equal(host(d2), host(dist)[lo:hi])
    # permuted batch
    p = np.random.default_rng(0).permutation(300)
    i3, d3 = pk.mask_query(gix, dev(Q[p]), 10, 7)
    assert np.array_equal(host(i3), host(ids)[p])
    assert np.array_equal(host(d3), host(dist)[p])


def test_query_identical_across_lds_classes_and_runs(pk):
    # Selections that need several rounds and several radix passes: the
    # result must not depend on the LDS class (forced through the ragged
    # entry point's r_max) nor change between runs.
    import torch
    X, Q = _mixture(60_000, 64, 120, seed=107, nq=3000)
    gix = pk.mask_build(dev(X), [(20, 300), (1, 100)], iters=6, seed=4)
    ids, dist = pk.mask_query(gix, dev(Q), 10, 64)
    ids, dist = host(ids), host(dist)
    for _ in range(2):
        i2, d2 = pk.mask_query(gix, dev(Q), 10, 64)
        assert np.array_equal(host(i2), ids)
        assert np.array_equal(host(d2), dist)
    ks = torch.full((3000,), 10, dtype=torch.int32)
    rs = torch.full((3000,), 64, dtype=torch.int32)
    for r_max in (200, 400, 600):  # the 512 class as r = 64, and the 2048 class
        i3, d3, off = pk.mask_query_ragged(gix, dev(Q), ks, rs, k_max=10, r_max=r_max)
        assert np.array_equal(host(i3).reshape(3000, 10), ids), r_max
        assert np.array_equal(host(d3).reshape(3000, 10), dist), r_max
    # k_max above 512 with beams of at most 512: the class with small
    # per-prototype arrays and a 2,048-key output
    i3, d3, off = pk.mask_query_ragged(gix, dev(Q), ks, rs, k_max=600, r_max=64)
    assert np.array_equal(host(i3).reshape(3000, 10), ids)
    assert np.array_equal(host(d3).reshape(3000, 10), dist)
    gix.free()
    # the precision form: its re-rank set does not depend on the class either
    g16 = pk.mask_build(dev(X), [(20, 300), (1, 100)], iters=6, seed=4, precision="bf16")
    ids, dist = (host(t) for t in pk.mask_query(g16, dev(Q), 10, 64))
    for k_max, r_max in ((10, 200), (10, 400), (10, 600), (600, 64)):
        i3, d3, off = pk.mask_query_ragged(g16, dev(Q), ks, rs, k_max=k_max, r_max=r_max)
        assert np.array_equal(host(i3).reshape(3000, 10), ids), (k_max, r_max)
        assert np.array_equal(host(d3).reshape(3000, 10), dist), (k_max, r_max)
    g16.free()


def test_build_is_deterministic(pk):
    X, _ = _mixture(20_000, 16, 50, seed=111)
    levels = [(10, 100), (1, 50)]
    a = pk.mask_build(dev(X), levels, iters=10, seed=1)
    b = pk.mask_build(dev(X), levels, iters=10, seed=1)
    for lev in (1, 2):
        Pa, pa = a.export_level(lev)
        Pb, pb = b.export_level(lev)
        assert np.array_equal(pa, pb) and np.array_equal(Pa, Pb)


# ------------------------------------------------------------------ L1 ---

def test_one_lloyd_step_l1_matches_oracle(pk):
    # k-medians: labels by sum |x - c|, update = per-dimension lower median
    n, d, C, k = 2001, 12, 3, 30
    X, _ = _mixture(n, d, 20, seed=131)
    Xd = dev(X)
    _, lab0, _ = pk.mask_kmeans(Xd, C, k, 0, metric="l1")
    cent1, _, inert = pk.mask_kmeans(Xd, C, k, 1, metric="l1")
    lab0, cent1, inert = host(lab0), host(cent1), host(inert)
    off = mo.chunk_offsets(n, C)
    for c in range(C):
        pts = X[off[c]:off[c + 1]].astype(np.float64)
        olab, onew, oin = mo.lloyd_step(pts, pts[:k], "l1")
        glab = lab0[off[c]:off[c + 1]] - c * k
        D = mo.pairwise(pts, pts[:k], "l1")
        diff = np.nonzero(glab != olab)[0]
        for i in diff:
            a, b = D[i, glab[i]], D[i, olab[i]]
            assert abs(a - b) <= 1e-12 * max(a, b), (c, i, a, b)
        assert abs(inert[0, c] - oin) <= 1e-9 * oin
        bad = set(glab[diff].tolist()) | set(olab[diff].tolist())
        for j in range(k):
            if j not in bad:
                # the lower median is a data value: exact equality
                assert np.array_equal(cent1[c * k + j], onew[j].astype(np.float32)), (c, j)


def test_full_l1_build_matches_oracle_on_separated_clouds(pk):
    # seed 58: every L1 assignment of the oracle build has a relative gap > 1e-4
    X = _separated(58)
    levels = mo.plan_levels(1600, 16, 8)
    oix = mo.build(X, levels, 6, seed=58, metric="l1")
    gix = pk.mask_build(dev(X), levels, iters=6, seed=58, metric="l1")
    for lev in range(1, len(levels) + 1):
        P, par = gix.export_level(lev)
        assert np.array_equal(par, oix.parents[lev - 1]), lev
        assert np.array_equal(P, oix.protos[lev - 1].astype(np.float32)), lev
    gix.free()


def test_l1_query_matches_oracle(pk):
    X, Q = _mixture(5000, 20, 30, seed=141, nq=80)
    gix = pk.mask_build(dev(X), [(5, 60), (1, 20)], iters=6, seed=3, metric="l1")
    oix = oracle_index_from_gpu(X, gix, metric="l1")
    for r, k in [(1, 5), (6, 10)]:
        ids, dist, sel = pk.mask_query(gix, dev(Q), k, r, debug=True)
        _, _, fails = check_query_against_oracle(oix, X, Q, k, r, host(ids), host(dist),
                                                 host(sel))
        assert not fails, (r, k, fails[:3])
    # probe-all is exact L1 kNN
    ids, dist = pk.mask_query(gix, dev(Q), 10, 512)
    tids, tdist = mo.exact_knn(X, Q, 10, metric="l1")
    true = oc.true_distances(X, Q, host(ids).astype(np.int64), "l1")
    assert oc.check_knn(host(ids), host(dist), tids, tdist, true, REL).ok


def test_per_level_beams(pk):
    X, Q = _mixture(8000, 40, 40, seed=151, nq=80)
    gix = pk.mask_build(dev(X), [(8, 80), (1, 64), (1, 8)], iters=6, seed=6)
    # uniform beams are the uniform descent, bit for bit
    i1, d1 = pk.mask_query(gix, dev(Q), 10, 6)
    i2, d2 = pk.mask_query_beams(gix, dev(Q), 10, [6, 6, 6])
    assert np.array_equal(host(i1), host(i2)) and np.array_equal(host(d1), host(d2))
    # a narrowing beam against the oracle's descent with the same beams
    oix = oracle_index_from_gpu(X, gix)
    beams = [2, 5, 12]
    ids, dist = pk.mask_query_beams(gix, dev(Q), 10, beams)
    ids, dist = host(ids).astype(np.int64), host(dist)
    o_ids = np.empty_like(ids)
    o_dist = np.empty(dist.shape)
    for i in range(Q.shape[0]):
        o_ids[i], o_dist[i] = mo.query_one(oix, Q[i], 10, beams)
    true = oc.true_distances(X, Q, ids)
    res = oc.check_knn(ids, dist, o_ids, o_dist, true, REL)
    assert res.ok, res.messages
