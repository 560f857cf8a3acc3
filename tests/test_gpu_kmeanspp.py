"""k-means++ seeding on the GPU against the FP64 oracle, called through the
C ABI.  The draws are the same counter-based SplitMix64 outputs on both
sides; a pick is an integer decided by a float64 running sum, so the picks
must agree except where the target falls within 1e-12 (relative to the sum)
of a running-sum boundary, after which that group's later picks are not
compared."""
import numpy as np
import pytest

import datagen
from oracle import mask_oracle as mo
from tests.gpu_helpers import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import torch
    assert torch.cuda.is_available()
    import paper_2208_02734_amd as pk
    pk.lib()
    return pk


def _mixture(n, d, n_comp, seed):
    mix = datagen.mixture_params(seed, n_comp, d, sigma_mode="loguniform", sigma_low=0.1,
                                 sigma_high=3.0)
    return datagen.sample_mixture(mix, n, seed + 1)


def _boundary_pick(pts, picks, t, seed, level, c, k, pick):
    """True when the GPU's pick at draw t lies on a running-sum boundary of
    the oracle's computation from the GPU's earlier picks."""
    X = pts.astype(np.float64)
    d2 = None
    for p in picks[:t]:
        diff = X - X[p][None, :]
        d = np.einsum("ij,ij->i", diff, diff)
        d2 = d if d2 is None else np.minimum(d2, d)
    u = mo.uniform01(seed, mo.KMEANSPP_LEVEL_STRIDE * level + c * k + t)
    total = d2.sum()
    run = np.cumsum(d2)
    target = u * total
    lo = run[pick - 1] if pick > 0 else 0.0
    return abs(lo - target) <= 1e-12 * total or abs(run[pick] - target) <= 1e-12 * total


def _compare(pts, gpu_picks, seed, level, c, k):
    ref = mo.kmeanspp_seeds(pts, k, seed, level, c)
    for t in range(k):
        if gpu_picks[t] != ref[t]:
            assert t > 0 and _boundary_pick(pts, gpu_picks, t, seed, level, c, k,
                                            gpu_picks[t]), (c, t, gpu_picks[t], ref[t])
            return t
    return k


@pytest.mark.parametrize("d,C,k,level", [(16, 4, 20, 1), (128, 3, 64, 2), (5, 6, 9, 3),
                                          (96, 3, 40, 1), (70, 2, 30, 2)])
def test_seeds_match_oracle(pk, d, C, k, level):
    n = 3001
    X = _mixture(n, d, 25, seed=1000 + d)
    cent, chosen = pk.mask_kmeanspp(dev(X), C, k, seed=77, level=level)
    cent, chosen = host(cent), host(chosen)
    off = mo.chunk_offsets(n, C)
    assert np.array_equal(cent, X[chosen])
    for c in range(C):
        pts = X[off[c]:off[c + 1]]
        picks = chosen[c * k:(c + 1) * k] - off[c]
        assert np.all((picks >= 0) & (picks < pts.shape[0]))
        assert _compare(pts, picks, 77, level, c, k) == k  # no boundary case expected


def test_seeds_match_oracle_when_float32_distances_overflow(pk):
    # Three clouds along the first coordinate: A spread over [-1.5e19,
    # 1.5e19], B near +3e19, C near -6e19.  The draws (seed 20) take C, then
    # B: at that draw most rows of A must fall from their distance to C to
    # their distance to B, but the FP32 sums of their BF16 screen overflow.
    # Such a row must be read exactly; settling it would keep its distance
    # to C and move the next pick.
    g = np.random.default_rng(5)
    m, d, k = 700, 96, 4
    A = g.standard_normal((m, d)).astype(np.float32)
    A[:, 0] = g.uniform(-1.5e19, 1.5e19, m)
    B = g.standard_normal((m, d)).astype(np.float32)
    B[:, 0] = 3e19 + 1e17 * g.standard_normal(m)
    C = g.standard_normal((m, d)).astype(np.float32)
    C[:, 0] = -6e19 + 1e17 * g.standard_normal(m)
    perm = g.permutation(3 * m)
    X = np.concatenate([A, B, C])[perm].astype(np.float32)
    cloud = np.repeat([0, 1, 2], m)[perm]
    ref = mo.kmeanspp_seeds(X, k, 20, 1, 0)
    assert list(cloud[ref[:3]]) == [2, 1, 0]  # the case described above
    cent, chosen = pk.mask_kmeanspp(dev(X), 1, k, seed=20, level=1)
    assert np.array_equal(host(chosen).astype(np.int64), ref)


def test_small_groups_and_identical_points(pk):
    X = _mixture(40, 4, 3, seed=1010)
    X[20:] = X[20]  # the second group: 20 identical points
    cent, chosen = pk.mask_kmeanspp(dev(X), 2, 25, seed=5, level=1)
    chosen = host(chosen)
    for c in range(2):
        pts = X[20 * c:20 * c + 20]
        ref = mo.kmeanspp_seeds(pts, 25, 5, 1, c)
        assert np.array_equal(chosen[25 * c:25 * c + 25] - 20 * c, ref)
    assert sorted(set((chosen[:20]).tolist())) == list(range(20))  # every member before repeats


def _separated(seed, n_per=200, clouds=8):
    g = np.random.default_rng(seed)
    ang = np.arange(clouds) * 2 * np.pi / clouds
    means = np.stack([100 * np.cos(ang), 100 * np.sin(ang)], 1)
    return np.concatenate([m + g.standard_normal((n_per, 2)) * 3
                           for m in means]).astype(np.float32)


def test_build_with_kmeanspp_matches_oracle(pk):
    # seed 5: every final assignment of the oracle build has a relative gap
    # above 0.1
    X = _separated(5)
    levels = mo.plan_levels(1600, 16, 8)
    oix = mo.build(X, levels, 10, seed=5, init="kmeans++")
    gix = pk.mask_build(dev(X), levels, iters=10, seed=5, init="kmeans++")
    for lev in range(1, len(levels) + 1):
        P, par = gix.export_level(lev)
        assert np.array_equal(par, oix.parents[lev - 1]), lev
        np.testing.assert_allclose(P, oix.protos[lev - 1], rtol=1e-5, atol=1e-4)
    gix.free()


def test_kmeanspp_starts_from_lower_inertia(pk):
    # the point of the seeding: on clustered data its initial prototypes
    # summarise the groups better than the first k members do
    X = _mixture(20000, 16, 40, seed=1020)
    C, k = 4, 40
    seeds, _ = pk.mask_kmeanspp(dev(X), C, k, seed=3, level=1)
    _, _, in_pp = pk.mask_kmeans(dev(X), C, k, 1, init=seeds)
    _, _, in_first = pk.mask_kmeans(dev(X), C, k, 1)
    assert host(in_pp)[0].sum() < 0.8 * host(in_first)[0].sum()


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_precision_forms_build_with_kmeanspp(pk, precision):
    X = _mixture(8000, 32, 30, seed=1030)
    levels = [(4, 50), (1, 20)]
    g = pk.mask_build(dev(X), levels, iters=4, seed=9, precision=precision, init="kmeans++")
    f = pk.mask_build(dev(X), levels, iters=0, seed=9, init="kmeans++")
    # both start from the same seeds: with no iterations the FP32 build's
    # prototypes are the seeds, which the oracle reproduces
    P0, _ = f.export_level(1)
    items = X[mo.permutation(9, 8000)]
    off = mo.chunk_offsets(8000, 4)
    for c in range(4):
        pts = items[off[c]:off[c + 1]]
        np.testing.assert_array_equal(P0[50 * c:50 * c + 50],
                                      pts[mo.kmeanspp_seeds(pts, 50, 9, 1, c)])
    ids, dist = pk.mask_query(g, dev(X[:50]), 1, 2048)
    assert np.all(host(dist)[:, 0] == 0.0)
    g.free()
    f.free()


def test_kmeanspp_on_given_groups_matches_oracle(pk):
    # seeding over ragged groups (as relocation leaves them), some smaller than k
    import torch
    X = _separated(9, n_per=60)
    n = X.shape[0]
    perm = np.random.default_rng(9).permutation(n)
    off = np.array([0, 3, 40, 41, 200, 480])
    levels = [(5, 8), (1, 6)]
    oix = mo.build(X, levels, 6, seed=4, perm=perm, group_off=off, init="kmeans++")
    gix = pk.mask_build(dev(X), levels, iters=6, seed=4, init="kmeans++", group_off=off,
                        perm=torch.from_numpy(perm.astype(np.int32)).cuda())
    for lev in (1, 2):
        P, par = gix.export_level(lev)
        assert np.array_equal(par, oix.parents[lev - 1]), lev
        np.testing.assert_allclose(P, oix.protos[lev - 1], rtol=1e-5, atol=1e-4)
    gix.free()


@pytest.mark.parametrize("d,m,C,k", [(128, 7_000, 20, 150), (7, 40_000, 55, 30),
                                     (96, 18_000, 10, 120)])
def test_seeds_at_scale_match_oracle(pk, d, m, C, k):
    # Levels whose rows take 64 MiB or more (longer tiles), on clustered data
    # where the triangle inequality skips most rows after the first draws.
    # Seeds of a group depend only on its members: the first two groups
    # seeded on their own (a small level, shorter tiles) give the same picks;
    # other tiles only regroup the FP64 sums, which could move a pick only at
    # a rounding boundary, and none occurs here.  Every group matches the
    # oracle.
    X = _mixture(m * C, d, 60, seed=1200 + d)
    ld = (d + 3) // 4 * 4
    assert m * C * ld * 4 >= 64 << 20 and 2 * m * ld * 4 < 64 << 20
    _, big = pk.mask_kmeanspp(dev(X), C, k, seed=31, level=1)
    _, small = pk.mask_kmeanspp(dev(X[:2 * m]), 2, k, seed=31, level=1)
    big, small = host(big), host(small)
    assert np.array_equal(big[:2 * k], small)
    for c in range(C):
        pts = X[c * m:(c + 1) * m]
        _compare(pts, big[c * k:(c + 1) * k] - c * m, 31, 1, c, k)


def test_seeding_row_counters(pk):
    # the device counts behind the benchmark's seeding roofline: draw 0 reads
    # and lowers every row; later draws read at most every row, and a row
    # whose D^2 fell was read
    X = _mixture(60_000, 32, 50, seed=1300)
    C, k = 6, 40
    pk.mask_timing_enable(True)
    pk.mask_kmeanspp(dev(X), C, k, seed=2, level=1)
    rep = pk.mask_timing_report()
    pk.mask_timing_enable(False)
    n = X.shape[0]
    read = rep["seeding_rows_read_level1"][0]
    exact = rep["seeding_rows_exact_level1"][0]
    low = rep["seeding_rows_lowered_level1"][0]
    assert rep["kmeanspp_level1"][0] == 1
    # draw 0 reads every row exactly; a lowered row was read exactly, and a
    # row read exactly was not ruled out by the triangle inequality
    assert n <= low <= exact <= read <= (k - 1) * n
    # clustered rows: the triangle inequality rules most of them out, and
    # the BF16 screen settles most of the rest
    assert read < 0.8 * (k - 1) * n
    assert exact - n < 0.5 * (read - n)


@pytest.mark.parametrize("n,C", [(70_001, 1), (280_000, 2)])
def test_seeds_of_groups_with_many_tiles_match_oracle(pk, n, C):
    # groups of 70,001 and 140,000 rows at d = 4 are cut into 547 and 1,094
    # tiles of 128 rows, so the pick keeps 16 and 32 tile sums per lane (the
    # variants for groups above 512 and 1,024 tiles)
    X = _mixture(n, 4, 40, seed=1030 + C)
    k = 24
    cent, chosen = pk.mask_kmeanspp(dev(X), C, k, seed=91, level=2)
    cent, chosen = host(cent), host(chosen)
    off = mo.chunk_offsets(n, C)
    assert np.array_equal(cent, X[chosen])
    for c in range(C):
        pts = X[off[c]:off[c + 1]]
        assert -(-pts.shape[0] // 128) > (512 if C == 1 else 1024)
        picks = chosen[c * k:(c + 1) * k] - off[c]
        assert np.all((picks >= 0) & (picks < pts.shape[0]))
        assert _compare(pts, picks, 91, 2, c, k) == k
