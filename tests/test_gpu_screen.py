"""The screened descent of the BF16 form: the small prototype levels are
scored for the whole query batch by one BF16 MFMA GEMM, and the descent
reads those scores.  It ranks the same BF16 prototypes as the gathered
descent with another rounding (expanded form, query split into two BF16
terms), so the two agree except at near-ties; slicing the batch to fit the
workspace changes nothing."""
import numpy as np
import pytest

import datagen
from oracle import compare as oc
from oracle import mask_oracle as mo
from tests.gpu_helpers import check_lowp_against_oracle, dev, host, oracle_index_from_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import torch
    assert torch.cuda.is_available()
    import paper_2208_02734_amd as pk
    pk.lib()
    return pk


def _mixture(n, d, n_comp, seed, nq=0):
    mix = datagen.mixture_params(seed, n_comp, d, sigma_mode="loguniform", sigma_low=0.1,
                                 sigma_high=3.0)
    X = datagen.sample_mixture(mix, n, seed + 1)
    Q = datagen.sample_mixture(mix, nq, seed + 2) if nq else None
    return X, Q


@pytest.mark.parametrize("d", [128, 40, 7])
def test_screened_agrees_with_the_gathered_descent(pk, d):
    X, Q = _mixture(40_000, d, 80, seed=1100 + d, nq=600)
    levels = [(20, 200), (1, 400), (1, 40)]  # 4,000 / 400 / 40 prototypes: levels 2 and 3 screened
    gix = pk.mask_build(dev(X), levels, iters=6, seed=2, precision="bf16")
    # score rows are padded to whole 128-byte lines (32 floats); 8 bytes per
    # query hold the launch order
    assert pk.mask_screen_bytes(gix) == 4 * (4000 + 416 + 64) + 8
    beams = [6, 24, 48]
    i1, d1 = (host(t) for t in pk.mask_query_beams(gix, dev(Q), 10, beams))
    i2, d2 = (host(t) for t in pk.mask_query_screened(gix, dev(Q), 10, beams))
    same = np.mean(np.all(i1 == i2, axis=1))
    assert same >= 0.95, same
    tids, tdist = mo.exact_knn(X, Q, 10)
    r1 = oc.recall_at_k(i1.astype(np.int64), tids, tdist,
                        oc.true_distances(X, Q, i1.astype(np.int64)), 10)
    r2 = oc.recall_at_k(i2.astype(np.int64), tids, tdist,
                        oc.true_distances(X, Q, i2.astype(np.int64)), 10)
    assert abs(r1 - r2) <= 0.01, (r1, r2)
    # the reported distances are the FP32 re-rank's, exact to FP32 rounding
    true = oc.true_distances(X, Q, i2.astype(np.int64))
    ok = i2 >= 0
    np.testing.assert_allclose(d2[ok], true[ok], rtol=1e-5, atol=1e-6)
    gix.free()


def test_probe_all_screened_is_exact_knn(pk):
    X, Q = _mixture(2000, 32, 10, seed=1110, nq=50)
    gix = pk.mask_build(dev(X), [(2, 40), (1, 8)], iters=4, seed=1, precision="bf16",
                        rerank_factor=256)
    ids, dist = (host(t) for t in pk.mask_query_screened(gix, dev(Q), 10, [2048, 2048]))
    tids, tdist = mo.exact_knn(X, Q, 10)
    true = oc.true_distances(X, Q, ids.astype(np.int64))
    res = oc.check_knn(ids.astype(np.int64), dist, tids, tdist, true, 1e-5)
    assert res.ok, res.messages
    gix.free()


def test_slices_change_nothing(pk):
    import torch
    X, Q = _mixture(20_000, 64, 40, seed=1120, nq=1000)
    gix = pk.mask_build(dev(X), [(10, 100), (1, 80)], iters=5, seed=3, precision="bf16")
    per = pk.mask_screen_bytes(gix)
    big = torch.empty(per * 1000 + 256, dtype=torch.uint8, device="cuda")
    small = torch.empty(per * 37, dtype=torch.uint8, device="cuda")  # 28 slices
    a = [host(t) for t in pk.mask_query_screened(gix, dev(Q), 10, [8, 16], workspace=big)]
    b = [host(t) for t in pk.mask_query_screened(gix, dev(Q), 10, [8, 16], workspace=small)]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    gix.free()


def test_screened_arguments(pk):
    import torch
    X, Q = _mixture(3000, 16, 10, seed=1130, nq=10)
    f32 = pk.mask_build(dev(X), [(2, 20)], iters=2, seed=1)
    with pytest.raises(pk.MaskError) as e:
        pk.mask_query_screened(f32, dev(Q), 5, [4])
    assert e.value.status == 4
    assert pk.mask_screen_bytes(f32) == 0
    f32.free()
    g = pk.mask_build(dev(X), [(2, 20)], iters=2, seed=1, precision="bf16")
    # one query: 40 scores padded to 64, and its launch-order slots
    tiny = torch.empty(4 * 64 + 8, dtype=torch.uint8, device="cuda")
    ids, _ = pk.mask_query_screened(g, dev(Q), 5, [4], workspace=tiny)
    with pytest.raises(pk.MaskError) as e:
        pk.mask_query_screened(g, dev(Q), 5, [4],
                               workspace=torch.empty(512, dtype=torch.uint8, device="cuda")[1:])
    assert e.value.status == 1  # misaligned
    g.free()


def test_mixed_screened_and_gathered_levels(pk):
    # level 1 has 20,000 prototypes (above the screening limit, gathered);
    # levels 2 and 3 are screened, as in the benchmark's index
    X, Q = _mixture(200_000, 16, 300, seed=1140, nq=400)
    levels = [(20, 1000), (1, 200), (1, 20)]
    gix = pk.mask_build(dev(X), levels, iters=3, seed=5, precision="bf16")
    assert pk.mask_screen_bytes(gix) == 4 * (224 + 32) + 8
    beams = [4, 16, 64]
    i1, _ = (host(t) for t in pk.mask_query_beams(gix, dev(Q), 10, beams))
    i2, d2 = (host(t) for t in pk.mask_query_screened(gix, dev(Q), 10, beams))
    assert np.mean(np.all(i1 == i2, axis=1)) >= 0.95
    true = oc.true_distances(X, Q, i2.astype(np.int64))
    ok = i2 >= 0
    np.testing.assert_allclose(d2[ok], true[ok], rtol=1e-5, atol=1e-6)
    gix.free()


def test_launch_order_changes_nothing(pk):
    # the screened path launches queries in the order of their greedy paths;
    # a permuted or partial batch must give every query the same result
    X, Q = _mixture(30_000, 32, 60, seed=1150, nq=700)
    gix = pk.mask_build(dev(X), [(15, 200), (1, 300), (1, 30)], iters=4, seed=6,
                        precision="bf16")
    beams = [4, 16, 48]
    ids, dist = (host(t) for t in pk.mask_query_screened(gix, dev(Q), 10, beams))
    p = np.random.default_rng(3).permutation(700)
    i2, d2 = (host(t) for t in pk.mask_query_screened(gix, dev(Q[p]), 10, beams))
    assert np.array_equal(i2, ids[p]) and np.array_equal(d2, dist[p])
    i3, d3 = (host(t) for t in pk.mask_query_screened(gix, dev(Q[100:137]), 10, beams))
    assert np.array_equal(i3, ids[100:137]) and np.array_equal(d3, dist[100:137])
    gix.free()


def _bf16_views(gix, X):
    """The oracle's view of a BF16 index: the exported prototypes, and every
    level's rows and the data rows rounded to bfloat16 as the descent reads
    them."""
    oix = oracle_index_from_gpu(X, gix)
    rank = [mo.quantize_bf16(P.astype(np.float32)) for P in oix.protos]
    return oix, rank, mo.quantize_bf16(X)


@pytest.mark.parametrize("d", [128, 40, 7])
def test_screened_and_gathered_descents_match_the_oracle(pk, d):
    # every prototype level screened (4,000 / 400 / 40 prototypes)
    X, Q = _mixture(40_000, d, 80, seed=1100 + d, nq=300)
    levels = [(20, 200), (1, 400), (1, 40)]
    gix = pk.mask_build(dev(X), levels, iters=6, seed=2, precision="bf16")
    oix, rank, leaf = _bf16_views(gix, X)
    beams = [6, 24, 48]  # 480 leaf candidates against a re-rank set of 40
    ids, dist, sel = (host(t) for t in pk.mask_query_screened(gix, dev(Q), 10, beams,
                                                               debug=True))
    fails = check_lowp_against_oracle(oix, Q, 10, beams, ids, dist, sel, rank, leaf, 4,
                                      screened_levels=(1, 2, 3))
    assert not fails, fails[:3]
    # the debug output does not change the results
    i0, d0 = (host(t) for t in pk.mask_query_screened(gix, dev(Q), 10, beams))
    assert np.array_equal(i0, ids) and np.array_equal(d0, dist)
    # the gathered descent on the same index: every level within 1e-5
    ids, dist, sel = (host(t) for t in pk.mask_query_beams(gix, dev(Q), 10, beams, debug=True))
    fails = check_lowp_against_oracle(oix, Q, 10, beams, ids, dist, sel, rank, leaf, 4)
    assert not fails, fails[:3]
    gix.free()


def test_mixed_screened_and_gathered_levels_match_the_oracle(pk):
    # level 1 gathered (20,000 prototypes), levels 2 and 3 screened
    X, Q = _mixture(200_000, 16, 300, seed=1140, nq=300)
    levels = [(20, 1000), (1, 200), (1, 20)]
    gix = pk.mask_build(dev(X), levels, iters=3, seed=5, precision="bf16")
    oix, rank, leaf = _bf16_views(gix, X)
    beams = [4, 16, 64]
    ids, dist, sel = (host(t) for t in pk.mask_query_screened(gix, dev(Q), 10, beams,
                                                               debug=True))
    fails = check_lowp_against_oracle(oix, Q, 10, beams, ids, dist, sel, rank, leaf, 4,
                                      screened_levels=(2, 3))
    assert not fails, fails[:3]
    gix.free()


def test_screened_debug_slices_keep_selections(pk):
    import torch
    X, Q = _mixture(20_000, 64, 40, seed=1160, nq=300)
    gix = pk.mask_build(dev(X), [(10, 100), (1, 80)], iters=5, seed=3, precision="bf16")
    per = pk.mask_screen_bytes(gix)
    small = torch.empty(per * 37, dtype=torch.uint8, device="cuda")
    a = [host(t) for t in pk.mask_query_screened(gix, dev(Q), 10, [8, 16], debug=True)]
    b = [host(t) for t in pk.mask_query_screened(gix, dev(Q), 10, [8, 16], workspace=small,
                                                 debug=True)]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # each level's selection is a set (its order comes from LDS slot atomics)
    assert np.array_equal(np.sort(a[2], axis=2), np.sort(b[2], axis=2))
    # every selection row: the beam's count of distinct ids, then -1 padding
    sel = a[2]
    for depth, beam in enumerate([8, 16]):
        rows = sel[:, depth, :]
        assert np.all(rows[:, beam:] == -1)
        assert np.all(rows[:, :beam] >= 0)  # the kept ids fill the first slots
        assert all(np.unique(r[:beam]).size == beam for r in rows)
    gix.free()
