"""The leaf-batched descent of the BF16 form: the data layer evaluated leaf
by leaf (each leaf's rows read once for every query that kept it), with
results equal to the screened descent's bit for bit (the same kept leaves,
the same BF16 arithmetic per row, the same re-rank and selection), and the
oracle's check on its selections and results."""
import numpy as np
import pytest

import datagen
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


def _same(pk, gix, Q, k, beams, **kw):
    a = [host(t) for t in pk.mask_query_screened(gix, dev(Q), k, beams)]
    b = [host(t) for t in pk.mask_query_batched(gix, dev(Q), k, beams, **kw)]
    assert np.array_equal(a[0], b[0]), (k, beams, int(np.sum(np.any(a[0] != b[0], axis=1))))
    assert np.array_equal(a[1], b[1]), (k, beams)
    return b


@pytest.mark.parametrize("d", [96, 40, 7, 128, 200])
def test_batched_equals_screened(pk, d):
    # every row width class of the BF16 descent (1, 2, 4 and 8 lanes per row);
    # a gathered level 1 under two screened levels, as in the benchmark
    X, Q = _mixture(60_000, d, 120, seed=1200 + d, nq=500)
    gix = pk.mask_build(dev(X), [(20, 1000), (1, 400), (1, 40)], iters=4, seed=2,
                        precision="bf16")
    for k, beams in ((10, [3, 3, 24]), (10, [6, 16, 64]), (1, [2, 2, 8]), (40, [4, 8, 30])):
        _same(pk, gix, Q, k, beams)
    gix.free()


def test_batched_without_a_rerank_and_with_large_k(pk):
    # few candidates (every one ranked in FP32: the data layer reads rows),
    # and k above 512 (another LDS class)
    X, Q = _mixture(30_000, 32, 60, seed=1210, nq=300)
    gix = pk.mask_build(dev(X), [(10, 300), (1, 50)], iters=4, seed=3, precision="bf16")
    _same(pk, gix, Q, 10, [1, 1])     # about 10 candidates, R = 40: no re-rank
    _same(pk, gix, Q, 600, [20, 80])  # k = 600
    _same(pk, gix, Q, 10, [50, 300])  # every leaf
    # the one-wave-per-query data layer takes re-rank sets and k up to 192 and
    # level-1 beams up to 128; beyond either, the workgroup-per-query one
    _same(pk, gix, Q, 48, [8, 128])   # R = 192, 128 leaves
    _same(pk, gix, Q, 49, [8, 100])   # R = 196
    _same(pk, gix, Q, 10, [8, 129])   # 129 leaves
    _same(pk, gix, Q, 192, [8, 120])  # k = 192, R = 768
    gix.free()
    # a re-rank set of 4 k r (factor -4): R = 96 at k = 1, above 192 at k = 10
    gix = pk.mask_build(dev(X), [(10, 300), (1, 50)], iters=4, seed=3, precision="bf16",
                        rerank_factor=-4)
    _same(pk, gix, Q, 1, [4, 24])
    _same(pk, gix, Q, 10, [4, 24])
    gix.free()


def test_batched_slices_and_selections(pk):
    import torch
    X, Q = _mixture(40_000, 64, 80, seed=1220, nq=700)
    gix = pk.mask_build(dev(X), [(20, 200), (1, 200), (1, 20)], iters=4, seed=4,
                        precision="bf16")
    beams = [4, 12, 40]
    ids, dist = _same(pk, gix, Q, 10, beams)
    # a workspace for 37 queries: 19 slices give the same rows
    small = torch.empty(pk.mask_batched_bytes(gix, beams, 37), dtype=torch.uint8, device="cuda")
    i2, d2 = (host(t) for t in pk.mask_query_batched(gix, dev(Q), 10, beams, workspace=small))
    assert np.array_equal(i2, ids) and np.array_equal(d2, dist)
    # the kept prototypes are the screened descent's (as sets)
    _, _, s1 = (host(t) for t in pk.mask_query_screened(gix, dev(Q), 10, beams, debug=True))
    _, _, s2 = (host(t) for t in pk.mask_query_batched(gix, dev(Q), 10, beams, debug=True))
    assert np.array_equal(np.sort(s1, axis=2), np.sort(s2, axis=2))
    # a workspace below one query is refused
    with pytest.raises(pk.MaskError) as e:
        pk.mask_query_batched(gix, dev(Q), 10, beams,
                              workspace=torch.empty(4096, dtype=torch.uint8, device="cuda"))
    assert e.value.status == 1
    gix.free()


def test_batched_matches_the_oracle(pk):
    X, Q = _mixture(50_000, 48, 100, seed=1230, nq=200)
    levels = [(10, 500), (1, 500), (1, 25)]
    gix = pk.mask_build(dev(X), levels, iters=4, seed=5, precision="bf16")
    oix = oracle_index_from_gpu(X, gix)
    rank = [mo.quantize_bf16(P.astype(np.float32)) for P in oix.protos]
    leaf = mo.quantize_bf16(X)
    beams = [4, 10, 32]
    ids, dist, sel = (host(t) for t in pk.mask_query_batched(gix, dev(Q), 10, beams,
                                                              debug=True))
    fails = check_lowp_against_oracle(oix, Q, 10, beams, ids, dist, sel, rank, leaf, 4,
                                      screened_levels=(2, 3))
    assert not fails, fails[:3]
    gix.free()


def test_batched_arguments(pk):
    import torch
    X, Q = _mixture(3000, 16, 10, seed=1240, nq=10)
    f32 = pk.mask_build(dev(X), [(2, 20)], iters=2, seed=1)
    with pytest.raises(pk.MaskError) as e:
        pk.mask_query_batched(f32, dev(Q), 5, [4])
    assert e.value.status == 4
    f32.free()
    g = pk.mask_build(dev(X), [(2, 20)], iters=2, seed=1, precision="bf16")
    assert pk.mask_batched_bytes(g, [4], 10) > pk.mask_batched_bytes(g, [4], 1) > 0
    ids, dist = pk.mask_query_batched(g, dev(Q[:0]), 5, [4])  # no queries
    assert ids.shape == (0, 5)
    # one level: the leaves are the top level
    _same(pk, g, Q, 5, [4])
    _same(pk, g, Q, 3, [40])  # every leaf
    g.free()


def test_batched_row_counters(pk):
    # the device counts behind the benchmark's query roofline, summed over
    # their per-workgroup slots: the (query, row) pairs the leaf scan
    # evaluates are the rows of every query's kept leaves, and the rows the
    # levels read are the gathered level's candidates (the children of the
    # kept level-2 prototypes) plus the data rows of the queries whose
    # candidates are all ranked in FP32 (no re-rank set)
    X, Q = _mixture(60_000, 48, 120, seed=1250, nq=3000)
    gix = pk.mask_build(dev(X), [(20, 1000), (1, 400), (1, 40)], iters=4, seed=2,
                        precision="bf16")
    _, par0 = gix.export_level(1)
    _, par1 = gix.export_level(2)
    rows = np.bincount(par0, minlength=20_000)
    kids = np.bincount(par1, minlength=20_000)
    k, beams = 10, [3, 3, 24]
    pk.mask_timing_enable(True)
    ids, dist, sel = (host(t) for t in pk.mask_query_batched(gix, dev(Q), k, beams, debug=True))
    rep = pk.mask_timing_report()
    pk.mask_timing_enable(False)
    s2, s1 = sel[:, 1, :3], sel[:, 2, :24]
    m = np.where(s1 >= 0, rows[np.maximum(s1, 0)], 0).sum(axis=1)
    assert rep["leaf_scan_pairs"][0] == int(m.sum())
    gathered = int(np.where(s2 >= 0, kids[np.maximum(s2, 0)], 0).sum())
    fp32_rows = int(m[m <= 4 * k].sum())  # default re-rank set 4 k
    assert rep["descent_rows"][0] == gathered + fp32_rows
    assert rep["leaf_scan"][0] == 1 and rep["leaf_select"][0] == 1 and rep["level_select"][0] == 1
    gix.free()


def test_batched_with_empty_leaves(pk):
    # groups of 100 rows with 150 prototypes each: the first-k start repeats
    # rows, so a third of the leaves end up empty; kept empty leaves (and
    # queries whose kept leaves hold no row at all) give the same rows as the
    # screened descent, -1 / inf past the candidates found
    X, Q = _mixture(3000, 24, 30, seed=1260, nq=400)
    gix = pk.mask_build(dev(X), [(30, 150), (1, 100)], iters=3, seed=6, precision="bf16")
    _, par0 = gix.export_level(1)
    assert np.sum(np.bincount(par0, minlength=4500) == 0) > 1000
    for k, beams in ((10, [2, 3]), (10, [1, 1]), (5, [4, 40]), (60, [8, 120])):
        ids, dist = _same(pk, gix, Q, k, beams)
        assert np.all((ids >= 0) == np.isfinite(dist))
    # empty leaves are among the kept ones (a repeated prototype ties with its
    # twin, which owns the rows)
    _, _, sel = (host(t) for t in pk.mask_query_batched(gix, dev(Q), 5, [4, 40], debug=True))
    kept = sel[:, 1, :40]
    sizes = np.bincount(par0, minlength=4500)
    assert np.any(sizes[kept[kept >= 0]] == 0)
    gix.free()
