"""Point query (Section 3.3) and the relocation loop (Sections 4.1-4.2, the
relocation table) on the GPU against the FP64 oracle, called through the C
ABI, on the eight-cloud benchmark of Section 4.2 with lengthGroup 16 and
nCentroids 8.

The point query's leaf, answer and exact match must equal the oracle's
unless the oracle's greedy path meets a near-tie (two candidates within
1e-5 relative) at some level; reported distances agree within 1e-5
relative.  Relocation is integer work and must agree exactly given the same
point-query results.
"""
import numpy as np
import pytest

import datagen
from oracle import mask_oracle as mo
from tests.gpu_helpers import dev, host, oracle_index_from_gpu

pytestmark = pytest.mark.gpu
REL = 1e-5
LG, NC = 16, 8


@pytest.fixture(scope="module")
def pk():
    import torch
    assert torch.cuda.is_available()
    import paper_2208_02734_amd as pk
    pk.lib()
    return pk


def _levels(n_groups):
    """Level 0 with n_groups groups, then Algorithm 1's schedule above it."""
    return [(n_groups, NC)] + mo.plan_levels(n_groups * NC, LG, NC)


def _near_tie_on_path(oix, q):
    _, _, tr = mo.query_one(oix, q, 1, 1, trace=True)
    for d in tr.cand_dist:
        if d.size >= 2:
            s = np.sort(d)
            if s[1] - s[0] <= REL * max(s[1], 1e-30):
                return True
    return False


def _check_points(oix, Q, ids, dist, leaf, match):
    bad = []
    for i in range(Q.shape[0]):
        a, d, lf, m = mo.point_query_one(oix, Q[i])
        same = ids[i] == a and leaf[i] == lf and match[i] == m
        if same and (a < 0 or abs(dist[i] - d) <= REL * max(d, 1e-30)):
            continue
        if not _near_tie_on_path(oix, Q[i]):
            bad.append((i, (int(ids[i]), int(leaf[i]), int(match[i]), float(dist[i])),
                        (a, lf, m, d)))
    return bad


def _wrong(labels, ids):
    """The error of Section 4.2: the point query's answer lies in another
    cloud than the query (or there is no answer)."""
    return (ids < 0) | (labels[np.maximum(ids, 0)] != labels)


def test_point_query_on_oracle_built_index(pk):
    c = datagen.eight_clouds(200, "moderate", seed=800)
    n = c.X.shape[0]
    levels = mo.plan_levels(n, LG, NC)
    oix = mo.build(c.X, levels, 10, seed=3)
    gix = pk.mask_import(dev(c.X), levels, oix.protos, oix.parents)
    # every data row (the paper's exhaustive point search) and fresh points
    fresh = datagen.eight_clouds(25, "moderate", seed=801).X
    Q = np.concatenate([c.X, fresh])
    ids, dist, leaf, match = (host(t) for t in pk.mask_point_query(gix, dev(Q)))
    bad = _check_points(oix, Q, ids, dist, leaf, match)
    assert not bad, bad[:3]
    assert np.all(match[n:] == -1)
    # the exact match, when found, is a data row equal to the query
    hit = np.nonzero(match[:n] >= 0)[0]
    assert hit.size > 0 and np.all(c.X[match[hit]] == c.X[hit])
    gix.free()


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
def test_point_query_on_gpu_built_index(pk, precision):
    c = datagen.eight_clouds(1000, "severe", seed=810)
    n = c.X.shape[0]
    gix = pk.mask_build(dev(c.X), mo.plan_levels(n, LG, NC), iters=10, seed=4,
                        precision=precision)
    oix = oracle_index_from_gpu(c.X, gix)
    ids, dist, leaf, match = (host(t) for t in pk.mask_point_query(gix, dev(c.X)))
    if precision == "fp32":
        bad = _check_points(oix, c.X, ids, dist, leaf, match)
        assert not bad, bad[:3]
    else:
        # the low-precision descent may reach another leaf; the scan of the
        # leaf it reached (FP32 rows) must still be exact
        kids = oix.children(0)
        for i in range(0, n, 7):
            pts = kids[leaf[i]] if leaf[i] >= 0 else np.zeros(0, np.int64)
            d = ((oix.data[pts] - c.X[i].astype(np.float64)) ** 2).sum(1)
            eq = pts[np.all(oix.data[pts] == c.X[i].astype(np.float64), axis=1)]
            assert match[i] == (eq.min() if eq.size else -1)
            if pts.size:
                best = pts[np.lexsort((pts, d))[0]]
                dbest = d[pts == best][0]
                assert ids[i] in pts
                assert ids[i] == best or abs(d[pts == ids[i]][0] - dbest) <= REL * dbest
            else:
                assert ids[i] == -1
    gix.free()


def test_point_query_edge_cases(pk):
    import torch
    c = datagen.eight_clouds(100, "none", seed=820)
    X = c.X.copy()
    X[17] = X[5]  # duplicate rows: the match is the lowest id of the leaf
    gix = pk.mask_build(dev(X), mo.plan_levels(800, LG, NC), iters=5, seed=1)
    ids, dist, leaf, match = (host(t) for t in pk.mask_point_query(gix, dev(X[[5, 17]])))
    oix = oracle_index_from_gpu(X, gix)
    for j, q in enumerate(X[[5, 17]]):
        a, d, lf, m = mo.point_query_one(oix, q)
        assert (ids[j], leaf[j], match[j]) == (a, lf, m)
    Qn = X[:3].copy()
    Qn[1, 0] = np.nan  # a NaN coordinate equals nothing
    _, _, _, m = (host(t) for t in pk.mask_point_query(gix, dev(Qn)))
    assert m[1] == -1
    out = pk.mask_point_query(gix, torch.zeros((0, 2), device="cuda"))
    assert all(t.numel() == 0 for t in out)
    gix.free()


def test_build_on_given_groups_matches_oracle(pk):
    import torch
    g = np.random.default_rng(830)
    c = datagen.eight_clouds(60, "none", seed=830)
    n = c.X.shape[0]
    perm = g.permutation(n)
    sizes = np.array([1, 3, 7, 8, 9, 40, 100, 128, 184])  # some smaller than k
    off = np.concatenate([[0], np.cumsum(sizes)])
    assert off[-1] == n
    levels = [(len(sizes), NC), (2, NC)]
    oix = mo.build(c.X, levels, 6, seed=0, perm=perm, group_off=off)
    gix = pk.mask_build(dev(c.X), levels, iters=6, perm=torch.from_numpy(perm.astype(np.int32))
                        .cuda(), group_off=off)
    for lev in (1, 2):
        P, par = gix.export_level(lev)
        assert np.array_equal(par, oix.parents[lev - 1]), lev
        np.testing.assert_allclose(P, oix.protos[lev - 1], rtol=1e-5, atol=1e-4)
    # a group of one point: its k prototypes are that point
    P, _ = gix.export_level(1)
    assert np.all(P[:NC] == c.X[perm[0]])
    gix.free()


def test_relocation_loop_matches_oracle(pk):
    import torch
    c = datagen.eight_clouds(200, "severe", seed=840)
    n = c.X.shape[0]
    perm = mo.permutation(7, n)
    off = mo.chunk_offsets(n, n // LG)
    t_perm = torch.from_numpy(perm.astype(np.int32)).cuda()
    errors = []
    for it in range(4):
        levels = _levels(off.shape[0] - 1)
        gix = pk.mask_build(dev(c.X), levels, iters=10, perm=t_perm, group_off=off)
        oix = oracle_index_from_gpu(c.X, gix)
        ids, dist, leaf, match = pk.mask_point_query(gix, dev(c.X))
        h_ids, h_leaf = host(ids), host(leaf)
        bad = _check_points(oix, c.X, h_ids, host(dist), h_leaf, host(match))
        assert not bad, (it, bad[:3])
        wrong = _wrong(c.labels, h_ids)
        errors.append(wrong.mean())
        t_perm, g_off = pk.mask_relocate(gix, leaf, dev(wrong.astype(np.int32)))
        o_perm, o_off = mo.relocate(perm, off, NC, h_leaf, wrong)
        assert np.array_equal(host(t_perm), o_perm), it
        assert np.array_equal(g_off, o_off), it
        perm, off = o_perm, o_off
        gix.free()
    # the first build is the plain split of a seeded permutation; relocation
    # moves points, so later groups are ragged
    assert np.diff(off).min() < LG < np.diff(off).max()
    assert 0.2 < errors[0] < 0.6


def test_relocate_rejects_bad_leaves_and_imported_indexes(pk):
    import torch
    c = datagen.eight_clouds(50, "none", seed=850)
    n = c.X.shape[0]
    levels = mo.plan_levels(n, LG, NC)
    gix = pk.mask_build(dev(c.X), levels, iters=3, seed=2)
    leaf = torch.full((n,), levels[0][0] * NC, dtype=torch.int32, device="cuda")
    wrong = torch.ones(n, dtype=torch.int32, device="cuda")
    with pytest.raises(pk.MaskError) as e:
        pk.mask_relocate(gix, leaf, wrong)
    assert e.value.status == 1
    # nothing wrong: the order and groups of the build come back
    _, _, lf, _ = pk.mask_point_query(gix, dev(c.X))
    p2, o2 = pk.mask_relocate(gix, lf, torch.zeros(n, dtype=torch.int32, device="cuda"))
    assert np.array_equal(host(p2), mo.permutation(2, n))
    assert np.array_equal(o2, mo.chunk_offsets(n, levels[0][0]))
    P = [gix.export_level(l)[0] for l in range(1, len(levels) + 1)]
    par = [gix.export_level(l)[1] for l in range(1, len(levels) + 1)]
    imp = pk.mask_import(dev(c.X), levels, P, par)
    with pytest.raises(pk.MaskError) as e:
        pk.mask_relocate(imp, lf, wrong)
    assert e.value.status == 4
    imp.free()
    gix.free()
