"""Dynamic insertion (Section 3.3) on the GPU against the FP64 oracle,
called through the C ABI: the leaf every new point joins, the level-0 groups
and leaf order after the batch, and the local rebuild of groups whose leaves
grow beyond a threshold.

Leaves equal the oracle's unless the oracle's insertion path meets a
near-tie (two candidates within 1e-5 relative) at some level; group order is
integer work and must agree exactly; rebuilt prototypes follow the plain
build's tolerance (labels exact, prototypes within 1e-5 relative / 1e-4
absolute of the FP64 means).
"""
import numpy as np
import pytest

import datagen
from oracle import mask_oracle as mo
from tests.gpu_helpers import check_query_against_oracle, dev, host, oracle_index_from_gpu

pytestmark = pytest.mark.gpu
REL = 1e-5


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


def _oracle_view(pk, X, gix):
    """The oracle's view of a GPU index, with the level-0 order and groups of
    its build (a relocation step with nothing wrong returns them)."""
    import torch
    oix = oracle_index_from_gpu(X, gix)
    n = X.shape[0]
    z = torch.zeros(n, dtype=torch.int32, device="cuda")
    perm, off = pk.mask_relocate(gix, z, z)
    oix.perm0 = host(perm).astype(np.int64)
    oix.group_off0 = off
    return oix


def _tie_on_insertion_path(oix, x):
    L = oix.n_levels
    cand = np.arange(oix.protos[L - 1].shape[0])
    x = np.asarray(x, np.float64)
    for l in range(L - 1, -1, -1):
        if l >= 1:
            kids = oix.children(l)
            cand = np.array([p for p in cand if kids[p].size > 0])
        d = mo.pairwise(x[None, :], oix.protos[l][cand])[0]
        s = np.sort(d)
        if s.size >= 2 and s[1] - s[0] <= REL * max(s[1], 1e-30):
            return True
        chosen = cand[np.lexsort((cand, d))[0]]
        if l >= 1:
            cand = oix.children(l)[chosen]
    return False


def _check_insert(pk, gix, oix_before, X_all, leaves_gpu, new_o, leaves_o, Xn):
    diff = np.nonzero(leaves_gpu != leaves_o)[0]
    for j in diff:
        assert _tie_on_insertion_path(oix_before, Xn[j]), (j, leaves_gpu[j], leaves_o[j])
    if diff.size:
        return False
    import torch
    n2 = X_all.shape[0]
    assert gix.info()["n"] == n2
    _, par = gix.export_level(1)
    assert np.array_equal(par, new_o.parents[0])
    z = torch.zeros(n2, dtype=torch.int32, device="cuda")
    perm, off = pk.mask_relocate(gix, z, z)
    assert np.array_equal(host(perm), new_o.perm0)
    assert np.array_equal(off, new_o.group_off0)
    return True


def test_insert_without_rebuild_matches_oracle(pk):
    X, Q = _mixture(6000, 16, 30, seed=900, nq=60)
    Xn, _ = _mixture(700, 16, 30, seed=905)
    levels = [(6, 40), (2, 30), (1, 10)]
    gix = pk.mask_build(dev(X), levels, iters=6, seed=3)
    oix = _oracle_view(pk, X, gix)
    leaves, nr = pk.mask_insert(gix, dev(Xn[:500]))
    assert nr == 0
    new_o, leaves_o, rebuilt = mo.insert(oix, Xn[:500], max_leaf=0)
    X_all = np.concatenate([X, Xn[:500]])
    assert _check_insert(pk, gix, oix, X_all, host(leaves), new_o, leaves_o, Xn[:500])
    # a second batch on the grown index
    leaves2, _ = pk.mask_insert(gix, dev(Xn[500:]))
    new_o2, leaves_o2, _ = mo.insert(new_o, Xn[500:], max_leaf=0)
    X_all2 = np.concatenate([X_all, Xn[500:]])
    assert _check_insert(pk, gix, new_o, X_all2, host(leaves2), new_o2, leaves_o2, Xn[500:])
    # queries on the grown index agree with the oracle's on the same structure
    oq = oracle_index_from_gpu(X_all2, gix)
    ids, dist, sel = pk.mask_query(gix, dev(Q), 10, 6, debug=True)
    _, _, fails = check_query_against_oracle(oq, X_all2, Q, 10, 6, host(ids), host(dist),
                                             host(sel))
    assert not fails, fails[:3]
    gix.free()


def test_insert_with_local_rebuild_matches_oracle(pk):
    X, _ = _mixture(5000, 8, 25, seed=910)
    g = np.random.default_rng(911)
    Xn = (X[g.choice(5000, 900)] + 0.05 * g.standard_normal((900, 8))).astype(np.float32)
    levels = [(5, 30), (1, 12)]
    gix = pk.mask_build(dev(X), levels, iters=5, seed=7)
    oix = _oracle_view(pk, X, gix)
    P2_before, par2_before = gix.export_level(2)
    new0, _, _ = mo.insert(oix, Xn, max_leaf=0)
    sizes = np.bincount(new0.parents[0], minlength=150)
    limit = int(np.sort(sizes)[-4])
    leaves, nr = pk.mask_insert(gix, dev(Xn), max_leaf=limit)
    new_o, leaves_o, rebuilt = mo.insert(oix, Xn, max_leaf=limit, iters=5)
    assert np.array_equal(host(leaves), leaves_o)
    assert nr == len(rebuilt) and nr >= 1
    P1, par1 = gix.export_level(1)
    np.testing.assert_allclose(P1, new_o.protos[0], rtol=1e-5, atol=1e-4)
    assert np.array_equal(par1, new_o.parents[0])
    P2, par2 = gix.export_level(2)
    assert np.array_equal(P2, P2_before) and np.array_equal(par2, par2_before)
    gix.free()


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_inserted_rows_are_searchable_in_the_precision_forms(pk, precision):
    X, _ = _mixture(4000, 32, 20, seed=920)
    Xn, _ = _mixture(300, 32, 20, seed=925)
    gix = pk.mask_build(dev(X), [(4, 25), (1, 10)], iters=4, seed=1, precision=precision)
    pk.mask_insert(gix, dev(Xn))
    assert gix.info()["n"] == 4300
    # probing every prototype is exhaustive: each new row is its own nearest
    ids, dist = pk.mask_query(gix, dev(Xn), 1, 2048)
    assert np.array_equal(host(ids)[:, 0], 4000 + np.arange(300))
    assert np.all(host(dist)[:, 0] == 0.0)
    gix.free()


def test_insert_edge_cases(pk):
    import torch
    X, _ = _mixture(2000, 8, 10, seed=930)
    levels = [(4, 20), (1, 8)]
    gix = pk.mask_build(dev(X), levels, iters=3, seed=2)
    leaves, nr = pk.mask_insert(gix, torch.zeros((0, 8), device="cuda"))
    assert leaves.numel() == 0 and nr == 0 and gix.info()["n"] == 2000
    with pytest.raises(pk.MaskError) as e:
        pk.mask_insert(gix, torch.zeros((3, 5), device="cuda"))
    assert e.value.status == 1
    # a copy of a data row joins a leaf; the copy and the original are both rows
    leaves, _ = pk.mask_insert(gix, dev(X[:4]))
    assert gix.info()["n"] == 2004
    _, par = gix.export_level(1)
    assert np.array_equal(par[2000:], host(leaves))
    P = [gix.export_level(l)[0] for l in (1, 2)]
    pr = [gix.export_level(l)[1] for l in (1, 2)]
    imp = pk.mask_import(dev(np.concatenate([X, X[:4]])), levels, P, pr)
    with pytest.raises(pk.MaskError) as e:
        pk.mask_insert(imp, dev(X[:2]))
    assert e.value.status == 4
    imp.free()
    gix.free()


def test_insert_and_point_query_with_l1(pk):
    X, _ = _mixture(3000, 8, 15, seed=940)
    Xn, _ = _mixture(200, 8, 15, seed=945)
    levels = [(3, 20), (1, 6)]
    gix = pk.mask_build(dev(X), levels, iters=4, seed=5, metric="l1")
    oix = _oracle_view(pk, X, gix)
    oix.metric = "l1"
    leaves, _ = pk.mask_insert(gix, dev(Xn))
    new_o, leaves_o, _ = mo.insert(oix, Xn, max_leaf=0)
    assert np.array_equal(host(leaves), leaves_o)
    X_all = np.concatenate([X, Xn])
    new_o2 = oracle_index_from_gpu(X_all, gix, metric="l1")
    ids, dist, leaf, match = (host(t) for t in pk.mask_point_query(gix, dev(Xn[:50])))
    for j in range(50):
        a, d, lf, m = mo.point_query_one(new_o2, Xn[j])
        assert (ids[j], leaf[j], match[j]) == (a, lf, m)
        assert abs(dist[j] - d) <= 1e-5 * max(d, 1e-30)
    gix.free()
