"""Range search (Algorithm 3) on the GPU against the FP64 oracle, called
through the C ABI.

Rows near the boundary are the only ones allowed to differ.  A data point may
differ when its distance is within 1e-5 relative of the radius, or when one of
its ancestors is.  The caps are chosen so that no level reaches them away from
the exhaustive test.  Everything else must match: the set of ids, ascending
distances within 1e-5 relative of the true ones, and the in-radius count.
"""
import numpy as np
import pytest

import datagen
from oracle import mask_oracle as mo
from tests.gpu_helpers import dev, host, oracle_index_from_gpu

pytestmark = pytest.mark.gpu
REL = 1e-5


@pytest.fixture(scope="module")
def pk():
    import torch
    assert torch.cuda.is_available()
    import paper_2208_02734_amd as pk
    pk.lib()
    return pk


def _mixture(n, d, n_comp, seed, nq):
    mix = datagen.mixture_params(seed, n_comp, d, sigma_mode="loguniform", sigma_low=0.1,
                                 sigma_high=3.0)
    return datagen.sample_mixture(mix, n, seed + 1), datagen.sample_mixture(mix, nq, seed + 2)


def _ancestors(oix, i):
    """Prototype ids on the path of data row i, level 1 first."""
    out, cur = [], i
    for l in range(oix.n_levels):
        cur = int(oix.parents[l][cur])
        out.append(cur)
    return out


def _boundary(oix, q, radius, i):
    """True when data row i's membership may flip on rounding: its own
    distance, or one of its ancestors' distance, is within REL of the
    radius."""
    q = np.asarray(q, np.float64)
    d = np.sqrt(((oix.data[i] - q) ** 2).sum())
    if abs(d - radius) <= REL * max(radius, 1e-30):
        return True
    for l, p in enumerate(_ancestors(oix, i)):
        dp = np.sqrt(((oix.protos[l][p] - q) ** 2).sum())
        if abs(dp - radius) <= REL * max(radius, 1e-30):
            return True
    return False


def _check_range(oix, Q, radius, max_out, cap, ids, dist, count):
    """max_out is chosen above every in-radius count, so both sides return
    their whole answer: the sets must agree up to boundary cases, the GPU
    list must be ascending with true distances inside the radius, and its
    count must equal its length."""
    bad = []
    for i in range(Q.shape[0]):
        o_ids, _, o_cnt = mo.range_query_one(oix, Q[i], radius, max_out, cap)
        assert o_cnt <= max_out, "test radius too large for max_out"
        g = ids[i][ids[i] >= 0].astype(np.int64)
        gd = dist[i][:g.size].astype(np.float64)
        if int(count[i]) != g.size or np.any(ids[i][g.size:] != -1):
            bad.append((i, "count", int(count[i]), g.size))
            continue
        true = np.sqrt(((oix.data[g] - Q[i].astype(np.float64)) ** 2).sum(1))
        if not np.all(np.abs(gd - true) <= REL * np.maximum(true, 1e-30)):
            bad.append((i, "distance"))
            continue
        if not np.all(true <= radius * (1 + REL)) or np.any(np.diff(gd) < 0):
            bad.append((i, "outside or unsorted"))
            continue
        diff = set(g.tolist()) ^ set(o_ids[o_ids >= 0].tolist())
        if not all(_boundary(oix, Q[i], radius, j) for j in diff):
            bad.append((i, "set", int(count[i]), o_cnt, sorted(diff)[:5]))
    return bad


@pytest.mark.parametrize("quantile", [0.002, 0.01, 0.05])
def test_range_on_oracle_built_index(pk, quantile):
    X, Q = _mixture(6000, 16, 30, seed=700, nq=80)
    levels = [(6, 50), (1, 20)]
    oix = mo.build(X, levels, 6, seed=1)
    gix = pk.mask_import(dev(X), levels, oix.protos, oix.parents)
    # a radius around the given quantile of query-to-data distances
    D = mo.pairwise(Q[:10], X)
    radius = float(np.sqrt(np.quantile(D, quantile)))
    ids, dist, count = pk.mask_query_range(gix, dev(Q), radius, 2048, 64)
    bad = _check_range(oix, Q, radius, 2048, 64, host(ids), host(dist), host(count))
    assert not bad, bad[:3]
    gix.free()


def test_range_with_every_prototype_inside_is_exhaustive(pk):
    X, Q = _mixture(3000, 8, 20, seed=710, nq=30)
    levels = [(5, 30), (1, 10)]
    gix = pk.mask_build(dev(X), levels, iters=5, seed=2)
    D = mo.pairwise(Q, X)
    radius = float(np.sqrt(D.max())) * 1.01  # every point, hence every prototype, inside
    ids, dist, count = pk.mask_query_range(gix, dev(Q), radius, 64, 2048)
    ids, dist, count = host(ids), host(dist), host(count)
    assert np.all(count == 3000)
    for i in range(Q.shape[0]):
        order = np.lexsort((np.arange(3000), D[i]))[:64]
        assert np.array_equal(ids[i], order)
        np.testing.assert_allclose(dist[i], np.sqrt(D[i, order]), rtol=REL)
    gix.free()


def test_range_on_gpu_built_index_and_negative_radius(pk):
    import torch
    X, Q = _mixture(8000, 32, 40, seed=720, nq=60)
    levels = [(8, 80), (1, 20)]
    gix = pk.mask_build(dev(X), levels, iters=6, seed=3)
    oix = oracle_index_from_gpu(X, gix)
    D = mo.pairwise(Q[:10], X)
    radius = float(np.sqrt(np.quantile(D, 0.01)))
    rad = torch.full((60,), radius, dtype=torch.float32, device="cuda")
    rad[5] = -1.0
    ids, dist, count = pk.mask_query_range(gix, dev(Q), rad, 2048, 32)
    ids, dist, count = host(ids), host(dist), host(count)
    assert count[5] == 0 and np.all(ids[5] == -1)
    keep = np.array([i for i in range(60) if i != 5])
    bad = _check_range(oix, Q[keep], radius, 2048, 32, ids[keep], dist[keep], count[keep])
    assert not bad, bad[:3]
    gix.free()


def test_range_on_csr_index(pk):
    S = datagen.sample_sparse(3000, 500, 20, seed=730)
    QS = datagen.sample_sparse(40, 500, 20, seed=731)
    X, Q = S.to_dense(), QS.to_dense()
    levels = [(3, 40), (1, 10)]
    oix = mo.build(X, levels, 4, seed=4)
    Xs = pk.CsrTensor.from_host(S.indptr, S.indices, S.values, S.n_cols)
    Qs = pk.CsrTensor.from_host(QS.indptr, QS.indices, QS.values, QS.n_cols)
    gix = pk.mask_import(Xs, levels, oix.protos, oix.parents)
    radius = 1.2  # unit rows: distances lie in [0, 2]
    ids, dist, count = pk.mask_query_range(gix, Qs, radius, 2048, 64)
    bad = _check_range(oix, Q, radius, 2048, 64, host(ids), host(dist), host(count))
    assert not bad, bad[:3]
    gix.free()


def test_range_is_refused_by_the_precision_forms(pk):
    X, Q = _mixture(2000, 16, 10, seed=740, nq=4)
    gix = pk.mask_build(dev(X), [(2, 20)], iters=2, precision="bf16")
    with pytest.raises(pk.MaskError) as e:
        pk.mask_query_range(gix, dev(Q), 1.0, 10, 4)
    assert e.value.status == 4
    gix.free()
