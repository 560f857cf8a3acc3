"""Parity of the CSR path (the sparse high-dimensional setting of Section
4.3) with the FP64 oracle, called through the C ABI.

The oracle is the same definition on the densified rows (a CSR row and its
dense form are the same point).  The GPU evaluates |x|^2 + |c|^2 - 2 x.c in
float64, so labels agree with the oracle's direct form except where two
prototypes are within about 1e-12 relative; the tolerances below are the
plain form's (1e-5 relative on reported distances, near-tie id swaps,
prototypes within one float32 ulp of the float64 mean).
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
    pk.lib()
    return pk


def _csr(pk, S):
    return pk.CsrTensor.from_host(S.indptr, S.indices, S.values, S.n_cols)


def _sparse(n, cols, nnz, seed, nq=0):
    X = datagen.sample_sparse(n, cols, nnz, seed)
    Q = datagen.sample_sparse(nq, cols, nnz, seed + 1) if nq else None
    return X, Q


def test_one_lloyd_step_matches_oracle(pk):
    n, cols, C, k = 3001, 700, 3, 40
    S, _ = _sparse(n, cols, 30, seed=500)
    X = S.to_dense()
    Xs = _csr(pk, S)
    _, lab0, _ = pk.mask_kmeans(Xs, C, k, 0)
    cent1, _, inert = pk.mask_kmeans(Xs, C, k, 1)
    lab0, cent1, inert = host(lab0), host(cent1), host(inert)
    off = mo.chunk_offsets(n, C)
    for c in range(C):
        pts = X[off[c]:off[c + 1]].astype(np.float64)
        init = pts[:k]
        olab, onew, oin = mo.lloyd_step(pts, init)
        D = mo.pairwise(pts, init)
        glab = lab0[off[c]:off[c + 1]] - c * k
        diff = np.nonzero(glab != olab)[0]
        for i in diff:
            a, b = D[i, glab[i]], D[i, olab[i]]
            assert abs(a - b) <= 1e-12 * max(a, b), (c, i, a, b)
        assert abs(inert[0, c] - oin) <= 1e-10 * oin
        bad = set(glab[diff].tolist()) | set(olab[diff].tolist())
        for j in range(k):
            if j in bad:
                continue
            ref = onew[j].astype(np.float32)
            got = cent1[c * k + j]
            ulp = np.spacing(np.abs(ref)).astype(np.float32)
            assert np.all(np.abs(got - ref) <= ulp), (c, j)


def test_lloyd_invariants(pk):
    n, cols, C, k, T = 8000, 1500, 4, 60, 8
    S, _ = _sparse(n, cols, 50, seed=510)
    X = S.to_dense()
    cent, lab, inert = pk.mask_kmeans(_csr(pk, S), C, k, T)
    cent, lab, inert = host(cent), host(lab), host(inert)
    assert np.all(inert[1:] <= inert[:-1] * (1 + 1e-12))
    off = mo.chunk_offsets(n, C)
    for c in range(C):
        D = mo.pairwise(X[off[c]:off[c + 1]], cent[c * k:(c + 1) * k])
        g = lab[off[c]:off[c + 1]] - c * k
        best = D.min(axis=1)
        assert np.all(D[np.arange(D.shape[0]), g] <= best * (1 + 1e-12) + 1e-15)


def test_full_build_matches_oracle(pk):
    n, cols = 4000, 600
    S, _ = _sparse(n, cols, 25, seed=520)
    X = S.to_dense()
    levels = [(4, 30), (1, 12)]
    oix = mo.build(X, levels, 6, seed=11)
    gix = pk.mask_build(_csr(pk, S), levels, iters=6, seed=11)
    info = gix.info()
    assert info["layout"] == "csr" and info["nnz"] == S.indices.shape[0]
    for lev in (1, 2):
        P, par = gix.export_level(lev)
        o_par = oix.parents[lev - 1]
        diff = np.nonzero(par != o_par)[0]
        assert diff.size == 0, (lev, diff[:10])
        np.testing.assert_allclose(P, oix.protos[lev - 1], rtol=1e-6, atol=1e-7)
    gix.free()


@pytest.mark.parametrize("r,k", [(1, 5), (4, 10), (25, 10)])
def test_query_on_oracle_built_index(pk, r, k):
    n, cols = 5000, 900
    S, QS = _sparse(n, cols, 30, seed=530, nq=100)
    X, Q = S.to_dense(), QS.to_dense()
    levels = [(5, 40), (1, 20)]
    oix = mo.build(X, levels, 5, seed=3)
    gix = pk.mask_import(_csr(pk, S), levels, oix.protos, oix.parents)
    ids, dist, sel = pk.mask_query(gix, _csr(pk, QS), k, r, debug=True)
    _, _, fails = check_query_against_oracle(oix, X, Q, k, r, host(ids), host(dist), host(sel))
    assert not fails, fails[:3]
    gix.free()


def test_query_on_gpu_built_index(pk):
    n, cols = 8000, 1200
    S, QS = _sparse(n, cols, 40, seed=540, nq=120)
    X, Q = S.to_dense(), QS.to_dense()
    levels = [(4, 80), (1, 25), (1, 5)]
    gix = pk.mask_build(_csr(pk, S), levels, iters=6, seed=4)
    oix = oracle_index_from_gpu(X, gix)
    for r, k in [(1, 5), (3, 10), (12, 10)]:
        ids, dist, sel = pk.mask_query(gix, _csr(pk, QS), k, r, debug=True)
        _, _, fails = check_query_against_oracle(oix, X, Q, k, r, host(ids), host(dist),
                                                 host(sel))
        assert not fails, (r, k, fails[:3])
    gix.free()


def test_probe_all_is_exact_knn_and_self_distance_is_zero(pk):
    n, cols = 3000, 800
    S, _ = _sparse(n, cols, 20, seed=550)
    X = S.to_dense()
    gix = pk.mask_build(_csr(pk, S), [(3, 50), (1, 20)], iters=4, seed=2)
    Xs = _csr(pk, S)
    qrows = Xs.rows(100, 164)  # 64 data rows as queries
    Q = X[100:164]
    ids, dist = pk.mask_query(gix, qrows, 10, 2048)
    ids, dist = host(ids), host(dist)
    tids, tdist = mo.exact_knn(X, Q, 10)
    true = oc.true_distances(X, Q, ids.astype(np.int64))
    res = oc.check_knn(ids, dist, tids, tdist, true, REL)
    assert res.ok, res.messages
    # a data row is at distance exactly 0 from itself
    assert np.all(dist[:, 0] == 0.0)
    assert np.all(ids[:, 0] == np.arange(100, 164))
    gix.free()


def test_ragged_and_beams_on_csr(pk):
    import torch
    n, cols = 4000, 500
    S, QS = _sparse(n, cols, 20, seed=560, nq=40)
    gix = pk.mask_build(_csr(pk, S), [(4, 40), (1, 10)], iters=4, seed=5)
    q = _csr(pk, QS)
    g = np.random.default_rng(3)
    ks = g.integers(1, 30, size=40).astype(np.int32)
    rs = g.choice([1, 4, 9], size=40).astype(np.int32)
    ids, dist, off = pk.mask_query_ragged(gix, q, torch.from_numpy(ks), torch.from_numpy(rs))
    ids, dist, off = host(ids), host(dist), host(off)
    for i in range(40):
        i1, d1 = pk.mask_query(gix, q.rows(i, i + 1), int(ks[i]), int(rs[i]))
        assert np.array_equal(ids[off[i]:off[i + 1]], host(i1)[0])
        assert np.array_equal(dist[off[i]:off[i + 1]], host(d1)[0])
    b_ids, b_dist = pk.mask_query_beams(gix, q, 10, [3, 7])
    oix = oracle_index_from_gpu(S.to_dense(), gix)
    for i in range(40):
        o_ids, o_dist = mo.query_one(oix, QS.to_dense()[i], 10, [3, 7])
        g_ids = host(b_ids)[i:i + 1].astype(np.int64)
        true = oc.true_distances(S.to_dense(), QS.to_dense()[i:i + 1], g_ids)
        assert oc.check_knn(g_ids, host(b_dist)[i:i + 1], o_ids[None], o_dist[None], true,
                            REL).ok
    gix.free()


def test_bad_csr_is_rejected(pk):
    import torch
    S, _ = _sparse(500, 100, 10, seed=570)
    bad_cols = S.indices.copy()
    bad_cols[5], bad_cols[6] = bad_cols[6], bad_cols[5]  # not increasing within row 0
    X = pk.CsrTensor.from_host(S.indptr, bad_cols, S.values, S.n_cols)
    with pytest.raises(pk.MaskError) as e:
        pk.mask_build(X, [(2, 10)], iters=1)
    assert e.value.status == 1
    # a CSR index takes CSR queries only
    gix = pk.mask_build(_csr(pk, S), [(2, 10)], iters=1)
    with pytest.raises(pk.MaskError):
        pk.mask_query(gix, torch.zeros((2, 100), device="cuda"), 5, 2)
    with pytest.raises(pk.MaskError) as e:
        pk.MaskServer(gix)
    assert e.value.status == 4
    gix.free()


def test_beams_above_2048_on_csr_match_the_oracle(pk):
    # Level-1 beams of 2,049 .. 3,072 (the CSR index's wider LDS class):
    # selections and results against the oracle's descent on the same index.
    n, cols = 24000, 400
    S, QS = _sparse(n, cols, 12, seed=580, nq=16)
    X, Q = S.to_dense(), QS.to_dense()
    gix = pk.mask_build(_csr(pk, S), [(4, 1000), (1, 40)], iters=3, seed=6)
    oix = oracle_index_from_gpu(X, gix)
    q = _csr(pk, QS)
    for beams, k in (([40, 2049], 10), ([40, 3072], 25), ([7, 2600], 1)):
        ids, dist, sel = pk.mask_query_beams(gix, q, k, beams, debug=True)
        n_rows, n_rep, fails = check_query_against_oracle(oix, X, Q, k, beams, host(ids),
                                                          host(dist), host(sel))
        assert not fails, (beams, k, fails[:3])
        if beams[0] == 40:  # every level-1 prototype is a candidate: the beam is kept
            assert np.all((host(sel)[:, 1] >= 0).sum(axis=1) == beams[1])
    # the uniform beam takes the same limit
    ids, dist = pk.mask_query(gix, q, 10, 3072)
    assert host(ids).shape == (16, 10)
    with pytest.raises(pk.MaskError) as e:
        pk.mask_query_beams(gix, q, 10, [40, 3073])
    assert e.value.status == 1
    with pytest.raises(pk.MaskError):
        pk.mask_query(gix, q, 2049, 8)  # k stays at most 2048
    gix.free()


def test_beams_above_2048_need_a_csr_index_of_at_most_12288_columns(pk):
    import torch
    S, QS = _sparse(3000, 12289, 8, seed=590, nq=4)
    gix = pk.mask_build(_csr(pk, S), [(2, 30)], iters=1)
    q = _csr(pk, QS)
    pk.mask_query(gix, q, 5, 2048)
    with pytest.raises(pk.MaskError) as e:
        pk.mask_query(gix, q, 5, 2049)
    assert e.value.status == 1
    gix.free()
    # and a dense index stays at 2048
    X = torch.randn(500, 8, device="cuda")
    dix = pk.mask_build(X, [(2, 10)], iters=1)
    with pytest.raises(pk.MaskError):
        pk.mask_query(dix, X[:3], 5, 2049)
    dix.free()
