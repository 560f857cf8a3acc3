"""The precision form (BF16 distances, FP32 re-rank, FP64 sums) and ragged
batches.  BF16 screening is not certified, so its build is pinned
statistically against the FP64 oracle (label agreement, inertia ratio);
the FP32 re-rank makes every returned distance exact to the FP32 tolerance,
and re-ranking every candidate reproduces exhaustive search."""
import numpy as np
import pytest

import datagen
from oracle import compare as oc
from oracle import mask_oracle as mo
from tests.gpu_helpers import check_lowp_against_oracle, dev, host, oracle_index_from_gpu

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


def _nearest_agreement(X, gix, chunks, k):
    """Fraction of level-1 labels equal to the FP64 nearest prototype of the
    item's group (exported prototypes), and the worst relative excess."""
    P, par = gix.export_level(1)
    agree, worst = 0, 0.0
    for c in range(chunks):
        members = np.nonzero(par // k == c)[0]
        D = mo.pairwise(X[members], P[c * k:(c + 1) * k])
        got = D[np.arange(members.size), par[members] - c * k]
        best = D.min(axis=1)
        agree += int(np.sum(got <= best * (1 + 1e-12)))
        worst = max(worst, float(np.max((got - best) / np.maximum(best, 1e-30))))
    return agree / X.shape[0], worst


@pytest.mark.parametrize("d", [96, 128])
def test_bf16_build_labels_are_nearly_nearest(pk, d):
    X, _ = _mixture(30_000, d, 60, seed=200 + d)
    levels = [(6, 200), (1, 40)]
    g16 = pk.mask_build(dev(X), levels, iters=10, seed=1, precision="bf16")
    frac, worst = _nearest_agreement(X, g16, 6, 200)
    # BF16 rounding of |x|, |c| ~ 10^2 moves a distance by ~1e-2 absolute
    assert frac > 0.97, frac
    assert worst < 0.05, worst
    # inertia of the BF16 build within 1% of the FP32 build's
    g32 = pk.mask_build(dev(X), levels, iters=10, seed=1)

    def inertia(ix):
        P, par = ix.export_level(1)
        return float(((X.astype(np.float64) - P[par]) ** 2).sum())
    assert inertia(g16) <= inertia(g32) * 1.01


@pytest.mark.parametrize("n,d", [(20_000, 96), (100_000, 96), (600_000, 90)])
def test_bf16_assignment_is_the_argmax_of_bf16_scores(pk, n, d):
    # The three workgroup shapes of the BF16 assignment at d <= 96 (chosen by
    # the row count: 128, 256 and 512 rows per workgroup, prototype tiles of
    # 64 or 128) with a ragged prototype tail (k = 300) and, at d = 90, zero
    # padding to 96.  Each sampled row's label must maximise
    # x~.c~ - |c~|^2 / 2 over its group (FP64 on the BF16-rounded values) up
    # to the kernel's FP32 accumulation and its 4 low bits of index.
    C, k = 2, 300
    X, _ = _mixture(n, d, 80, seed=400 + d)
    gix = pk.mask_build(dev(X), [(C, k)], iters=2, seed=1, precision="bf16")
    P, par = gix.export_level(1)
    gix.free()
    pi = mo.permutation(1, n)
    off = mo.chunk_offsets(n, C)
    g = np.random.default_rng(n)
    Pq = mo.quantize_bf16(P.astype(np.float32))
    for c in range(C):
        sample = g.choice(pi[off[c]:off[c + 1]], 2000, replace=False)
        assert np.all(par[sample] // k == c)
        xq = mo.quantize_bf16(X[sample])
        pc = Pq[c * k:(c + 1) * k]
        p2 = np.sum(pc * pc, axis=1)
        S = xq @ pc.T - 0.5 * p2[None, :]
        tol = 2.0 ** -15 * (np.linalg.norm(xq, axis=1)[:, None] * np.sqrt(p2)[None, :]
                            + p2[None, :]).max(axis=1)
        got = S[np.arange(sample.size), par[sample] - c * k]
        gap = S.max(axis=1) - got
        assert np.all(gap <= tol), (c, float(np.max(gap - tol)), int(np.sum(gap > tol)))
        # the kernel does pick the maximum, not merely a near one, almost always
        assert np.mean(gap == 0) > 0.99


def test_bf16_query_distances_are_fp32_exact(pk):
    X, Q = _mixture(20_000, 96, 50, seed=210, nq=100)
    levels = [(10, 100), (1, 40)]
    gix = pk.mask_build(dev(X), levels, iters=8, seed=2, precision="bf16", rerank_factor=4)
    for r in (4, 16):
        ids, dist = pk.mask_query(gix, dev(Q), 10, r)
        ids, dist = host(ids).astype(np.int64), host(dist)
        true = oc.true_distances(X, Q, ids)
        v = ids >= 0
        assert np.all(np.abs(dist[v] - true[v]) <= REL * true[v])
        assert np.all(dist[:, 1:] >= dist[:, :-1])


def test_bf16_rerank_of_everything_is_exact(pk):
    # probe every prototype and re-rank all candidates: exhaustive search
    X, Q = _mixture(4000, 32, 20, seed=220, nq=50)
    levels = [(4, 50), (1, 20)]
    oix = mo.build(X, levels, 5, seed=3)
    gix = pk.mask_import(dev(X), levels, oix.protos, oix.parents, precision="bf16",
                         rerank_factor=1000)
    ids, dist = pk.mask_query(gix, dev(Q), 10, 2048)
    tids, tdist = mo.exact_knn(X, Q, 10)
    true = oc.true_distances(X, Q, host(ids).astype(np.int64))
    assert oc.check_knn(host(ids), host(dist), tids, tdist, true, REL).ok


def test_bf16_recall_close_to_fp32_on_shared_index(pk):
    X, Q = _mixture(30_000, 64, 80, seed=230, nq=200)
    levels = [(10, 300), (1, 60)]
    oix = mo.build(X, levels, 6, seed=4)
    g32 = pk.mask_import(dev(X), levels, oix.protos, oix.parents)
    g16 = pk.mask_import(dev(X), levels, oix.protos, oix.parents, precision="bf16")
    tids, tdist = mo.exact_knn(X, Q, 10)
    rec = {}
    for name, ix in (("fp32", g32), ("bf16", g16)):
        ids, _ = pk.mask_query(ix, dev(Q), 10, 8)
        ids = host(ids).astype(np.int64)
        rec[name] = oc.recall_at_k(ids, tids, tdist, oc.true_distances(X, Q, ids), 10)
    assert rec["bf16"] >= rec["fp32"] - 0.02, rec


def test_ragged_rows_equal_single_queries(pk):
    import torch
    X, Q = _mixture(10_000, 48, 40, seed=240, nq=60)
    gix = pk.mask_build(dev(X), [(5, 100), (1, 25)], iters=6, seed=5)
    g = np.random.default_rng(9)
    ks = g.integers(1, 40, size=60).astype(np.int32)
    rs = g.choice([2, 8, 20], size=60).astype(np.int32)
    ids, dist, off = pk.mask_query_ragged(gix, dev(Q), torch.from_numpy(ks), torch.from_numpy(rs))
    ids, dist, off = host(ids), host(dist), host(off)
    for i in range(60):
        i1, d1 = pk.mask_query(gix, dev(Q[i:i + 1]), int(ks[i]), int(rs[i]))
        assert np.array_equal(ids[off[i]:off[i + 1]], host(i1)[0])
        assert np.array_equal(dist[off[i]:off[i + 1]], host(d1)[0])


# --------------------------------------------------------------- FP8 form
# OCP e4m3 rows with one FP32 scale per row: 3 mantissa bits, so a rounded
# value is within 2^-4 relative of the original.  The FP8 screening is not
# certified; the returned distances are FP32 re-ranked and so exact.

def test_fp8_build_is_close_to_fp32(pk):
    X, _ = _mixture(30_000, 128, 60, seed=328)
    levels = [(6, 200), (1, 40)]
    g8 = pk.mask_build(dev(X), levels, iters=10, seed=1, precision="fp8")
    frac, worst = _nearest_agreement(X, g8, 6, 200)
    g32 = pk.mask_build(dev(X), levels, iters=10, seed=1)

    def inertia(ix):
        P, par = ix.export_level(1)
        return float(((X.astype(np.float64) - P[par]) ** 2).sum())
    ratio = inertia(g8) / inertia(g32)
    print(f"fp8 label agreement {frac:.4f}, worst excess {worst:.4f}, inertia ratio {ratio:.4f}")
    assert frac > 0.9, frac
    assert ratio <= 1.03, ratio
    # Rounding bound: x^ = x + dx with |dx| <= 2^-4 |x| (likewise c), so
    # | |x^ - c^|^2 - |x - c|^2 | <= (2^-3 + 2^-8)(|x| + |c|)^2
    #                           <= 0.26 (|x|^2 + |c|^2),
    # and the chosen prototype is at most twice that above the nearest.
    P, par = g8.export_level(1)
    X64 = X.astype(np.float64)
    for c in range(6):
        members = np.nonzero(par // 200 == c)[0]
        Pc = P[c * 200:(c + 1) * 200].astype(np.float64)
        D = mo.pairwise(X[members], Pc)
        got = D[np.arange(members.size), par[members] - c * 200]
        bound = 0.52 * ((X64[members] ** 2).sum(1) + (Pc ** 2).sum(1).max())
        assert np.all(got - D.min(axis=1) <= bound)


@pytest.mark.parametrize("d", [40, 96, 128])
def test_fp8_labels_are_the_argmax_of_the_fp8_scores(pk, d):
    # The FP8 assignment ranks s_i s_j (q_i . q_j) - |c^_j|^2 / 2 with the
    # rows and prototypes quantised as the oracle quantises them (OCP e4m3,
    # one scale per row) and the product accumulated in FP32.  Every label
    # must be an argmax of that score computed in FP64 here, up to the FP32
    # accumulation of the products (d terms, each exact).  d = 40 takes the
    # K = 16 MFMA shape, 96 and 128 the K = 64 one (96 with a half-empty
    # last block).
    X, _ = _mixture(20_000, d, 60, seed=380 + d)
    C, k = 4, 150
    g8 = pk.mask_build(dev(X), [(C, k)], iters=3, seed=1, precision="fp8")
    P, par = g8.export_level(1)
    qx, sx = mo.quantize_fp8(X)
    qp, sp = mo.quantize_fp8(P)
    cn = ((qp * sp[:, None]) ** 2).sum(1)
    exact = 0
    for c in range(C):
        members = np.nonzero(par // k == c)[0]
        Qm = qx[members].astype(np.float64)
        Pc = qp[c * k:(c + 1) * k].astype(np.float64)
        dot = Qm @ Pc.T
        score = sx[members, None] * sp[None, c * k:(c + 1) * k] * dot - 0.5 * cn[None, c * k:(c + 1) * k]
        absdot = np.abs(Qm) @ np.abs(Pc).T
        tol = (d * 2.0 ** -24) * sx[members, None] * sp[None, c * k:(c + 1) * k] * absdot
        got = par[members] - c * k
        row = np.arange(members.size)
        best = score.max(axis=1)
        # the chosen prototype's score reaches the best within both scores' bounds
        slack = tol[row, got] + tol.max(axis=1) + 1e-6 * np.abs(cn[c * k:(c + 1) * k]).max()
        assert np.all(score[row, got] >= best - slack), c
        exact += int(np.sum(score[row, got] == best))
    assert exact >= 0.99 * X.shape[0], exact
    g8.free()


def test_fp8_query_distances_are_fp32_exact(pk):
    X, Q = _mixture(20_000, 96, 50, seed=310, nq=100)
    levels = [(10, 100), (1, 40)]
    gix = pk.mask_build(dev(X), levels, iters=8, seed=2, precision="fp8")
    for r in (4, 16):
        ids, dist = pk.mask_query(gix, dev(Q), 10, r)
        ids, dist = host(ids).astype(np.int64), host(dist)
        true = oc.true_distances(X, Q, ids)
        v = ids >= 0
        assert np.all(np.abs(dist[v] - true[v]) <= REL * true[v])
        assert np.all(dist[:, 1:] >= dist[:, :-1])


def test_fp8_rerank_of_everything_is_exact(pk):
    X, Q = _mixture(4000, 32, 20, seed=320, nq=50)
    levels = [(4, 50), (1, 20)]
    oix = mo.build(X, levels, 5, seed=3)
    gix = pk.mask_import(dev(X), levels, oix.protos, oix.parents, precision="fp8",
                         rerank_factor=1000)
    ids, dist = pk.mask_query(gix, dev(Q), 10, 2048)
    tids, tdist = mo.exact_knn(X, Q, 10)
    true = oc.true_distances(X, Q, host(ids).astype(np.int64))
    assert oc.check_knn(host(ids), host(dist), tids, tdist, true, REL).ok


def test_fp8_recall_close_to_fp32_on_shared_index(pk):
    X, Q = _mixture(30_000, 64, 80, seed=330, nq=200)
    levels = [(10, 300), (1, 60)]
    oix = mo.build(X, levels, 6, seed=4)
    g32 = pk.mask_import(dev(X), levels, oix.protos, oix.parents)
    g8 = pk.mask_import(dev(X), levels, oix.protos, oix.parents, precision="fp8")
    tids, tdist = mo.exact_knn(X, Q, 10)
    rec = {}
    for name, ix in (("fp32", g32), ("fp8", g8)):
        ids, _ = pk.mask_query(ix, dev(Q), 10, 8)
        ids = host(ids).astype(np.int64)
        rec[name] = oc.recall_at_k(ids, tids, tdist, oc.true_distances(X, Q, ids), 10)
    print(rec)
    assert rec["fp8"] >= rec["fp32"] - 0.05, rec


def test_fp8_descent_matches_the_oracle(pk):
    # prototype levels in FP32, the data layer in FP8 with a per-row scale;
    # 16 leaves of about 20 rows against a re-rank set of 40
    X, Q = _mixture(20_000, 96, 50, seed=340, nq=300)
    levels = [(10, 100), (1, 40)]
    gix = pk.mask_build(dev(X), levels, iters=8, seed=2, precision="fp8", rerank_factor=4)
    oix = oracle_index_from_gpu(X, gix)
    code, scale = mo.quantize_fp8(X)
    leaf = code * scale[:, None]
    for beams in ([4, 16], [2, 40]):
        ids, dist, sel = (host(t) for t in pk.mask_query_beams(gix, dev(Q), 10, beams,
                                                                debug=True))
        fails = check_lowp_against_oracle(oix, Q, 10, beams, ids, dist, sel, oix.protos,
                                          leaf, 4)
        assert not fails, (beams, fails[:3])
    gix.free()


def test_bf16_gathered_descent_matches_the_oracle_at_d96(pk):
    X, Q = _mixture(20_000, 96, 50, seed=350, nq=300)
    levels = [(10, 100), (1, 40)]
    gix = pk.mask_build(dev(X), levels, iters=8, seed=2, precision="bf16")
    oix = oracle_index_from_gpu(X, gix)
    rank = [mo.quantize_bf16(P.astype(np.float32)) for P in oix.protos]
    leaf = mo.quantize_bf16(X)
    for beams in ([4, 16], [1, 3]):
        ids, dist, sel = (host(t) for t in pk.mask_query_beams(gix, dev(Q), 10, beams,
                                                                debug=True))
        fails = check_lowp_against_oracle(oix, Q, 10, beams, ids, dist, sel, rank, leaf, 4)
        assert not fails, (beams, fails[:3])
    gix.free()


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_ragged_rerank_set_follows_each_query(pk, precision):
    # a query with k above 512 moves the batch to the large LDS class; the
    # other queries' re-rank sets must stay what they are alone
    import torch
    X, Q = _mixture(40_000, 32, 60, seed=360, nq=40)
    gix = pk.mask_build(dev(X), [(10, 100), (1, 25)], iters=6, seed=5, precision=precision)
    g = np.random.default_rng(19)
    ks = g.integers(1, 220, size=40).astype(np.int32)
    ks[::7] = 600
    rs = g.choice([8, 32], size=40).astype(np.int32)
    ids, dist, off = pk.mask_query_ragged(gix, dev(Q), torch.from_numpy(ks),
                                          torch.from_numpy(rs))
    ids, dist, off = host(ids), host(dist), host(off)
    for i in range(40):
        i1, d1 = pk.mask_query(gix, dev(Q[i:i + 1]), int(ks[i]), int(rs[i]))
        assert np.array_equal(ids[off[i]:off[i + 1]], host(i1)[0]), i
        assert np.array_equal(dist[off[i]:off[i + 1]], host(d1)[0]), i
    gix.free()


@pytest.mark.parametrize("precision", ["fp8", "bf16"])
def test_rerank_of_4kr_candidates_matches_the_oracle(pk, precision):
    # rerank_factor -4: the re-rank set is 4 k r1 (r1 = leaves probed), above
    # 512 for the wider beams (the large LDS class) and below it for the
    # narrow ones
    X, Q = _mixture(30_000, 96, 60, seed=370, nq=200)
    levels = [(10, 150), (1, 50)]  # leaves of about 20 rows
    gix = pk.mask_build(dev(X), levels, iters=6, seed=2, precision=precision,
                        rerank_factor=-4)
    oix = oracle_index_from_gpu(X, gix)
    if precision == "fp8":
        code, scale = mo.quantize_fp8(X)
        leaf, rank = code * scale[:, None], oix.protos
    else:
        leaf = mo.quantize_bf16(X)
        rank = [mo.quantize_bf16(P.astype(np.float32)) for P in oix.protos]
    for beams in ([4, 8], [6, 24]):  # R = 320, then 960
        assert mo.rerank_size(10, beams, -4) == 40 * beams[-1]
        ids, dist, sel = (host(t) for t in pk.mask_query_beams(gix, dev(Q), 10, beams,
                                                                debug=True))
        fails = check_lowp_against_oracle(oix, Q, 10, beams, ids, dist, sel, rank, leaf, -4)
        assert not fails, (beams, fails[:3])
    gix.free()
