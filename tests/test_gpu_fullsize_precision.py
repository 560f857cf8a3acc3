"""Parity of the precision form at its full benchmark size (10,000,000 x 96
Gaussian mixture, levels 10 x 10,000 -> 10,000 -> 100 from k-means++ seeds,
30 Lloyd iterations; 100,000 queries), in the launch configurations the
benchmark times: BF16 through the leaf-batched descent (equal to the
screened descent bit for bit) at beams 3/3/24 with the 4k re-rank, and FP8 (per-row scale) through the gathered descent at 3/3/28
with the 4·k·r re-rank.  Checked on outputs the oracle can check one by
one: sampled queries against the oracle's descent on the exported index
(every level's selection a nearest set by FP64 distance to the rows as the
descent reads them, the result the FP32 re-rank of an R-nearest set), and
sampled level-1 BF16 assignments against the FP64 scores of the
BF16-rounded rows and prototypes of their group; and the serving loop with
the benchmark's server on the same index (rows in the mix equal rows alone,
and a sample passes the oracle's check).
The oracle reads the data rows it needs one query at a time (rows are
converted when indexed), so no FP64 copy of the 10M rows is made."""
import numpy as np
import pytest

import datagen
from oracle import mask_oracle as mo
from tests.gpu_helpers import check_lowp_against_oracle, dev, host

pytestmark = pytest.mark.gpu

LEVELS = [(10, 10_000), (1, 10_000), (1, 100)]
BEAMS = [3, 3, 24]


class _Fp8Rows:
    """Data rows as FP8 e4m3 codes times their row scale, on demand."""

    def __init__(self, X):
        self.X = X

    def __getitem__(self, idx):
        code, scale = mo.quantize_fp8(self.X[idx])
        return code * scale[:, None]


class _Bf16Rows:
    """Data rows rounded to BF16 (as the descent reads them), on demand."""

    def __init__(self, X):
        self.X = X

    def __getitem__(self, idx):
        return mo.quantize_bf16(self.X[idx])


@pytest.fixture(scope="module")
def built():
    import torch
    import paper_2208_02734_amd as pk
    pk.lib()
    cfg = datagen.config_precision()
    X, Q = cfg.X, cfg.Q
    assert cfg.levels == LEVELS
    print(f"full-size precision form: n={X.shape[0]} d={X.shape[1]} levels={LEVELS}", flush=True)
    gix = pk.mask_build(dev(X), LEVELS, iters=30, seed=1, precision="bf16", init="kmeans++")
    torch.cuda.synchronize()
    protos, parents = [], []
    for lev in range(1, len(LEVELS) + 1):
        P, par = gix.export_level(lev)
        protos.append(P)
        parents.append(par)
    # the exported prototypes and parents; data rows stay FP32 (each check
    # converts the rows it indexes)
    oix = mo.OracleIndex(data=X, protos=[np.asarray(P, dtype=np.float64) for P in protos],
                         parents=[np.asarray(p, dtype=np.int64) for p in parents],
                         levels=[(0, 0)] * len(LEVELS), metric="l2", inertia=[])
    yield pk, X, Q, gix, oix, protos
    gix.free()


def test_fullsize_precision_sampled_queries(built):
    pk, X, Q, gix, oix, protos = built
    ids, dist, sel = (host(t) for t in pk.mask_query_screened(gix, dev(Q), 10, BEAMS,
                                                               debug=True))
    rows = np.sort(np.random.default_rng(8).choice(Q.shape[0], 48, replace=False))
    rank = [mo.quantize_bf16(P.astype(np.float32)) for P in protos]
    # levels 3 (100 prototypes) and 2 (10,000) are scored by the batched GEMM
    fails = check_lowp_against_oracle(oix, Q, 10, BEAMS, ids, dist, sel, rank, _Bf16Rows(X),
                                      4, screened_levels=(2, 3), rows=rows)
    assert not fails, fails[:3]
    assert np.all(ids >= 0) and np.all(dist[:, 1:] >= dist[:, :-1])
    # the leaf-batched descent the benchmark times (all 100,000 queries in one
    # slice): the same rows and kept sets, and the oracle's check on its own
    # selections
    ib, db, sb = (host(t) for t in pk.mask_query_batched(gix, dev(Q), 10, BEAMS, debug=True))
    assert np.array_equal(ib, ids) and np.array_equal(db, dist)
    assert np.array_equal(np.sort(sb, axis=2), np.sort(sel, axis=2))
    fails = check_lowp_against_oracle(oix, Q, 10, BEAMS, ib, db, sb, rank, _Bf16Rows(X),
                                      4, screened_levels=(2, 3), rows=rows[:16])
    assert not fails, fails[:3]


def test_fullsize_precision_sampled_assignments(built):
    pk, X, Q, gix, oix, protos = built
    n = X.shape[0]
    C, k = LEVELS[0]
    pi = mo.permutation(1, n)
    off = mo.chunk_offsets(n, C)
    par = oix.parents[0]
    Pq = mo.quantize_bf16(protos[0].astype(np.float32))
    g = np.random.default_rng(9)
    for c in g.choice(C, 3, replace=False):
        sample = g.choice(pi[off[c]:off[c + 1]], 1000, replace=False)
        assert np.all(par[sample] // k == c)
        xq = mo.quantize_bf16(X[sample])
        pc = Pq[c * k:(c + 1) * k]
        p2 = np.sum(pc * pc, axis=1)
        S = xq @ pc.T - 0.5 * p2[None, :]
        # the kernel's FP32 accumulation and its 4 low bits of index
        tol = 2.0 ** -15 * (np.linalg.norm(xq, axis=1)[:, None] * np.sqrt(p2)[None, :]
                            + p2[None, :]).max(axis=1)
        gap = S.max(axis=1) - S[np.arange(sample.size), par[sample] - c * k]
        assert np.all(gap <= tol), (c, float(np.max(gap - tol)))


def test_fullsize_fp8_sampled_queries(built):
    pk, X, Q, gix, oix, protos = built
    beams = [3, 3, 28]
    f8 = pk.mask_build(dev(X), LEVELS, iters=30, seed=1, precision="fp8", init="kmeans++",
                       rerank_factor=-4)
    try:
        ids, dist, sel = (host(t) for t in pk.mask_query_beams(f8, dev(Q), 10, beams,
                                                                debug=True))
        fprotos, fparents = [], []
        for lev in range(1, len(LEVELS) + 1):
            P, par = f8.export_level(lev)
            fprotos.append(np.asarray(P, dtype=np.float64))
            fparents.append(np.asarray(par, dtype=np.int64))
    finally:
        f8.free()
    foix = mo.OracleIndex(data=X, protos=fprotos, parents=fparents,
                          levels=[(0, 0)] * len(LEVELS), metric="l2", inertia=[])
    assert mo.rerank_size(10, beams, -4) == 4 * 10 * 28
    rows = np.sort(np.random.default_rng(10).choice(Q.shape[0], 32, replace=False))
    # prototype levels are read in FP32, the data rows in FP8
    fails = check_lowp_against_oracle(foix, Q, 10, beams, ids, dist, sel, fprotos, _Fp8Rows(X),
                                      -4, rows=rows)
    assert not fails, fails[:3]


def test_fullsize_serving_in_the_mix_equals_alone_and_the_oracle(built):
    # The serving form on the full-size BF16 index with the benchmark's
    # server (4 GiB arena, batches of up to 32,768 queries, three streams,
    # beam profile 3/3/24 eighths of r): requests of 1-512 queries
    # (log-uniform), k in [1, 100], r in {8, 32}, submitted back to back.
    # Every request's rows equal the same queries' descent alone at the
    # profile's beams, and a sample of them passes the oracle's check.
    import time
    pk, X, Q, gix, oix, protos = built
    profile = [3, 3, 24]
    srv = pk.MaskServer(gix, arena_bytes=4 << 30, max_batch_queries=32768, n_streams=3,
                        batch_window_us=5_000, beam_eighths=profile)
    g = np.random.default_rng(12)
    reqs, tickets = [], []
    pos = 0
    for _ in range(40):
        n = int(np.floor(np.exp(g.uniform(0.0, np.log(513)))))
        k = int(g.integers(1, 101))
        r = int(g.choice([8, 32]))
        reqs.append((pos, n, k, r))
        tickets.append(srv.submit(Q[pos:pos + n], k, r))
        pos += n
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                res = srv.poll(t)
                if res is not None:
                    out[t] = res
        assert time.time() - t0 < 120, "requests did not finish"
    st = srv.stats()
    srv.close()
    assert st["completed_requests"] == 40
    rank = [mo.quantize_bf16(P.astype(np.float32)) for P in protos]
    leaf = _Bf16Rows(X)
    checked = 0
    for j, ((p, n, k, r), t) in enumerate(zip(reqs, tickets)):
        ids, dist, _ = out[t]
        beams = [max(1, (r * e + 7) // 8) for e in profile]
        i1, d1, sel = (host(x) for x in pk.mask_query_beams(gix, dev(Q[p:p + n]), k, beams,
                                                             debug=True))
        assert np.array_equal(ids, i1) and np.array_equal(dist, d1), (p, n, k, r)
        if j % 4 == 0:  # the oracle on the first two queries of every fourth request
            rows = range(min(n, 2))
            fails = check_lowp_against_oracle(oix, Q[p:p + n], k, beams, ids, dist, sel, rank,
                                              leaf, 4, rows=rows)
            assert not fails, (p, n, k, r, fails[:2])
            checked += len(rows)
    assert checked >= 10
