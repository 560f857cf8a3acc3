"""The serving form: continuous batching with memory admission.  Each
request's rows must be the same whether it ran alone or batched with
others (bit-exact: the descent runs one query per workgroup)."""
import time

import numpy as np
import pytest

import datagen
from tests.gpu_helpers import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    import paper_2208_02734_amd as pk
    pk.lib()
    mix = datagen.mixture_params(300, 40, 32, sigma_mode="loguniform", sigma_low=0.1,
                                 sigma_high=3.0)
    X = datagen.sample_mixture(mix, 20_000, 301)
    Q = datagen.sample_mixture(mix, 4_000, 302)
    ix = pk.mask_build(dev(X), [(10, 100), (1, 40)], iters=6, seed=7)
    torch.cuda.synchronize()
    return pk, ix, Q


def _drain(srv, tickets, timeout=60.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout, "requests did not finish"
    return out


def test_results_in_the_mix_equal_results_alone(setup):
    pk, ix, Q = setup
    g = np.random.default_rng(11)
    # a 20 ms batching window: requests submitted back to back share launches
    srv = pk.MaskServer(ix, arena_bytes=64 << 20, max_batch_queries=2048, n_streams=3,
                        batch_window_us=20_000)
    reqs, tickets = [], []
    pos = 0
    for _ in range(120):
        n = int(g.integers(1, 48))
        k = int(g.integers(1, 60))
        r = int(g.choice([2, 8, 16]))
        reqs.append((pos, n, k, r))
        tickets.append(srv.submit(Q[pos:pos + n], k, r))
        pos = (pos + n) % (Q.shape[0] - 64)
    res = _drain(srv, tickets)
    st = srv.stats()
    srv.close()
    assert st["completed_requests"] == 120
    assert st["batches"] < 120  # requests were batched together
    for (p, n, k, r), t in zip(reqs, tickets):
        ids, dist, t_done = res[t]
        i1, d1 = pk.mask_query(ix, dev(Q[p:p + n]), k, r)
        assert np.array_equal(ids, host(i1)) and np.array_equal(dist, host(d1))


def test_memory_admission_serialises_but_serves_everything(setup):
    pk, ix, Q = setup
    # an arena that holds about one 64-query batch at a time
    srv = pk.MaskServer(ix, arena_bytes=96 * 1024, max_batch_queries=4096, n_streams=2)
    tickets = [srv.submit(Q[i * 64:(i + 1) * 64], 10, 4) for i in range(20)]
    res = _drain(srv, tickets)
    st = srv.stats()
    assert st["completed_queries"] == 20 * 64
    assert st["peak_arena_bytes"] <= 96 * 1024
    # a request that can never fit is refused at submission
    with pytest.raises(pk.MaskError) as e:
        srv.submit(Q[:1000], 50, 4)
    assert e.value.status == 5
    srv.close()
    for i, t in enumerate(tickets):
        i1, _ = pk.mask_query(ix, dev(Q[i * 64:(i + 1) * 64]), 10, 4)
        assert np.array_equal(res[t][0], host(i1))


def test_latency_stamps(setup):
    pk, ix, Q = setup
    srv = pk.MaskServer(ix, arena_bytes=16 << 20, n_streams=2)
    t0 = pk.mask_clock()
    t = srv.submit(Q[:8], 5, 4, t_arrival=t0)
    ids, dist, t_done = _drain(srv, [t])[t]
    srv.close()
    assert t_done >= t0 and t_done - t0 < 5.0


def test_batching_window_holds_partial_batches(setup):
    pk, ix, Q = setup
    srv = pk.MaskServer(ix, arena_bytes=16 << 20, max_batch_queries=64, n_streams=1,
                        batch_window_us=50_000)
    t0 = pk.mask_clock()
    t1 = srv.submit(Q[:8], 5, 4, t_arrival=t0)
    _, _, t_done = _drain(srv, [t1])[t1]
    assert t_done - t0 >= 0.05  # a partial batch waits out the window
    t0 = pk.mask_clock()
    t2 = srv.submit(Q[:64], 5, 4, t_arrival=t0)  # a full batch launches at once
    ids, _, t_done = _drain(srv, [t2])[t2]
    srv.close()
    assert t_done - t0 < 0.05
    i1, _ = pk.mask_query(ix, dev(Q[:64]), 5, 4)
    assert np.array_equal(ids, host(i1))


def test_replay_serves_a_schedule(setup):
    pk, ix, Q = setup
    rs = datagen.request_stream(2000.0, 0.05, seed=9, pool_rows=Q.shape[0], max_queries=64)
    n = rs.t_arrival.shape[0]
    assert n > 20
    srv = pk.MaskServer(ix, arena_bytes=32 << 20, max_batch_queries=4096, n_streams=2)
    lat, span = srv.replay(Q, rs.t_arrival, rs.n_queries, rs.pool_offset, rs.k, rs.r)
    st = srv.stats()
    srv.close()
    assert st["completed_requests"] == n
    assert st["completed_queries"] == int(rs.n_queries.sum())
    assert np.all(lat > 0) and np.all(lat < 5.0)
    assert span >= rs.t_arrival[-1]


# ------------------------------------------------ precision forms, served

@pytest.fixture(scope="module")
def lowp_setup():
    import torch
    import paper_2208_02734_amd as pk
    pk.lib()
    mix = datagen.mixture_params(310, 60, 32, sigma_mode="loguniform", sigma_low=0.1,
                                 sigma_high=3.0)
    X = datagen.sample_mixture(mix, 40_000, 311)
    Q = datagen.sample_mixture(mix, 3_000, 312)
    levels = [(10, 100), (1, 25)]  # leaves of about 40 rows
    ixs = {p: pk.mask_build(dev(X), levels, iters=6, seed=7, precision=p)
           for p in ("bf16", "fp8")}
    torch.cuda.synchronize()
    yield pk, ixs, X, Q
    for ix in ixs.values():
        ix.free()


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_lowp_results_in_the_mix_equal_results_alone(lowp_setup, precision):
    # requests with k above 512 share batches with small ones: every
    # request's rows must still equal its rows alone (the re-rank set of a
    # query follows its own k and r, not the batch's)
    pk, ixs, X, Q = lowp_setup
    ix = ixs[precision]
    g = np.random.default_rng(21)
    srv = pk.MaskServer(ix, arena_bytes=64 << 20, max_batch_queries=2048, n_streams=3,
                        batch_window_us=20_000)
    reqs, tickets = [], []
    pos = 0
    for j in range(60):
        n = int(g.integers(1, 24))
        k = 600 if j % 9 == 4 else int(g.integers(1, 220))
        r = int(g.choice([8, 32]))
        reqs.append((pos, n, k, r))
        tickets.append(srv.submit(Q[pos:pos + n], k, r))
        pos = (pos + n) % (Q.shape[0] - 32)
    res = _drain(srv, tickets)
    st = srv.stats()
    srv.close()
    assert st["completed_requests"] == 60 and st["batches"] < 60
    for (p, n, k, r), t in zip(reqs, tickets):
        ids, dist, _ = res[t]
        i1, d1 = pk.mask_query(ix, dev(Q[p:p + n]), k, r)
        assert np.array_equal(ids, host(i1)), (p, n, k, r)
        assert np.array_equal(dist, host(d1)), (p, n, k, r)


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_served_rows_match_the_oracle(lowp_setup, precision):
    # served rows against the FP64 oracle on the exported index: each level's
    # selection (from the same query's debug descent, whose rows must equal
    # the served ones bit for bit) is a nearest set of the low-precision rows,
    # and the result is the FP32 re-rank of the R nearest leaf candidates
    from oracle import mask_oracle as mo
    from tests.gpu_helpers import check_lowp_against_oracle, oracle_index_from_gpu
    pk, ixs, X, Q = lowp_setup
    ix = ixs[precision]
    oix = oracle_index_from_gpu(X, ix)
    if precision == "bf16":
        rank = [mo.quantize_bf16(P.astype(np.float32)) for P in oix.protos]
        leaf = mo.quantize_bf16(X)
        factor = 4
    else:
        rank = oix.protos
        code, scale = mo.quantize_fp8(X)
        leaf = code * scale[:, None]
        factor = 48
    g = np.random.default_rng(23)
    srv = pk.MaskServer(ix, arena_bytes=64 << 20, max_batch_queries=2048, n_streams=3,
                        batch_window_us=10_000)
    reqs, tickets = [], []
    pos = 0
    for _ in range(30):
        n = int(g.integers(1, 12))
        k = int(g.integers(1, 100))
        r = int(g.choice([8, 32]))
        reqs.append((pos, n, k, r))
        tickets.append(srv.submit(Q[pos:pos + n], k, r))
        pos += n
    res = _drain(srv, tickets)
    srv.close()
    checked = 0
    for (p, n, k, r), t in zip(reqs, tickets):
        ids, dist, _ = res[t]
        ids, dist = ids.reshape(n, k), dist.reshape(n, k)
        beams = [r] * oix.n_levels
        i1, d1, sel = (host(x) for x in pk.mask_query_beams(ix, dev(Q[p:p + n]), k, beams,
                                                             debug=True))
        assert np.array_equal(ids, i1) and np.array_equal(dist, d1)
        fails = check_lowp_against_oracle(oix, Q[p:p + n], k, beams, ids, dist, sel, rank,
                                          leaf, factor)
        assert not fails, (p, n, k, r, fails[:2])
        checked += n
    assert checked >= 100


# ----------------------------------------------- beam profile of a request

PROFILE = [3, 3, 24]  # eighths of r per level, top first: r = 8 -> (3, 3, 24)


def _profile_beams(r, n_levels):
    prof = PROFILE[-n_levels:]
    return [max(1, (r * e + 7) // 8) for e in prof]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_profile_ragged_equals_beams_alone(precision):
    # a ragged batch with a beam profile: each query keeps ceil(r_i e / 8)
    # prototypes per level and equals mask_query_beams alone with those beams
    import torch
    import paper_2208_02734_amd as pk
    pk.lib()
    mix = datagen.mixture_params(330, 60, 48, sigma_mode="loguniform", sigma_low=0.1,
                                 sigma_high=3.0)
    X = datagen.sample_mixture(mix, 50_000, 331)
    Q = datagen.sample_mixture(mix, 60, 332)
    ix = pk.mask_build(dev(X), [(10, 200), (1, 200), (1, 20)], iters=5, seed=3,
                       precision=precision)
    g = np.random.default_rng(31)
    ks = g.integers(1, 100, size=60).astype(np.int32)
    rs = g.choice([8, 32], size=60).astype(np.int32)
    ids, dist, off = pk.mask_query_ragged(ix, dev(Q), torch.from_numpy(ks),
                                          torch.from_numpy(rs), beam_eighths=PROFILE)
    ids, dist, off = host(ids), host(dist), host(off)
    for i in range(60):
        beams = _profile_beams(int(rs[i]), 3)
        i1, d1 = pk.mask_query_beams(ix, dev(Q[i:i + 1]), int(ks[i]), beams)
        assert np.array_equal(ids[off[i]:off[i + 1]], host(i1)[0]), (i, beams)
        assert np.array_equal(dist[off[i]:off[i + 1]], host(d1)[0]), (i, beams)
    with pytest.raises(pk.MaskError) as e:  # a profile beam above 2048 at r_max
        pk.mask_query_ragged(ix, dev(Q), torch.from_numpy(ks), torch.from_numpy(rs),
                             r_max=1000, beam_eighths=PROFILE)
    assert e.value.status == 1
    ix.free()


def test_server_with_a_beam_profile_serves_the_profile_beams(lowp_setup):
    pk, ixs, X, Q = lowp_setup
    ix = ixs["bf16"]
    prof = PROFILE[-2:]  # two levels: r = 8 -> (3, 24), r = 32 -> (12, 96)
    srv = pk.MaskServer(ix, arena_bytes=64 << 20, max_batch_queries=2048, n_streams=3,
                        batch_window_us=10_000, beam_eighths=prof)
    g = np.random.default_rng(37)
    reqs, tickets = [], []
    pos = 0
    for _ in range(40):
        n = int(g.integers(1, 16))
        k = int(g.integers(1, 100))
        r = int(g.choice([8, 32]))
        reqs.append((pos, n, k, r))
        tickets.append(srv.submit(Q[pos:pos + n], k, r))
        pos += n
    res = _drain(srv, tickets)
    st = srv.stats()
    srv.close()
    assert st["batches"] < 40
    for (p, n, k, r), t in zip(reqs, tickets):
        ids, dist, _ = res[t]
        beams = [max(1, (r * e + 7) // 8) for e in prof]
        i1, d1 = pk.mask_query_beams(ix, dev(Q[p:p + n]), k, beams)
        assert np.array_equal(ids, host(i1)), (p, n, k, r)
        assert np.array_equal(dist, host(d1)), (p, n, k, r)
