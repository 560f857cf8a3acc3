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
