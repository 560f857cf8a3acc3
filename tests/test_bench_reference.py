"""The benchmark's recall reference (an FP64 exhaustive search written in
bench.py, which may not call the oracle outside its CPU-baseline leg)
agrees with the oracle's exhaustive search and recall.  CPU only."""
import importlib.util
import os

import numpy as np

from oracle import compare as oc
from oracle import mask_oracle as mo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_exact_knn64_matches_the_oracle():
    b = _bench()
    g = np.random.default_rng(5)
    X = (g.standard_normal((30000, 24)) * 3).astype(np.float32)
    X[100] = X[7]  # an exact tie, broken by the lower id
    Q = np.concatenate([g.standard_normal((40, 24)).astype(np.float32), X[[7, 100, 5]]])
    ids, dist = b.exact_knn64(X, Q, 10, block=4096)
    tids, tdist = mo.exact_knn(X, Q, 10)
    assert np.array_equal(ids, tids)
    np.testing.assert_allclose(dist, tdist, rtol=1e-12, atol=0)


def test_recall_matches_the_oracle_comparator():
    b = _bench()
    g = np.random.default_rng(6)
    X = g.standard_normal((5000, 8)).astype(np.float32)
    Q = g.standard_normal((30, 8)).astype(np.float32)
    tids, tdist = mo.exact_knn(X, Q, 10)
    got = tids.copy()
    got[::3, 9] = (got[::3, 9] + 17) % 5000  # some misses
    got[1, 4] = -1
    r1 = b.recall_at_k(X, Q, got, tids, tdist, 10)
    r2 = oc.recall_at_k(got, tids, tdist, oc.true_distances(X, Q, got), 10)
    assert r1 == r2 and r1 < 1.0


def test_rerank_set_follows_the_oracle_rule():
    b = _bench()
    for form in ("bf16", "fp8"):
        for beams in ([3, 3, 24], [4, 8, 48], [2, 2, 16], [8, 16, 96]):
            f = b.RERANK[form] or 4
            assert b.rerank_set(form, 10, beams) == mo.rerank_size(10, beams, f)


def test_profile_beams_round_up():
    b = _bench()
    assert b.profile_beams([3, 3, 24], 8) == [3, 3, 24]
    assert b.profile_beams([3, 3, 24], 32) == [12, 12, 96]
    assert b.profile_beams([3, 4, 28], 1) == [1, 1, 4]
