"""The seeded generators are deterministic and have the stated structure."""
import hashlib

import numpy as np

import datagen


def _h(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_mixture_is_deterministic():
    a = datagen.config_small(n=3000, n_queries=50)
    b = datagen.config_small(n=3000, n_queries=50)
    assert _h(a.X) == _h(b.X) and _h(a.Q) == _h(b.Q)
    assert a.X.dtype == np.float32 and a.X.shape == (3000, 16)
    # queries are fresh draws, not dataset rows
    assert not np.any((a.X[None, :, :] == a.Q[:, None, :]).all(-1))


def test_mixture_params():
    m = datagen.mixture_params(5, 40, 8, sigma_mode="loguniform", sigma_low=0.1, sigma_high=3.0)
    assert m.means.min() >= -10 and m.means.max() <= 10
    assert m.sigmas.min() >= 0.1 and m.sigmas.max() <= 3.0
    assert abs(m.weights.sum() - 1) < 1e-12


def test_sparse_structure():
    S = datagen.sample_sparse(500, 2000, 20, seed=9)
    assert S.indptr[-1] == 500 * 20
    for i in range(500):
        cols = S.indices[S.indptr[i]:S.indptr[i + 1]]
        assert np.all(np.diff(cols) > 0)
        v = S.values[S.indptr[i]:S.indptr[i + 1]].astype(np.float64)
        assert abs(np.sqrt((v * v).sum()) - 1) < 1e-6
        assert np.all(v > 0)
    # Zipf head: column 0 is the most frequent
    counts = np.bincount(S.indices, minlength=2000)
    assert counts.argmax() < 5


def test_request_stream():
    rs = datagen.request_stream(1000.0, 2.0, seed=3, pool_rows=100_000)
    assert np.all(np.diff(rs.t_arrival) > 0)
    assert rs.n_queries.min() >= 1 and rs.n_queries.max() <= 512
    assert rs.k.min() >= 1 and rs.k.max() <= 100
    assert set(np.unique(rs.r).tolist()) <= {8, 32}
    assert 1500 < rs.t_arrival.size < 2500
