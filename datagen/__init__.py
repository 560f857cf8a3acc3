"""Seeded synthetic inputs for the MASK hot path.

This module only draws random inputs.  It holds none of the method's
arithmetic (no distances, no k-means, no permutation of the method), so both
the FP64 oracle and the HIP path can take their inputs from here without
sharing any code with each other.

Every array is drawn with numpy's ``Generator(PCG64(seed))`` and stored as
float32 (draws are made in float64 and rounded once).  The shapes, value
distributions and structure follow the workloads the paper evaluates
(Gaussian clouds, Section 4.2 "Synthetic dataset results"; a sparse,
non-negative, high-dimensional TF-IDF-like corpus, Section 4.3), scaled to
the sizes stated in each ``config_*`` function.  The sparse generator stands
in for the Reuters-21578 corpus, which is not used or reproduced here.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

DATA_SEED_BASE = 20220805
QUERY_SEED_OFFSET = 1000


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclasses.dataclass
class Mixture:
    """Parameters of an isotropic Gaussian mixture."""

    means: np.ndarray  # (n_comp, d) float64
    sigmas: np.ndarray  # (n_comp,) float64
    weights: np.ndarray  # (n_comp,) float64, sums to 1


def mixture_params(
    seed: int,
    n_comp: int,
    d: int,
    mean_low: float = -10.0,
    mean_high: float = 10.0,
    sigma_mode: str = "uniform",
    sigma_low: float = 0.3,
    sigma_high: float = 2.0,
) -> Mixture:
    """Component means U[mean_low, mean_high]^d, sigmas uniform or
    log-uniform in [sigma_low, sigma_high], weights Dirichlet(1)."""
    g = _rng(seed)
    means = g.uniform(mean_low, mean_high, size=(n_comp, d))
    if sigma_mode == "uniform":
        sigmas = g.uniform(sigma_low, sigma_high, size=n_comp)
    elif sigma_mode == "loguniform":
        sigmas = np.exp(g.uniform(math.log(sigma_low), math.log(sigma_high), size=n_comp))
    else:
        raise ValueError(f"unknown sigma_mode {sigma_mode!r}")
    weights = g.dirichlet(np.ones(n_comp))
    return Mixture(means=means, sigmas=sigmas, weights=weights)


def sample_mixture(mix: Mixture, n: int, seed: int, block: int = 1 << 20,
                   return_components: bool = False):
    """n points from the mixture, float32, drawn block by block so that
    10M x 96 never needs a float64 copy of the whole array."""
    g = _rng(seed)
    d = mix.means.shape[1]
    comp = g.choice(mix.weights.shape[0], size=n, p=mix.weights)
    out = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, block):
        e = min(n, s + block)
        c = comp[s:e]
        z = g.standard_normal((e - s, d))
        z *= mix.sigmas[c, None]
        z += mix.means[c]
        out[s:e] = z
    if return_components:
        return out, comp.astype(np.int32)
    return out


@dataclasses.dataclass
class DenseConfig:
    name: str
    X: np.ndarray
    Q: np.ndarray
    levels: list  # [(n_chunks, k)] bottom-up
    iters: int
    k: int
    r_values: list
    description: str


def _dense_config(name, cfg_index, n, d, n_comp, sigma_mode, sigma_low, sigma_high,
                  n_queries, levels, iters, k, r_values, description,
                  n_override: Optional[int] = None, q_override: Optional[int] = None):
    seed = DATA_SEED_BASE + cfg_index
    mix = mixture_params(seed, n_comp, d, sigma_mode=sigma_mode,
                         sigma_low=sigma_low, sigma_high=sigma_high)
    n_eff = n if n_override is None else n_override
    q_eff = n_queries if q_override is None else q_override
    X = sample_mixture(mix, n_eff, seed + 1)
    Q = sample_mixture(mix, q_eff, seed + QUERY_SEED_OFFSET)
    return DenseConfig(name=name, X=X, Q=Q, levels=levels, iters=iters, k=k,
                       r_values=r_values, description=description)


def config_small(n: Optional[int] = None, n_queries: Optional[int] = None) -> DenseConfig:
    """20,000 points, d = 16, 50 Gaussian components (means U[-10,10],
    sigma U[0.3,2], Dirichlet(1) weights); 2 levels: 10 chunks x 100
    prototypes, then one chunk of 50; 30 Lloyd iterations; 1,000 queries
    from the same mixture, k = 10, r = 5."""
    return _dense_config(
        "mixture-20k-d16", 1, 20_000, 16, 50, "uniform", 0.3, 2.0, 1_000,
        [(10, 100), (1, 50)], 30, 10, [1, 5, 20, 50],
        "20k x 16 Gaussian mixture (50 comps), levels 10x100 -> 1x50",
        n_override=n, q_override=n_queries)


def config_scale(n: Optional[int] = None, n_queries: Optional[int] = None) -> DenseConfig:
    """1,000,000 points, d = 128, 1,000 components with log-uniform sigma
    in [0.1, 3]; 3 levels: 100 chunks x 1,000, one chunk of 5,000, one chunk
    of 100; 30 Lloyd iterations; 10,000 queries, k = 10."""
    return _dense_config(
        "mixture-1M-d128", 2, 1_000_000, 128, 1_000, "loguniform", 0.1, 3.0, 10_000,
        [(100, 1_000), (1, 5_000), (1, 100)], 30, 10, [4, 16, 64, 128, 256],
        "1M x 128 Gaussian mixture (1000 comps), levels 100x1000 -> 1x5000 -> 1x100",
        n_override=n, q_override=n_queries)


def scale_insertions(n_new: int) -> np.ndarray:
    """Fresh rows from the mixture of ``config_scale`` (same components), for
    dynamic insertion into its index."""
    seed = DATA_SEED_BASE + 2
    mix = mixture_params(seed, 1_000, 128, sigma_mode="loguniform", sigma_low=0.1,
                         sigma_high=3.0)
    return sample_mixture(mix, n_new, seed + 2 * QUERY_SEED_OFFSET)


def precision_insertions(n_new: int) -> np.ndarray:
    """Fresh rows from the mixture of ``config_precision`` (same components),
    for dynamic insertion into its index."""
    seed = DATA_SEED_BASE + 4
    mix = mixture_params(seed, 10_000, 96, sigma_mode="loguniform", sigma_low=0.1,
                         sigma_high=3.0)
    return sample_mixture(mix, n_new, seed + 2 * QUERY_SEED_OFFSET)


def config_precision(n: Optional[int] = None, n_queries: Optional[int] = None,
                     levels=None) -> DenseConfig:
    """10,000,000 points, d = 96, 10,000 components, log-uniform sigma in
    [0.1, 3]; 100,000 queries, k = 10.  Level sizes are not fixed by the
    workload statement; the default gives every group about one prototype
    per mixture component (as many prototypes as resources allow): 10
    groups of 1,000,000 rows x 10,000 prototypes, then one group of
    10,000, then 100."""
    if levels is None:
        levels = [(10, 10_000), (1, 10_000), (1, 100)]
    return _dense_config(
        "mixture-10M-d96", 4, 10_000_000, 96, 10_000, "loguniform", 0.1, 3.0, 100_000,
        levels, 30, 10, [8, 32, 64, 128],
        "10M x 96 Gaussian mixture (10000 comps)",
        n_override=n, q_override=n_queries)


@dataclasses.dataclass
class SparseMatrix:
    """CSR matrix with int64 row pointers, int32 column ids, float32 values."""

    indptr: np.ndarray
    indices: np.ndarray
    values: np.ndarray
    n_cols: int

    @property
    def n_rows(self) -> int:
        return self.indptr.shape[0] - 1

    def to_dense(self) -> np.ndarray:
        out = np.zeros((self.n_rows, self.n_cols), dtype=np.float32)
        rows = np.repeat(np.arange(self.n_rows), np.diff(self.indptr))
        out[rows, self.indices] = self.values
        return out


def sample_sparse(n_rows: int, n_cols: int, nnz_per_row: int, seed: int,
                  zipf_s: float = 1.1, ln_mu: float = 0.0, ln_sigma: float = 1.0) -> SparseMatrix:
    """Non-negative sparse rows: exactly ``nnz_per_row`` distinct columns per
    row, drawn one after another without replacement with probability
    proportional to (j+1)^-zipf_s (draw with replacement, keep first
    occurrences in draw order); values LogNormal(ln_mu, ln_sigma); each row
    scaled to unit L2 norm.  Column ids are sorted within a row."""
    if nnz_per_row > n_cols:
        raise ValueError("nnz_per_row > n_cols")
    g = _rng(seed)
    p = (np.arange(1, n_cols + 1, dtype=np.float64)) ** (-zipf_s)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    indices = np.empty((n_rows, nnz_per_row), dtype=np.int32)
    block = 4096
    for s in range(0, n_rows, block):
        e = min(n_rows, s + block)
        rows_left = np.arange(s, e)
        draws = 4 * nnz_per_row + 64  # doubled only for this block's retries
        while rows_left.size:
            m = rows_left.size
            u = g.random((m, draws))
            cols = np.minimum(np.searchsorted(cdf, u, side="right"), n_cols - 1)
            # first occurrence of each value in draw order
            order = np.argsort(cols, axis=1, kind="stable")
            sc = np.take_along_axis(cols, order, axis=1)
            first = np.ones_like(sc, dtype=bool)
            first[:, 1:] = sc[:, 1:] != sc[:, :-1]
            is_first = np.zeros_like(first)
            np.put_along_axis(is_first, order, first, axis=1)
            rank = np.cumsum(is_first, axis=1)
            ok = rank[:, -1] >= nnz_per_row
            keep = is_first & (rank <= nnz_per_row)
            good_rows = np.nonzero(ok)[0]
            if good_rows.size:
                sel = cols[good_rows][keep[good_rows]].reshape(good_rows.size, nnz_per_row)
                indices[rows_left[good_rows]] = np.sort(sel, axis=1)
            rows_left = rows_left[~ok]
            draws *= 2
    values = np.exp(g.normal(ln_mu, ln_sigma, size=(n_rows, nnz_per_row)))
    values /= np.sqrt((values * values).sum(axis=1, keepdims=True))
    indptr = np.arange(0, (n_rows + 1) * nnz_per_row, nnz_per_row, dtype=np.int64)
    return SparseMatrix(indptr=indptr, indices=indices.reshape(-1),
                        values=values.astype(np.float32).reshape(-1), n_cols=n_cols)


@dataclasses.dataclass
class SparseConfig:
    name: str
    X: SparseMatrix
    Q: SparseMatrix
    levels: list
    iters: int
    k: int
    r_values: list
    description: str


def config_sparse(n: Optional[int] = None, n_queries: Optional[int] = None,
                  n_cols: int = 10_000, nnz_per_row: int = 100, levels=None) -> SparseConfig:
    """200,000 rows x 10,000 columns, 1% non-zeros (100 per row), Zipf(1.1)
    column popularity, LogNormal(0,1) values, unit L2 rows; levels 20 chunks
    x 2,000, one chunk of 2,000, one chunk of 50; 5,000 queries, k = 10."""
    seed = DATA_SEED_BASE + 3
    n_eff = 200_000 if n is None else n
    q_eff = 5_000 if n_queries is None else n_queries
    if levels is None:
        levels = [(20, 2_000), (1, 2_000), (1, 50)]
    X = sample_sparse(n_eff, n_cols, nnz_per_row, seed + 1)
    Q = sample_sparse(q_eff, n_cols, nnz_per_row, seed + QUERY_SEED_OFFSET)
    return SparseConfig(name="sparse-200k-D10000", X=X, Q=Q, levels=levels, iters=30, k=10,
                        r_values=[4, 16, 64], description="CSR 200k x 10000, 100 nnz/row")


@dataclasses.dataclass
class RequestStream:
    """Poisson arrivals; each request carries (n_queries, k, r) and the
    offset of its queries in a pre-drawn query pool."""

    t_arrival: np.ndarray  # float64 seconds
    n_queries: np.ndarray  # int32, log-uniform in [1, max_queries]
    k: np.ndarray  # int32, uniform in [k_low, k_high]
    r: np.ndarray  # int32, drawn from r_choices
    pool_offset: np.ndarray  # int64 start row in the query pool


def request_stream(rate: float, duration: float, seed: int, pool_rows: int,
                   max_queries: int = 512, k_low: int = 1, k_high: int = 100,
                   r_choices=(8, 32)) -> RequestStream:
    g = _rng(seed)
    n_exp = int(rate * duration * 1.5) + 16
    gaps = g.exponential(1.0 / rate, size=n_exp)
    t = np.cumsum(gaps)
    t = t[t < duration]
    m = t.shape[0]
    nq = np.floor(np.exp(g.uniform(0.0, math.log(max_queries + 1), size=m))).astype(np.int32)
    nq = np.clip(nq, 1, max_queries)
    kk = g.integers(k_low, k_high + 1, size=m).astype(np.int32)
    rr = np.asarray(r_choices, dtype=np.int32)[g.integers(0, len(r_choices), size=m)]
    off = g.integers(0, max(1, pool_rows - max_queries), size=m).astype(np.int64)
    return RequestStream(t_arrival=t, n_queries=nq, k=kk, r=rr, pool_offset=off)


# Standard deviation of each cloud by degree of overlap.  The eight means sit
# on a circle of radius 10, so adjacent means are 2 * 10 * sin(pi / 8) = 7.65
# apart: 15 sigma with no overlap, 3.8 sigma with moderate overlap and 1.9
# sigma with severe overlap.
CLOUD_SIGMA = {"none": 0.5, "moderate": 2.0, "severe": 4.0}


@dataclasses.dataclass
class Clouds:
    X: np.ndarray       # (8 * npc, 2) float32, cloud-major order
    labels: np.ndarray  # (8 * npc,) int32 cloud index


def eight_clouds(npc: int, overlap: str, seed: int) -> Clouds:
    """The synthetic benchmark of Section 4.2: eight isotropic Gaussian clouds
    in the plane with npc points each; the paper does not give the means and
    spreads, so they are the ones stated above."""
    sigma = CLOUD_SIGMA[overlap]
    g = _rng(seed)
    ang = 2.0 * math.pi * np.arange(8) / 8.0
    means = 10.0 * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    X = np.repeat(means, npc, axis=0) + sigma * g.standard_normal((8 * npc, 2))
    labels = np.repeat(np.arange(8, dtype=np.int32), npc)
    return Clouds(X=X.astype(np.float32), labels=labels)
