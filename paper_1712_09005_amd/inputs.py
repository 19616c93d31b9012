"""Seeded synthetic inputs for the t-SNE gradient path.

This module builds *inputs only*: embeddings Y, a random-graph P in CSR form,
and high-dimensional point clouds X for the perplexity workloads (their
affinities are computed from X by the library, or by the oracle in tests).
It holds none of the method's arithmetic (no neighbours, bandwidths,
interpolation or forces), so both the GPU library's tests and the CPU oracle
can be fed from it without sharing any of the method's code.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64).  Mixture
components are equiprobable: each point's label is drawn uniformly, then the
point is drawn from N(centre, sd^2 I).

The paper measures on datasets that are not available here (Infinite MNIST,
retinal and brain single-cell data, Section 2.5 and Section 5); the Gaussian
mixtures below stand in for them at the paper's scale of one million points.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "CSR", "mixture_embedding", "random_graph_P", "mixture_highdim",
    "serving_jobs", "poisson_arrivals", "config_inputs",
    "low_rank_factors", "pca_matrix", "pca_omega",
]


@dataclasses.dataclass
class CSR:
    """Sparse symmetric P: ``row_ptr`` int64 [N+1], ``col`` int32 [nnz]
    (sorted within each row), ``val`` float32 [nnz]; sum(val) == 1."""
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])


def mixture_embedding(n: int, s: int, n_clusters: int, lo: float, hi: float,
                      sd: float, seed: int, dtype=np.float32) -> np.ndarray:
    """Y [n, s]: ``n_clusters`` isotropic Gaussians with centres uniform in
    [lo, hi]^s and standard deviation ``sd``.  Row-major, C-contiguous."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(lo, hi, size=(n_clusters, s))
    labels = rng.integers(0, n_clusters, size=n)
    y = centres[labels] + sd * rng.standard_normal(size=(n, s))
    return np.ascontiguousarray(y.astype(dtype))


def _csr_from_edges(n: int, r: np.ndarray, c: np.ndarray, w: np.ndarray) -> CSR:
    import scipy.sparse as sp
    a = sp.csr_matrix((w, (r, c)), shape=(n, n))   # sums repeated (r, c)
    a = (a + a.T).tocsr()
    a.sum_duplicates()
    a.sort_indices()
    total = float(a.data.sum())
    val = (a.data / total).astype(np.float32)
    return CSR(row_ptr=a.indptr.astype(np.int64),
               col=a.indices.astype(np.int32), val=val)


def random_graph_P(n: int, k: int, seed: int) -> CSR:
    """Symmetric P from a random k-neighbour graph.

    Each row draws k/2 out-neighbours j != i uniformly (a repeated draw merges
    with the earlier one), each directed edge gets weight exp(-u) with
    u ~ U(0, 5), then W + W^T is normalised to sum 1.  The average row degree
    is about k, which gives ~9e7 non-zeros at n = 1e6, k = 90."""
    if n < 2:
        raise ValueError("random_graph_P needs n >= 2")
    half = max(1, k // 2)
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n, dtype=np.int64), half)
    cols = rng.integers(0, n - 1, size=n * half, dtype=np.int64)
    cols += cols >= rows                      # skip the diagonal
    w = np.exp(-rng.uniform(0.0, 5.0, size=n * half))
    return _csr_from_edges(n, rows, cols, w)


def mixture_highdim(n: int, d: int, n_clusters: int, centre_sd: float,
                    seed: int) -> np.ndarray:
    """X [n, d] float32: unit-variance clusters with centres ~ N(0, centre_sd^2 I)."""
    rng = np.random.default_rng(seed)
    centres = centre_sd * rng.standard_normal(size=(n_clusters, d))
    labels = rng.integers(0, n_clusters, size=n)
    x = centres[labels] + rng.standard_normal(size=(n, d))
    return np.ascontiguousarray(x.astype(np.float32))


def serving_jobs(n_jobs: int = 64, n_min: int = 5_000, n_max: int = 200_000):
    """The serving workload's raw inputs: job j uses seed 100 + j; N
    log-uniform in [n_min, n_max], K ~ U{5..30} unit-variance clusters in
    50-d with centres N(0, 25 I), Y0 ~ N(0, 1e-4 I).  Returns a list of
    (Y0 float32 [N, 2], X float32 [N, 50]); the affinities P are built from X
    by the caller (90 nearest neighbours at perplexity 30)."""
    out = []
    for j in range(n_jobs):
        rng = np.random.default_rng(100 + j)
        n = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
        kc = int(rng.integers(5, 31))
        x = mixture_highdim(n, 50, kc, 5.0, seed=100 + j)
        y = (1e-2 * rng.standard_normal((n, 2))).astype(np.float32)
        out.append((np.ascontiguousarray(y), x))
    return out


def poisson_arrivals(n: int, rate: float, seed: int = 7) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def config_inputs(name: str, small: bool = False):
    """Inputs of the named workload.  Returns a dict with ``Y`` (float32
    [N, s]), either ``P`` (CSR) or ``X`` (float32 [N, 50], from which P is
    built with 90 nearest neighbours at perplexity 30) and workload metadata.

    c1: N=2048 2-D check; c3: N=1e6 2-D; c4: N=1e6 1-D; c2: N=1e5 2-D full run
    from a 50-d mixture.  ``small`` shrinks c2/c3/c4 for CPU tests while
    keeping their structure."""
    if name == "c1":
        y = mixture_embedding(2048, 2, 10, -30.0, 30.0, 2.0, seed=0)
        return dict(Y=y, P=random_graph_P(2048, 90, seed=1), s=2,
                    policy="paper", min_intervals=50)
    if name == "c3":
        n = 20_000 if small else 1_000_000
        y = mixture_embedding(n, 2, 50, -95.0, 95.0, 2.0, seed=0)
        return dict(Y=y, P=random_graph_P(n, 90, seed=1), s=2,
                    policy="fixed", min_intervals=1)
    if name == "c4":
        n = 20_000 if small else 1_000_000
        y = mixture_embedding(n, 1, 30, -195.0, 195.0, 1.5, seed=0)
        return dict(Y=y, P=random_graph_P(n, 90, seed=1), s=1,
                    policy="fixed", min_intervals=1)
    if name == "c2":
        n = 5_000 if small else 100_000
        x = mixture_highdim(n, 50, 20, 5.0, seed=0)
        rng = np.random.default_rng(2)
        y = np.ascontiguousarray((1e-2 * rng.standard_normal((n, 2))).astype(np.float32))
        return dict(Y=y, X=x, s=2, policy="paper", min_intervals=50)
    raise KeyError(name)


def low_rank_factors(m: int, n: int, rank: int, seed: int, s_max: float = 1.0,
                     s_min: float = 1e-2):
    """Planted factors of a rank-`rank` matrix A = U0 diag(s) V0^T with
    exactly these singular values: U0 (m x rank) and V0 (n x rank) have
    orthonormal columns, cosine vectors of distinct random frequencies,
    sqrt(2/len) cos(pi f (2i + 1) / (2 len)), with random row signs and a
    random row order; s decreases geometrically from s_max to s_min.
    (Section 6.3 measures on a random rank-50 matrix of doubles.)"""
    rng = np.random.default_rng(seed)

    def basis(length: int) -> np.ndarray:
        f = rng.choice(np.arange(1, length), size=rank, replace=False).astype(np.float64)
        i = np.arange(length, dtype=np.float64)[:, None]
        B = np.sqrt(2.0 / length) * np.cos(np.pi * f[None, :] * (2.0 * i + 1.0) / (2.0 * length))
        B *= rng.choice(np.array([-1.0, 1.0]), size=(length, 1))
        return np.ascontiguousarray(B[rng.permutation(length)])

    U0 = basis(m)
    V0 = basis(n)
    s = s_max * (s_min / s_max) ** (np.arange(rank, dtype=np.float64) / max(rank - 1, 1))
    return U0, s, V0


def pca_matrix(m: int, n: int, rank: int, seed: int, noise: float = 0.0, **kw):
    """A = U0 diag(s) V0^T (+ noise * standard normal entries), m x n FP64,
    with the planted factors of low_rank_factors."""
    U0, s, V0 = low_rank_factors(m, n, rank, seed, **kw)
    A = (U0 * s) @ V0.T
    if noise > 0.0:
        A += noise * np.random.default_rng(seed + 1).standard_normal((m, n))
    return np.ascontiguousarray(A), U0, s, V0


def pca_omega(n: int, l: int, seed: int) -> np.ndarray:
    """The random n x l matrix of the first step of Algorithm 2 (Section 6):
    entries uniform on [-1, 1)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, l))
