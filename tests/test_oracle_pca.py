"""Pins of the randomised-PCA oracle (Section 6, Algorithm 2) against what
the mathematics fixes: planted singular values and vectors of exactly
low-rank matrices, the exact SVD of dense matrices within the accuracy the
power iterations reach, invariants of the factors, and the LU
renormalisation's defining properties."""
import numpy as np
import pytest

from oracle import pca as opca
from paper_1712_09005_amd import inputs


def _subspace_cos(U, U0):
    """Per-column |<u_j, u0_j>|: 1 when the columns agree up to sign."""
    return np.abs(np.sum(U * U0, axis=0))


@pytest.mark.parametrize("m,n,its", [(500, 300, 0), (500, 300, 2), (300, 520, 1)])
def test_planted_rank_is_recovered_exactly(m, n, its):
    # rank 6 <= l = 8: A Omega already spans the range (Section 6.1), so the
    # planted singular values and vectors come back to rounding, for any its
    A, U0, s0, V0 = inputs.pca_matrix(m, n, 6, seed=3, s_min=0.05)
    om = inputs.pca_omega(n, 8, seed=4)
    U, s, V = opca.oocpca(A, om, k=6, its=its, b=64)
    np.testing.assert_allclose(s, s0, rtol=1e-12)
    assert _subspace_cos(U, U0).min() > 1 - 1e-10
    assert _subspace_cos(V, V0).min() > 1 - 1e-10
    np.testing.assert_allclose(U.T @ U, np.eye(6), atol=1e-12)
    np.testing.assert_allclose(V.T @ V, np.eye(6), atol=1e-12)
    np.testing.assert_allclose((U * s) @ V.T, A, atol=1e-12)


def test_dense_matrix_matches_the_exact_svd():
    # a decaying spectrum plus noise: the top singular values converge to
    # those of the exact SVD with the power iterations
    A, _, _, _ = inputs.pca_matrix(400, 300, 20, seed=5, noise=1e-4, s_min=0.02)
    sx = np.linalg.svd(A, compute_uv=False)
    U, s, V = opca.oocpca(A, inputs.pca_omega(300, 12, seed=6), k=8, its=4, b=100)
    np.testing.assert_allclose(s, sx[:8], rtol=1e-6)
    # Rayleigh-Ritz values never exceed the true ones
    assert np.all(s <= sx[:8] * (1 + 1e-12))
    # the residual of the rank-8 approximation approaches sigma_9
    res = np.linalg.norm(A - (U * s) @ V.T, 2)
    assert res <= sx[8] * (1 + 1e-6)


def test_power_iterations_improve_a_slow_spectrum():
    # singular values 1 / (1 + j / 4): without power iterations the top-k
    # values are visibly short; with more iterations the error falls
    rng = np.random.default_rng(8)
    m, n = 300, 200
    Ua, _ = np.linalg.qr(rng.standard_normal((m, n)))
    Va, _ = np.linalg.qr(rng.standard_normal((n, n)))
    sx = 1.0 / (1.0 + np.arange(n) / 4.0)
    A = (Ua * sx) @ Va.T
    om = inputs.pca_omega(n, 7, seed=9)
    err = []
    for its in (0, 1, 3, 6):
        _, s, _ = opca.oocpca(A, om, k=5, its=its, b=50)
        err.append(np.max(np.abs(s - sx[:5]) / sx[:5]))
    assert err[0] > 1e-2
    assert err[0] > err[1] > err[2] > err[3]
    assert err[3] < 1e-3


def test_blocking_only_reorders_sums():
    # b rows at a time (Section 6.2): any b gives the same factors to rounding
    A, _, _, _ = inputs.pca_matrix(257, 190, 10, seed=10, noise=1e-3)
    om = inputs.pca_omega(190, 9, seed=11)
    ref = opca.oocpca(A, om, k=7, its=2, b=257)
    for b in (1, 7, 64, 1000):
        U, s, V = opca.oocpca(A, om, k=7, its=2, b=b)
        np.testing.assert_allclose(s, ref[1], rtol=1e-12)
        assert _subspace_cos(U, ref[0]).min() > 1 - 1e-10
        assert _subspace_cos(V, ref[2]).min() > 1 - 1e-10


def test_block_products():
    rng = np.random.default_rng(12)
    A = rng.standard_normal((53, 17))
    X = rng.standard_normal((17, 3))
    Y = rng.standard_normal((53, 4))
    np.testing.assert_allclose(opca.apply_A(A, X, 10), A @ X, rtol=1e-14, atol=1e-13)
    np.testing.assert_allclose(opca.apply_At(A, Y, 10), A.T @ Y, rtol=1e-14, atol=1e-13)


def test_lu_renormalisation():
    # L: a row permutation of a unit lower-trapezoidal matrix, entries <= 1
    # in size (partial pivoting), with the span of Y
    rng = np.random.default_rng(13)
    Y = rng.standard_normal((40, 5)) @ rng.standard_normal((5, 5))
    L = opca.lu_renorm(Y)
    assert np.abs(L).max() <= 1 + 1e-15
    coef, *_ = np.linalg.lstsq(L, Y, rcond=None)
    np.testing.assert_allclose(L @ coef, Y, atol=1e-12)
    # its rows, ordered by the pivots, form a unit lower-trapezoidal matrix
    rows = []
    for j in range(5):
        cand = [i for i in range(40) if i not in rows and abs(L[i, j] - 1) < 1e-15
                and np.all(np.abs(L[i, j + 1:]) == 0)]
        assert cand, j
        rows.append(cand[0])
    assert np.all(np.abs(np.triu(L[rows], 1)) == 0)


def test_argument_checks():
    A = np.zeros((10, 8))
    with pytest.raises(ValueError):
        opca.oocpca(A, np.zeros((8, 9)), k=2, its=1, b=4)   # l >= min(m, n)
    with pytest.raises(ValueError):
        opca.oocpca(A, np.zeros((8, 3)), k=4, its=1, b=4)   # k > l
    with pytest.raises(ValueError):
        opca.oocpca(A, np.zeros((7, 3)), k=2, its=1, b=4)   # omega rows != n


def test_planted_factors_are_orthonormal():
    U0, s, V0 = inputs.low_rank_factors(1000, 600, 12, seed=14)
    np.testing.assert_allclose(U0.T @ U0, np.eye(12), atol=1e-12)
    np.testing.assert_allclose(V0.T @ V0, np.eye(12), atol=1e-12)
    assert np.all(np.diff(s) < 0) and s[0] == 1.0 and abs(s[-1] - 1e-2) < 1e-15
