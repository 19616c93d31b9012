"""Randomised PCA on the device (tsne_pca, Algorithm 2 of Section 6) against
the oracle on the same A and Omega: singular values and singular vectors
(up to the sign of each column), with A in device memory and streamed from
host memory in b-row blocks; planted low-rank matrices at a sample of the
paper's 30,000-column shape checked against their planted factors."""
import numpy as np
import pytest
import torch

from oracle import pca as opca
from paper_1712_09005_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def PCA():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_09005_amd import pca, tsne
    tsne.lib()
    return pca


def _cos(U, U0):
    return np.abs(np.sum(U * U0, axis=0))


def _check(U, s, V, ref, s_rtol=1e-9, v_tol=1e-8):
    Uo, so, Vo = ref
    np.testing.assert_allclose(s, so, rtol=s_rtol, atol=1e-13 * so[0])
    assert _cos(U, Uo).min() > 1 - v_tol
    assert _cos(V, Vo).min() > 1 - v_tol
    k = s.shape[0]
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-11)
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-11)


@pytest.mark.parametrize("m,n,rank,k,l,its", [
    (3001, 517, 30, 10, 12, 2),     # ragged row and column tiles
    (517, 3001, 30, 10, 12, 2),     # wide
    (2000, 300, 40, 6, 8, 0),       # no power iteration
    (1200, 700, 60, 20, 64, 1),     # the largest l
    (20000, 517, 30, 10, 12, 2),    # A^T T split over row ranges
])
def test_pca_vs_oracle_device(PCA, m, n, rank, k, l, its):
    print("case: pca device m=%d n=%d k=%d l=%d its=%d" % (m, n, k, l, its), flush=True)
    A, _, _, _ = inputs.pca_matrix(m, n, rank, seed=21, noise=1e-6, s_min=1e-2)
    om = inputs.pca_omega(n, l, seed=22)
    ref = opca.oocpca(A, om, k=k, its=its, b=512)
    U, s, V = PCA.oocpca(torch.from_numpy(A).to(DEV), om, k=k, its=its)
    torch.cuda.synchronize()
    _check(U.cpu().numpy(), s.cpu().numpy(), V.cpu().numpy(), ref)


@pytest.mark.parametrize("b", [700, 3001, 64])
def test_pca_host_streamed_matches(PCA, b):
    # A in host memory, copied b rows at a time: the same factors as the oracle
    print("case: pca host b=%d" % b, flush=True)
    m, n, k, l, its = 3001, 517, 10, 12, 2
    A, _, _, _ = inputs.pca_matrix(m, n, 30, seed=23, noise=1e-6)
    om = inputs.pca_omega(n, l, seed=24)
    ref = opca.oocpca(A, om, k=k, its=its, b=b)
    U, s, V = PCA.oocpca(A, om, k=k, its=its, b=b)
    torch.cuda.synchronize()
    _check(U.cpu().numpy(), s.cpu().numpy(), V.cpu().numpy(), ref)
    # the same call on the device copy gives the same numbers up to rounding
    Ud, sd, Vd = PCA.oocpca(torch.from_numpy(A).to(DEV), om, k=k, its=its, b=b)
    torch.cuda.synchronize()
    np.testing.assert_allclose(s.cpu().numpy(), sd.cpu().numpy(), rtol=1e-13)


def test_pca_row_stride(PCA):
    # A as a column slice of a wider matrix (lda > n)
    print("case: pca lda", flush=True)
    A, _, _, _ = inputs.pca_matrix(1500, 400, 20, seed=25, noise=1e-6)
    wide = torch.zeros((1500, 450), dtype=torch.float64, device=DEV)
    wide[:, 17:417] = torch.from_numpy(A).to(DEV)
    om = inputs.pca_omega(400, 10, seed=26)
    ref = opca.oocpca(A, om, k=8, its=2, b=1500)
    U, s, V = PCA.oocpca(wide[:, 17:417], om, k=8, its=2)
    torch.cuda.synchronize()
    _check(U.cpu().numpy(), s.cpu().numpy(), V.cpu().numpy(), ref)


def test_pca_planted_rank_below_l(PCA):
    # rank 6 < l = 8: two directions of A Omega are numerically zero and are
    # dropped; the planted values and vectors still come back
    print("case: pca planted rank 6, l 8", flush=True)
    A, U0, s0, V0 = inputs.pca_matrix(2500, 900, 6, seed=27, s_min=0.05)
    om = inputs.pca_omega(900, 8, seed=28)
    U, s, V = PCA.oocpca(torch.from_numpy(A).to(DEV), om, k=6, its=2)
    torch.cuda.synchronize()
    U, s, V = U.cpu().numpy(), s.cpu().numpy(), V.cpu().numpy()
    np.testing.assert_allclose(s, s0, rtol=1e-11)
    assert _cos(U, U0).min() > 1 - 1e-10 and _cos(V, V0).min() > 1 - 1e-10


def test_pca_zero_matrix(PCA):
    print("case: pca zero matrix", flush=True)
    A = torch.zeros((500, 300), dtype=torch.float64, device=DEV)
    U, s, V = PCA.oocpca(A, inputs.pca_omega(300, 6, seed=29), k=4, its=1)
    torch.cuda.synchronize()
    assert torch.all(s == 0) and torch.all(U == 0) and torch.all(V == 0)


def test_pca_paper_shape_sample(PCA):
    # 200,000 x 30,000 rank-50 (a fifth of the paper's 1,000,000 rows,
    # 48 GB of doubles), k = 50, l = 52, its = 2: the planted singular values,
    # orthonormal factors, and sampled rows of A reproduced by U diag(s) V^T
    print("case: pca 200000 x 30000 rank 50", flush=True)
    m, n, r = 200_000, 30_000, 50
    U0, s0, V0 = inputs.low_rank_factors(m, n, r, seed=30)
    U0t = torch.from_numpy(U0).to(DEV)
    V0t = torch.from_numpy(V0).to(DEV)
    A = (U0t * torch.from_numpy(s0).to(DEV)) @ V0t.T.contiguous()
    om = inputs.pca_omega(n, 52, seed=31)
    U, s, V = PCA.oocpca(A, om, k=50, its=2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(s.cpu().numpy(), s0, rtol=1e-10)
    eye = torch.eye(50, dtype=torch.float64, device=DEV)
    assert float((U.T @ U - eye).abs().max()) < 1e-11
    assert float((V.T @ V - eye).abs().max()) < 1e-11
    rows = np.random.default_rng(32).choice(m, 64, replace=False)
    Ar = A[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    Ur = U[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    approx = (Ur * s.cpu().numpy()) @ V.cpu().numpy().T
    assert np.abs(approx - Ar).max() < 1e-12
    del A, U0t, V0t
    torch.cuda.empty_cache()
