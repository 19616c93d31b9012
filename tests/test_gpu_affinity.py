"""Input affinities on the device (tsne_knn, tsne_perplexity,
tsne_symmetrize) against the oracle.

kNN: the GPU accumulates squared distances in FP32, so distances are
compared rank by rank to a relative 1e-5, and a neighbour set may differ from
the oracle's only by points whose exact distance ties the k-th one to that
tolerance (either choice is a correct k-nearest set).  Perplexity and
symmetrisation take inputs produced on the oracle side (FP32 values seen by
both), so rows and CSR structure must match exactly and values to the FP32
output rounding.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1712_09005_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_09005_amd import tsne
    tsne.lib()
    return tsne


def check_knn(X, idx_g, d2_g, idx_o, d2_o, tol=1e-5):
    """Distances rank by rank; sets equal up to ties with the k-th distance."""
    np.testing.assert_allclose(d2_g, d2_o, rtol=tol, atol=tol * d2_o[:, -1:].max())
    assert np.all(np.diff(d2_g, axis=1) >= 0)
    n, k = idx_o.shape
    Xd = X.astype(np.float64)
    mism = 0
    for i in range(n):
        a, b = set(idx_g[i].tolist()), set(idx_o[i].tolist())
        if a == b:
            continue
        mism += 1
        kth = d2_o[i, -1]
        for j in a ^ b:
            dj = float(((Xd[i] - Xd[j]) ** 2).sum())
            assert abs(dj - kth) <= tol * kth, (i, j, dj, kth)
        assert len(a) == k and i not in a
    return mism


@pytest.mark.parametrize("n,dim,k", [(3001, 50, 90), (1500, 7, 30), (517, 3, 5), (40, 70, 39)])
def test_knn_vs_oracle(T, n, dim, k):
    print("case: knn n=%d dim=%d k=%d" % (n, dim, k), flush=True)
    X = inputs.mixture_highdim(n, dim, 10, 5.0, seed=n + dim)
    idx, d2 = T.knn(torch.from_numpy(X).to(DEV), k)
    torch.cuda.synchronize()
    io, do = oracle.knn(X.astype(np.float64), k)
    m = check_knn(X, idx.cpu().numpy(), d2.cpu().numpy().astype(np.float64), io, do)
    print("  rows whose sets differ at a tie: %d of %d" % (m, n))


def test_knn_duplicates_tie_by_index(T):
    """Exact duplicates are at distance 0 and ordered by index, as in the oracle."""
    base = inputs.mixture_highdim(300, 8, 4, 3.0, seed=5)
    X = np.ascontiguousarray(np.concatenate([base, base[:100], base[:50]]))
    idx, d2 = T.knn(torch.from_numpy(X).to(DEV), 6)
    io, do = oracle.knn(X.astype(np.float64), 6)
    dup = np.arange(100)                           # points 0..49 have two copies, 50..99 one
    np.testing.assert_array_equal(idx.cpu().numpy()[dup, :2], io[dup, :2])
    d2h = d2.cpu().numpy()
    assert np.all(d2h[:50, :2] == 0.0) and np.all(d2h[50:100, 0] == 0.0)
    np.testing.assert_array_equal(idx.cpu().numpy()[:50, :2], np.stack([300 + dup[:50], 400 + dup[:50]], 1))
    check_knn(X, idx.cpu().numpy(), d2.cpu().numpy().astype(np.float64), io, do)


@pytest.mark.parametrize("k,perp", [(90, 30.0), (30, 10.0), (128, 50.0), (7, 6.9)])
def test_perplexity_vs_oracle(T, k, perp):
    print("case: perplexity k=%d perp=%g" % (k, perp), flush=True)
    X = inputs.mixture_highdim(2000, 20, 6, 4.0, seed=k)
    _, do = oracle.knn(X.astype(np.float64), k)
    d32 = do.astype(np.float32)                  # the FP32 distances both sides see
    p, beta = T.perplexity(torch.from_numpy(d32).to(DEV), perp, want_beta=True)
    po, bo = oracle.perplexity(d32.astype(np.float64), perp)
    np.testing.assert_allclose(beta.cpu().numpy(), bo, rtol=1e-8)
    np.testing.assert_allclose(p.cpu().numpy(), po, rtol=2e-6, atol=1e-12)


def _oracle_rows(n, k, seed, hub=False):
    rng = np.random.default_rng(seed)
    idx = np.empty((n, k), np.int32)
    for i in range(n):
        c = rng.choice(np.delete(np.arange(n), i), k, replace=False)
        if hub and i != 0 and 0 not in c:
            c[0] = 0                              # point 0 in every list: one long row
        idx[i] = c
    p = rng.uniform(0.05, 1.0, size=(n, k))
    p = (p / p.sum(1, keepdims=True)).astype(np.float32)
    return idx, p


@pytest.mark.parametrize("n,k,hub", [(5003, 90, False), (3000, 5, True), (16000, 3, True), (7, 3, False)])
def test_symmetrize_vs_oracle(T, n, k, hub):
    """Structure exact, values to FP32 rounding; with hub=True one row holds
    n - 1 entries (the block-sorted path for rows over 1024)."""
    print("case: symmetrize n=%d k=%d hub=%s" % (n, k, hub), flush=True)
    idx, p = _oracle_rows(n, k, seed=n + k, hub=hub)
    rp, col, val = T.symmetrize(torch.from_numpy(idx).to(DEV), torch.from_numpy(p).to(DEV))
    rpo, colo, valo = oracle.symmetrize(idx, p.astype(np.float64))
    np.testing.assert_array_equal(rp.cpu().numpy(), rpo)
    np.testing.assert_array_equal(col.cpu().numpy(), colo)
    np.testing.assert_allclose(val.cpu().numpy(), valo, rtol=2e-6)


def test_symmetrize_rejects_oversized_row(T):
    """A row over 16384 entries is reported (status), not written past."""
    n, k = 17000, 1
    idx = np.zeros((n, k), np.int32)
    idx[0, 0] = 1                                  # every other row lists point 0
    p = np.ones((n, k), np.float32)
    with pytest.raises(T.TsneError):
        T.symmetrize(torch.from_numpy(idx).to(DEV), torch.from_numpy(p).to(DEV))


def test_affinities_end_to_end(T):
    """kNN -> perplexity -> symmetrise on the device against the oracle's
    pipeline in FP64: same structure where the neighbour sets agree, values
    to 1e-4 (FP32 distances move beta slightly), total 1, symmetric."""
    print("case: affinities end to end", flush=True)
    n, k, perp = 2500, 30, 10.0
    X = inputs.mixture_highdim(n, 12, 5, 4.0, seed=77)
    rp, col, val = T.affinities(torch.from_numpy(X).to(DEV), k, perp)
    rp, col, val = rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy().astype(np.float64)
    io, do = oracle.knn(X.astype(np.float64), k)
    po, _ = oracle.perplexity(do, perp)
    rpo, colo, valo = oracle.symmetrize(io, po)
    assert val.sum() == pytest.approx(1.0, rel=1e-5)
    G = {(i, c): v for i in range(n) for c, v in zip(col[rp[i]:rp[i + 1]], val[rp[i]:rp[i + 1]])}
    O = {(i, c): v for i in range(n) for c, v in zip(colo[rpo[i]:rpo[i + 1]], valo[rpo[i]:rpo[i + 1]])}
    for (i, c), v in G.items():
        assert G[(c, i)] == pytest.approx(v, rel=1e-6)
    common = set(G) & set(O)
    assert len(common) >= 0.999 * len(O)
    a = np.array([G[e] for e in common])
    b = np.array([O[e] for e in common])
    assert np.max(np.abs(a - b) / b) < 1e-4


def test_affinities_full_size_sampled(T):
    """N = 1e5, 50-d, k = 90, perplexity 30 (the full-run workload): sampled
    rows' neighbours against the oracle's exact ones, and the CSR totals."""
    print("case: affinities full size", flush=True)
    n, k = 100_000, 90
    X = inputs.mixture_highdim(n, 50, 20, 5.0, seed=0)
    Xt = torch.from_numpy(X).to(DEV)
    idx, d2 = T.knn(Xt, k)
    rows = np.sort(np.random.default_rng(9).choice(n, 64, replace=False))
    io, do = oracle.knn_rows(X.astype(np.float64), rows, k)
    check_knn(X, idx.cpu().numpy()[rows], d2.cpu().numpy()[rows].astype(np.float64), io, do)
    p = T.perplexity(d2, 30.0)
    rp, col, val = T.symmetrize(idx, p)
    assert float(val.double().sum()) == pytest.approx(1.0, rel=1e-5)
    assert int(rp[-1]) == col.shape[0] and k * n <= col.shape[0] <= 2 * k * n
