"""Kullback-Leibler divergence on the device (tsne_kl_divergence) against the
oracle's definition: with the oracle's own interpolated Z (same geometry),
with the exact Z, and at full size through the Z-free part of the sum."""
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


def _plan(T, Y, P, dtype, w=0.75, cap=128, layout=0):
    n, s = Y.shape
    plan = T.Plan(n, s, dtype, p=5, interval_width=w, max_intervals=cap, nnz=P.nnz, device=DEV,
                  attr_layout=layout)
    plan.bind_P(torch.from_numpy(P.row_ptr).to(DEV), torch.from_numpy(P.col).to(DEV),
                torch.from_numpy(P.val).to(DEV, dtype))
    return plan


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 5e-5)])
@pytest.mark.parametrize("n,s", [(3001, 2), (4001, 1)])
@pytest.mark.parametrize("layout", [1, 2])
def test_kl_vs_oracle(T, dtype, tol, n, s, layout):
    """The divergence through the CSR kernel's divergence mode (layout 1) and
    through the row-block sweep's (layout 2)."""
    print("case: kl n=%d s=%d %s layout %d" % (n, s, dtype, layout), flush=True)
    Y = inputs.mixture_embedding(n, s, 8, -20, 20, 1.5, seed=41)
    P = inputs.random_graph_P(n, 90, seed=42)
    plan = _plan(T, Y, P, dtype, layout=layout)
    Yt = torch.from_numpy(Y).to(DEV, dtype)
    kl = float(plan.kl_divergence(Yt).item())
    st = plan.query()
    assert st["status"] == 0
    Yd = Y.astype(np.float64)
    Pd = inputs.CSR(P.row_ptr, P.col, P.val.astype(np.float64))
    o, w, m = oracle.geometry(Yd, "fixed", 1, 0.75)
    Zi = oracle.interp_rep(Yd, o, w, m, 5)["Z"]
    ref = oracle.kl(Yd, Pd, Z=Zi)
    exact = oracle.kl(Yd, Pd)
    print("  GPU %.12f  oracle (interpolated Z) %.12f  exact %.12f" % (kl, ref, exact))
    assert abs(kl - ref) < tol * max(1.0, abs(ref))
    # against the exact divergence: only the interpolation error of Z remains
    assert abs(kl - exact) < 1e-4
    # the call leaves the plan usable and agrees with itself
    assert float(plan.kl_divergence(Yt).item()) == pytest.approx(kl, abs=tol)


def test_kl_needs_P(T):
    Y = torch.zeros(10, 2, dtype=torch.float32, device=DEV)
    plan = T.Plan(10, 2, torch.float32, nnz=20, max_intervals=16, device=DEV)
    with pytest.raises(T.TsneError) as e:
        plan.kl_divergence(Y)
    assert e.value.code == 7


@pytest.mark.parametrize("layout", [1, 2])
def test_kl_full_size(T, layout):
    """N = 1e6, 2-D, FP32: the divergence minus (sum p) log Z equals the
    oracle's sum of p log(p / K1) (its definition with Z = 1), O(nnz); CSR
    rows and the row-block sweep."""
    print("case: kl full size layout %d" % layout, flush=True)
    n = 1_000_000
    Y = inputs.mixture_embedding(n, 2, 50, -95.0, 95.0, 2.0, seed=0)
    P = inputs.random_graph_P(n, 90, seed=1)
    plan = _plan(T, Y, P, torch.float32, w=0.9, cap=512, layout=layout)
    Yt = torch.from_numpy(Y).to(DEV)
    kl = float(plan.kl_divergence(Yt).item())
    Z = plan.query()["Z"]
    Pd = inputs.CSR(P.row_ptr, P.col, P.val.astype(np.float64))
    part = oracle.kl(Y.astype(np.float64), Pd, Z=1.0)
    psum = float(P.val.astype(np.float64).sum())
    got = kl - psum * np.log(Z)
    print("  KL %.8f; sum p log(p/K1): GPU %.8f oracle %.8f" % (kl, got, part))
    assert abs(got - part) < 1e-4 * max(1.0, abs(part))
