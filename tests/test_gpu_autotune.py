"""The autotuner: its error estimate against the direct sum computed by the
oracle, the width it picks against the accuracy target, and that every knob
it can return gives the same forces (launch knobs change summation order
only)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1712_09005_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def A():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_09005_amd import autotune, tsne
    tsne.lib()
    return autotune


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("s", [1, 2])
def test_error_estimate_tracks_direct_sum(A, s):
    """The half-width estimate is within a factor of two of the true error of
    the FP64 path against the direct sum, at several widths."""
    print("case: error estimate s=%d" % s, flush=True)
    n = 4000
    Y = inputs.mixture_embedding(n, s, 8, -25, 25, 2.0, seed=21).astype(np.float64)
    Fd, _ = oracle.direct_rep(Y)
    from paper_1712_09005_amd import tsne
    for w in (1.5, 1.0, 0.75):
        est = A.estimate_error(Y, w, p=5, device=DEV)
        plan = tsne.Plan(n, s, torch.float64, p=5, interval_width=w, max_intervals=128, device=DEV)
        F, _ = plan.repulsive(torch.from_numpy(Y).to(DEV))
        true = rel(F.cpu().numpy(), Fd)
        print("  w=%.2f estimate %.2e true %.2e" % (w, est, true))
        assert 0.5 * true < est < 2.0 * true


def test_width_meets_target(A, tmp_path):
    print("case: tune_width", flush=True)
    n = 3000
    Y = inputs.mixture_embedding(n, 2, 8, -25, 25, 2.0, seed=22).astype(np.float64)
    cache = str(tmp_path / "tune.json")
    r = A.tune_width(Y, target=1e-3, safety=2.0, p=5, device=DEV, cache=cache)
    w = r["interval_width"]
    from paper_1712_09005_amd import tsne
    plan = tsne.Plan(n, 2, torch.float32, p=5, interval_width=w, max_intervals=128, device=DEV)
    F, _ = plan.repulsive(torch.from_numpy(Y.astype(np.float32)).to(DEV))
    Fd, _ = oracle.direct_rep(Y)
    e = rel(F.cpu().numpy(), Fd)
    print("  chose w=%.2f (estimate %.2e), FP32 error vs direct %.2e" % (w, r["estimate"], e))
    assert e < 1e-3
    # the next wider width on the ladder fails the target (the choice is the largest)
    wider = [x for x in A.WIDTHS if x > w]
    if wider:
        assert 2.0 * A.estimate_error(Y, min(wider), p=5, device=DEV) > 1e-3
    # cache round trip
    assert A.tune_width(Y, target=1e-3, safety=2.0, p=5, device=DEV, cache=cache) == r


def test_attraction_knobs_agree(A, tmp_path):
    """Every candidate layout times without error, the fastest is one of them,
    and it gives the oracle's F_attr."""
    print("case: tune_attraction", flush=True)
    n = 20011
    Y = inputs.mixture_embedding(n, 2, 10, -30, 30, 2.0, seed=0)
    P = inputs.random_graph_P(n, 90, seed=1)
    r = A.tune_attraction(Y, P, device=DEV, reps=3, cache=str(tmp_path / "t.json"))
    assert len(r["table"]) == len(A.CSR_KNOBS)
    assert (r["lanes_per_row"], r["attr_slabs"], r["attr_layout"]) in A.CSR_KNOBS
    from paper_1712_09005_amd import tsne
    plan = tsne.Plan(n, 2, torch.float32, nnz=P.nnz, lanes_per_row=r["lanes_per_row"],
                     attr_slabs=r["attr_slabs"], attr_layout=r["attr_layout"], max_intervals=16,
                     device=DEV)
    plan.bind_P(torch.from_numpy(P.row_ptr).to(DEV), torch.from_numpy(P.col).to(DEV),
                torch.from_numpy(P.val).to(DEV))
    Fa = plan.attractive(torch.from_numpy(Y).to(DEV)).cpu().numpy()
    ref = oracle.attr(Y.astype(np.float64), inputs.CSR(P.row_ptr, P.col, P.val.astype(np.float64)))
    assert rel(Fa, ref) < 1e-6


def test_spread_and_batch_lanes(A, tmp_path):
    print("case: tune_spread / tune_batch_lanes", flush=True)
    Y = inputs.mixture_embedding(30000, 2, 10, -30, 30, 2.0, seed=3)
    r = A.tune_spread(Y, device=DEV, reps=3, max_intervals=128, cache=str(tmp_path / "s.json"))
    assert r["points_per_lane"] in A.KPTS
    jobs = [(inputs.mixture_embedding(n, 2, 5, -10, 10, 1.0, seed=n),
             inputs.random_graph_P(n, 90, seed=n)) for n in (5000, 12000)]
    b = A.tune_batch_lanes(jobs, device=DEV, reps=3, cache=str(tmp_path / "b.json"))
    assert b["lanes_per_row"] in (4, 8, 16, 32, 64)


def test_interp_choice_meets_target(A, tmp_path):
    """Joint choice of nodes per interval and width: the chosen pair meets the
    accuracy target against the direct sum."""
    print("case: tune_interp", flush=True)
    n = 3000
    Y = inputs.mixture_embedding(n, 2, 8, -25, 25, 2.0, seed=23).astype(np.float64)
    r = A.tune_interp(Y, target=1e-3, safety=2.5, max_intervals=128, device=DEV, reps=3,
                      cache=str(tmp_path / "i.json"), forms=("A", "V"))
    assert r["p"] in A.PS and r["form"] in ("A", "V")
    # one row per (form, p), the paper's p = 3 among them, each timed or with its reason
    assert [(t["form"], t["p"]) for t in r["table"]] == [(f, p) for f in ("A", "V") for p in A.PS]
    assert all(t["seconds"] is not None or t["note"] for t in r["table"])
    from paper_1712_09005_amd import tsne
    plan = tsne.Plan(n, 2, torch.float32, p=r["p"], interval_width=r["interval_width"],
                     max_intervals=r["max_intervals"], form=r["form"], device=DEV)
    F, _ = plan.repulsive(torch.from_numpy(Y.astype(np.float32)).to(DEV))
    Fd, _ = oracle.direct_rep(Y)
    e = rel(F.cpu().numpy(), Fd)
    print("  chose form %s p=%d w=%.2f, FP32 error vs direct %.2e (table %s)"
          % (r["form"], r["p"], r["interval_width"], e, r["table"]))
    assert e < 1e-3
