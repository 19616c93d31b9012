"""Reproducibility of the FP32 path: the binning is a stable sort into the
canonical order (cell, then point index), and every later sum runs in a fixed
order, so identical inputs give bit-identical results, a run split into two
calls equals the run in one call, and the binning itself equals a plain
stable sort by cell computed on the host."""
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


def _job(n, seed, spread=1e-2):
    rng = np.random.default_rng(seed)
    Y = (spread * rng.standard_normal((n, 2))).astype(np.float32)
    P = inputs.random_graph_P(n, 30, seed=seed + 1)
    return Y, P


def _plan(T, n, P, form, cap=256):
    plan = T.Plan(n, 2, torch.float32, p=5, policy="fixed", interval_width=0.75,
                  max_intervals=cap, form=form, nnz=P.nnz, device=DEV)
    plan.bind_P(torch.from_numpy(P.row_ptr).to(DEV), torch.from_numpy(P.col).to(DEV),
                torch.from_numpy(P.val).to(DEV))
    return plan


def _state(Y):
    Yt = torch.from_numpy(Y).to(DEV)
    return Yt, torch.zeros_like(Yt), torch.ones_like(Yt)


def _bits(*ts):
    return [t.cpu().numpy().view(np.uint32).copy() for t in ts]


@pytest.mark.parametrize("form", ["A", "V"])
def test_run_twice_and_split_run_bitwise(T, form):
    print("case: determinism n=20011 form %s" % form, flush=True)
    n = 20011
    Y, P = _job(n, 3)
    sched = T.Schedule(ee_stop=20, mom_switch=20)
    out = []
    for _ in range(2):                           # two fresh plans, one call each
        plan = _plan(T, n, P, form)
        s = _state(Y)
        plan.run(*s, sched, 0, 40)
        torch.cuda.synchronize()
        assert plan.query()["status"] == 0
        out.append(_bits(*s))
    plan = _plan(T, n, P, form)                  # one plan, the run split in two calls
    s = _state(Y)
    plan.run(*s, sched, 0, 25)
    plan.run(*s, sched, 25, 15)
    torch.cuda.synchronize()
    assert plan.query()["status"] == 0
    out.append(_bits(*s))
    plan = _plan(T, n, P, form)                  # and in single steps
    s = _state(Y)
    for it in range(40):
        plan.step(*s, sched, it)
    torch.cuda.synchronize()
    out.append(_bits(*s))
    for k in range(1, len(out)):
        for a, b, name in zip(out[0], out[k], ("Y", "uY", "gains")):
            assert np.array_equal(a, b), (k, name, int((a != b).sum()))


# (points, intervals capacity, interval width): one radix pass of at most 9
# bits does not cover the capacity's cells, so these take two passes (few and
# many tiles) and three passes (a capacity above 2^18 cells)
BINNING = [(50_000, 128, 0.75), (300_001, 512, 0.1), (100_000, 600, 0.08)]


@pytest.mark.parametrize("n,cap,width", BINNING)
def test_binning_is_the_stable_sort_by_cell(T, n, cap, width):
    """The sorted permutation equals numpy's stable argsort of the cells the
    oracle assigns (same box, same interval rule), and the cell offsets are its
    run boundaries: exact, for a square and a rectangular box."""
    for rect in (False, True):
        print("case: binning permutation n=%d cap=%d rect=%s" % (n, cap, rect), flush=True)
        Y = inputs.mixture_embedding(n, 2, 10, -20.0, 20.0, 1.5, seed=4)
        if rect:
            Y[:, 1] *= 0.3
        plan = T.Plan(n, 2, torch.float32, p=5, policy="fixed", interval_width=width,
                      max_intervals=cap, form="V", rect=rect, device=DEV)
        plan.repulsive(torch.from_numpy(Y).to(DEV))
        torch.cuda.synchronize()
        st = plan.query()
        assert st["status"] == 0
        perm = np.frombuffer(plan.export(4), np.int32)
        cs = np.frombuffer(plan.export(3), np.int32)
        o, w, m = oracle.geometry(Y.astype(np.float64), "fixed", 1, width, rect=rect)
        mx, my = (m, m) if not rect else m
        assert (mx, my) == (st["n_int"], st["n_int_y"])
        cx = np.clip(np.floor((Y[:, 0].astype(np.float64) - o[0]) / w), 0, mx - 1).astype(np.int64)
        cy = np.clip(np.floor((Y[:, 1].astype(np.float64) - o[1]) / w), 0, my - 1).astype(np.int64)
        cell = cy * mx + cx
        ref = np.argsort(cell, kind="stable")
        assert np.array_equal(perm, ref)
        starts = np.searchsorted(cell[ref], np.arange(mx * my + 1), side="left")
        assert np.array_equal(cs, starts)
