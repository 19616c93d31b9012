"""Batching: independent embeddings of uneven N sharing every launch give the
same results as each embedding run alone, bit for bit (same kernels, same
per-instance work decomposition, and a binning into the canonical order by
cell and point index, so every sum runs in the same order)."""
import numpy as np
import pytest
import torch

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


def _job(n, seed):
    rng = np.random.default_rng(seed)
    Y = (1e-2 * rng.standard_normal((n, 2))).astype(np.float64)
    P = inputs.random_graph_P(n, 30, seed=seed + 1)
    return Y, P


def _alone(T, Y, P, dtype, sched, it0, n_it, form="A"):
    n = Y.shape[0]
    plan = T.Plan(n, 2, dtype, p=5, policy="fixed", interval_width=0.75, max_intervals=256, form=form,
                  nnz=P.nnz, lanes_per_row=32, attr_slabs=1, attr_layout=1, device=DEV)
    plan.bind_P(torch.from_numpy(P.row_ptr).to(DEV), torch.from_numpy(P.col).to(DEV),
                torch.from_numpy(P.val).to(DEV, dtype))
    Yt = torch.from_numpy(Y).to(DEV, dtype)
    uY = torch.zeros_like(Yt)
    g = torch.ones_like(Yt)
    plan.run(Yt, uY, g, sched, it0, n_it)
    torch.cuda.synchronize()
    assert plan.query()["status"] == 0
    return Yt.cpu().numpy()


# 30 iterations (through the end of early exaggeration at 10) in both
# precisions, compared bit for bit
@pytest.mark.parametrize("dtype,tol,iters", [(torch.float64, 0.0, 30), (torch.float32, 0.0, 30)])
@pytest.mark.parametrize("form", ["A", "V"])
def test_alone_equals_in_the_mix(T, dtype, tol, iters, form):
    print("case: batch alone vs mix %s form %s" % (dtype, form), flush=True)
    sched = T.Schedule(ee_stop=10, mom_switch=10)
    sizes = [(3000, 10, iters), (7001, 3, iters), (1500, 20, iters - 1)]   # (n, seed, iterations)
    jobs = [_job(n, sd) for n, sd, _ in sizes]
    alone = [_alone(T, Y, P, dtype, sched, 0, it, form) for (Y, P), (_, _, it) in zip(jobs, sizes)]
    b = T.Batch(4, s=2, dtype=dtype, p=5, form=form, device=DEV)
    slots = []
    for (Y, P), (_, _, it) in zip(jobs[:2], sizes[:2]):
        slots.append(b.admit(Y, (P.row_ptr, P.col, P.val), sched, 0, it, max_intervals=256))
    b.tick(1)                                   # third job arrives while the others run
    Y, P = jobs[2]
    slots.append(b.admit(Y, (P.row_ptr, P.col, P.val), sched, 0, sizes[2][2], max_intervals=256))
    b.tick(40)                                  # more ticks than any job needs
    for k, sl in enumerate(slots):
        done, st = b.poll(sl)
        assert st == 0 and done == sizes[k][2], (k, done, st)
        job = b.retire(sl)
        Yb = job["Y"].cpu().numpy()
        e = np.linalg.norm(Yb - alone[k]) / np.linalg.norm(alone[k])
        print("  job %d n=%d rel diff %.2e" % (k, sizes[k][0], e))
        assert e <= tol and (tol > 0 or np.array_equal(Yb, alone[k]))
    # slot reuse after retirement
    Y, P = jobs[0]
    sl = b.admit(Y, (P.row_ptr, P.col, P.val), sched, 0, 12, max_intervals=256)
    assert sl in slots
    b.tick(12)
    done, st = b.poll(sl)
    assert done == 12 and st == 0
    ref = _alone(T, Y, P, dtype, sched, 0, 12, form)
    Yb = b.retire(sl)["Y"].cpu().numpy()
    assert np.array_equal(Yb, ref)


def test_batch_rejects_mismatched_jobs(T):
    b = T.Batch(2, s=2, dtype=torch.float32, p=5, device=DEV)
    Y, P = _job(500, 3)
    with pytest.raises(ValueError):
        b.admit(Y[:, :1].copy(), (P.row_ptr, P.col, P.val), T.Schedule(), 0, 5)   # s = 1 job
    for _ in range(2):
        b.admit(Y, (P.row_ptr, P.col, P.val), T.Schedule(), 0, 5, max_intervals=64)
    with pytest.raises(T.TsneError) as e:
        b.admit(Y, (P.row_ptr, P.col, P.val), T.Schedule(), 0, 5, max_intervals=64)
    assert e.value.code == 4                    # no free slot
