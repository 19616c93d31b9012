"""The serving loop's host logic on the CPU, over a fake batch that stands in
for the device: FIFO admission by slots and HBM footprint, slot reuse, the
capacity re-plan that resumes a job at the iteration it reached with its uY
and gains, rejection and failure of single jobs without stopping the others,
and nearest-rank latency percentiles."""
import math

import numpy as np
import torch

from paper_1712_09005_amd import serve


class FakeBatch:
    """Device stand-in.  Each iteration adds 1 to every coordinate of Y and to
    uY, and multiplies gains by 2, so a resumed job ends with the right values
    only if the server hands back its state.  A job "needs" more intervals as
    it runs (``need(jid, it)``); at the first iteration that needs more than
    the slot's capacity the slot latches status 4 there (not committed)."""

    def __init__(self, max_slots, need=None, fail_admit=(), footprint=None, budget=None):
        self.max_slots = max_slots
        self.need = need or (lambda jid, it: 0)
        self.fail_admit = set(fail_admit)
        self.footprint = footprint
        self.budget = budget
        self.live = {}
        self.log = []                  # (jid, slot, it0, n_it, cap, resumed)
        self.peak_used = 0

    def admit(self, Y, P, sched, it0, n_it, max_intervals=512, interval_width=0.75, uY=None,
              gains=None):
        jid = int(P[0][0])             # the tests store the job id in row_ptr[0] of a fake P
        if jid in self.fail_admit:
            raise RuntimeError("admission refused")
        assert len(self.live) < self.max_slots
        slot = min(set(range(self.max_slots)) - set(self.live))
        Yt = torch.as_tensor(np.asarray(Y, dtype=np.float64)).clone()
        st = dict(jid=jid, n=Yt.shape[0], Y=Yt,
                  uY=torch.zeros_like(Yt) if uY is None else torch.as_tensor(uY).clone(),
                  gains=torch.ones_like(Yt) if gains is None else torch.as_tensor(gains).clone(),
                  it=it0, end=it0 + n_it, cap=max_intervals, status=0)
        self.live[slot] = st
        self.log.append((jid, slot, it0, n_it, max_intervals, uY is not None))
        if self.footprint is not None:
            used = sum(self.footprint(s["n"], s["cap"]) for s in self.live.values())
            self.peak_used = max(self.peak_used, used)
            assert used <= self.budget
        return slot

    def tick(self, k):
        for st in self.live.values():
            for _ in range(k):
                if st["status"] != 0 or st["it"] >= st["end"]:
                    break
                if self.need(st["jid"], st["it"]) > st["cap"]:
                    st["status"] = 4
                    break
                st["Y"] += 1.0
                st["uY"] += 1.0
                st["gains"] *= 2.0
                st["it"] += 1

    def poll(self, slot):
        st = self.live[slot]
        return st["it"], st["status"]

    def retire(self, slot):
        st = self.live.pop(slot)
        return dict(Y=st["Y"], uY=st["uY"], gains=st["gains"])


class _P:
    """A fake P whose row_ptr[0] carries the job id."""

    def __init__(self, jid, nnz=100):
        self.row_ptr = np.array([jid, 0], dtype=np.int64)
        self.col = np.zeros(nnz, np.int32)
        self.val = np.zeros(nnz, np.float32)
        self.nnz = nnz


def _jobs(ns, n_iter=30, arrivals=None):
    arrivals = arrivals if arrivals is not None else [0.0] * len(ns)
    return [serve.Job(j, a, np.full((n, 2), float(j)), _P(j), n_iter=n_iter)
            for j, (n, a) in enumerate(zip(ns, arrivals))]


def _fp(job, cap):
    return job.n * 10 + cap


def test_fifo_admission_and_slot_reuse():
    jobs = _jobs([100, 200, 300, 400, 500])
    fb = FakeBatch(2)
    srv = serve.Server(max_slots=2, hbm_budget=10 ** 9, ticks_per_poll=10, batch=fb, footprint=_fp)
    out = srv.run(jobs)
    assert [e[0] for e in fb.log] == [0, 1, 2, 3, 4]          # FIFO
    assert sorted({e[1] for e in fb.log}) == [0, 1]           # two slots, reused
    assert out["jobs"] == 5 and out["rejected"] == 0 and out["failed"] == 0
    for j in jobs:
        assert j.status == serve.OK and j.replans == 0
        np.testing.assert_array_equal(j.Y_out, np.full((j.n, 2), j.jid + 30.0))
        assert j.finished >= j.admitted >= j.arrival


def test_admission_by_footprint():
    """Four slots but a budget for two of these jobs at a time: the head of the
    queue waits for memory, and the admitted footprint never exceeds it."""
    jobs = _jobs([1000, 1000, 1000, 1000, 1000, 1000])
    cap = serve.capacity_for(1000, 0.75)
    budget = 2 * _fp(jobs[0], cap) + 5
    fb = FakeBatch(4, footprint=lambda n, c: n * 10 + c, budget=budget)
    srv = serve.Server(max_slots=4, hbm_budget=budget, batch=fb, footprint=_fp)
    out = srv.run(jobs)
    assert out["jobs"] == 6
    assert fb.peak_used == 2 * _fp(jobs[0], cap)
    assert [e[0] for e in fb.log] == list(range(6))


def test_capacity_replan_resumes_with_state():
    """Job 1 outgrows its grid at iteration 17: it is re-admitted with twice
    the capacity at iteration 17 with its uY and gains, and ends exactly as an
    uninterrupted run would; the other jobs are not disturbed."""
    jobs = _jobs([100, 4000, 100], n_iter=40)
    cap1 = serve.capacity_for(4000, 0.75)
    fb = FakeBatch(3, need=lambda jid, it: cap1 + 1 if (jid == 1 and it >= 17) else 0)
    srv = serve.Server(max_slots=3, hbm_budget=10 ** 9, ticks_per_poll=5, batch=fb, footprint=_fp)
    out = srv.run(jobs)
    assert out["jobs"] == 3
    again = [e for e in fb.log if e[0] == 1]
    assert len(again) == 2
    assert again[0][2:5] == (0, 40, cap1)
    assert again[1][2] == 17 and again[1][3] == 23 and again[1][4] == 2 * cap1 and again[1][5]
    j = jobs[1]
    assert j.replans == 1 and j.status == serve.OK
    np.testing.assert_array_equal(j.Y_out, np.full((4000, 2), 1.0 + 40.0))


def test_rejection_and_failures_stay_per_job():
    """A job larger than the whole budget is rejected on arrival; a job whose
    admission raises, and one that outgrows the largest capacity, fail; the
    rest of the trace is served."""
    jobs = _jobs([100, 10 ** 7, 200, 300, 400])
    cap_max = serve.max_capacity(5)
    fb = FakeBatch(2, fail_admit={2}, need=lambda jid, it: cap_max + 1 if (jid == 3 and it >= 3) else 0)
    srv = serve.Server(max_slots=2, hbm_budget=10 ** 6, batch=fb, footprint=_fp)
    out = srv.run(jobs)
    st = {j.jid: j.status for j in jobs}
    assert st == {0: serve.OK, 1: serve.REJECTED, 2: serve.FAILED, 3: serve.FAILED, 4: serve.OK}
    assert out["jobs"] == 2 and out["rejected"] == 1 and out["failed"] == 2
    assert "intervals" in jobs[3].reason and jobs[3].replans >= 1
    # job 3 was re-planned up to the largest capacity, never past it
    assert max(e[4] for e in fb.log if e[0] == 3) == cap_max


def test_later_arrival_waits_for_its_time():
    jobs = _jobs([100, 100], n_iter=10, arrivals=[0.0, 0.05])
    fb = FakeBatch(2)
    srv = serve.Server(max_slots=2, batch=fb, footprint=_fp)
    srv.run(jobs)
    assert jobs[1].admitted >= 0.05 and all(j.status == serve.OK for j in jobs)


def test_nearest_rank_percentiles():
    v = np.arange(1, 101, dtype=float)[::-1]
    assert serve.percentile(v, 50) == 50.0 and serve.percentile(v, 99) == 99.0
    assert serve.percentile(v, 100) == 100.0 and serve.percentile([7.0], 99) == 7.0
    w = np.arange(1, 65, dtype=float)                         # 64 jobs, as in the serving trace
    assert serve.percentile(w, 50) == 32.0 and serve.percentile(w, 99) == 64.0
    jobs = _jobs([10] * 4)
    for j, lat in zip(jobs, (4.0, 1.0, 3.0, 2.0)):
        j.status, j.finished = serve.OK, j.arrival + lat
    s = serve.summarize(jobs, 8.0)
    assert s["runs_per_s"] == 0.5 and s["p50_latency_s"] == 2.0 and s["p99_latency_s"] == 4.0
    assert math.isclose(s["mean_latency_s"], 2.5)


def test_capacity_ladder_bounds():
    assert serve.max_capacity(5) == 1228 and serve.max_capacity(2) == 3072
    assert serve.capacity_for(5000, 0.75) < serve.capacity_for(200000, 0.75) <= serve.max_capacity(5)
