"""Serving loop for t-SNE embedding jobs on one GPU: continuous batching.

Jobs arrive over time (an arrival trace), wait in a FIFO queue and are
admitted into slots of a ``tsne.Batch`` while a slot is free and the HBM
footprint of the admitted jobs stays within a budget.  Every tick runs a few
iterations of all live slots with one launch per kernel (a replayed HIP
graph); finished jobs are retired and their slot and memory are reused at the
next tick boundary, so later arrivals overlap with jobs already running.
A job whose box outgrows its grid capacity is re-admitted with twice the
capacity (up to the library's largest), resuming at the iteration it reached
with its uY and gains.

A job never takes the server down: one whose footprint exceeds the whole
budget is rejected on arrival, and one that cannot be admitted, outgrows the
largest capacity or latches a device status ends with that status recorded
in ``Job.status``; every other job goes on.

``sequential`` runs the same trace one job at a time with ``Plan.run`` (the
unbatched path), the baseline the batched server is compared with.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque

import numpy as np

OK, REJECTED, FAILED = "ok", "rejected", "failed"


@dataclasses.dataclass
class Job:
    jid: int
    arrival: float                 # seconds after the start of the trace
    Y: np.ndarray                  # initial embedding [n, 2]
    P: object                      # inputs.CSR
    n_iter: int = 1000
    sched: object = None           # tsne.Schedule (default schedule when None)
    # filled in by the server
    admitted: float = math.nan
    finished: float = math.nan
    Y_out: np.ndarray = None
    replans: int = 0
    status: str = ""               # OK, REJECTED or FAILED
    reason: str = ""

    @property
    def n(self) -> int:
        return int(self.Y.shape[0])

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def capacity_for(n: int, interval_width: float = 0.75) -> int:
    """Intervals per dimension to plan for: the final t-SNE box grows roughly
    like sqrt(N); 1.5x margin over 40 + sqrt(N)/2 units."""
    return int(math.ceil(1.5 * (40.0 + 0.5 * math.sqrt(n)) / interval_width))


def max_capacity(p: int) -> int:
    """Largest interval count a plan accepts: the circulant of 2 N_int p nodes
    must stay within the library's 12288-point transforms."""
    return 12288 // (2 * p)


def percentile(values, q: float) -> float:
    """Nearest-rank percentile: the smallest value with at least q% of the
    values at or below it."""
    v = np.sort(np.asarray(values, dtype=np.float64))
    k = len(v)
    return float(v[min(k - 1, max(0, int(math.ceil(q / 100.0 * k)) - 1))])


def summarize(jobs, makespan: float) -> dict:
    """Runs/s and latency percentiles over the jobs that finished; jobs that
    were rejected or failed are counted beside them."""
    ok = [j for j in jobs if j.status == OK]
    lat = [j.latency for j in ok]
    out = {"jobs": len(ok), "rejected": sum(j.status == REJECTED for j in jobs),
           "failed": sum(j.status == FAILED for j in jobs), "makespan_s": makespan,
           "runs_per_s": len(ok) / makespan if makespan > 0 else 0.0}
    if ok:
        out.update(p50_latency_s=percentile(lat, 50), p99_latency_s=percentile(lat, 99),
                   mean_latency_s=float(np.mean(lat)))
    return out


class Server:
    """Continuous batching over ``batch`` (a ``tsne.Batch``, built here unless
    given).  ``footprint(job, cap)`` is the device bytes a job holds at
    capacity ``cap`` (``tsne.Batch.footprint`` unless given)."""

    def __init__(self, max_slots: int = 8, hbm_budget: int = 200 << 30, ticks_per_poll: int = 10,
                 interval_width: float = 0.75, p: int = 5, lanes_per_row: int = 32, device="cuda",
                 form="A", batch=None, footprint=None, clock=time.perf_counter):
        if batch is None:
            import torch
            from . import tsne
            batch = tsne.Batch(max_slots, s=2, dtype=torch.float32, p=p, form=form,
                               lanes_per_row=lanes_per_row, device=torch.device(device))
        if footprint is None:
            from . import tsne

            def footprint(job, cap):
                return tsne.Batch.footprint(job.n, job.P.nnz, s=2, p=p, max_intervals=cap,
                                            interval_width=interval_width, form=form)
        self.batch = batch
        self._footprint = footprint
        self.form = form
        self.max_slots = max_slots
        self.budget = hbm_budget
        self.k = ticks_per_poll
        self.w = interval_width
        self.p = p
        self.clock = clock

    def footprint(self, job: Job, cap: int) -> int:
        return int(self._footprint(job, cap))

    def run(self, jobs, log=None) -> dict:
        clock = self.clock
        pending = deque(sorted(jobs, key=lambda j: j.arrival))
        queue = deque()                            # (job, cap, it0, state)
        live = {}                                  # slot -> (job, cap, footprint)
        used = 0
        t0 = clock()
        ended = []
        cap_max = max_capacity(self.p)

        def end(job, status, reason=""):
            job.status, job.reason = status, reason
            job.finished = clock() - t0
            ended.append(job)
            if log:
                log("job %d n=%d %s at %.2fs %s" % (job.jid, job.n, status, job.finished, reason))

        while pending or queue or live:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                job = pending.popleft()
                cap = min(capacity_for(job.n, self.w), cap_max)
                fp = self.footprint(job, cap)
                if fp > self.budget:               # can never fit: reject on arrival
                    end(job, REJECTED, "footprint %d B over the %d B budget" % (fp, self.budget))
                    continue
                queue.append((job, cap, 0, None))
            # FIFO admission by slots and HBM footprint: the head of the queue
            # waits until enough memory is retired
            while queue and len(live) < self.max_slots:
                job, cap, it0, state = queue[0]
                fp = self.footprint(job, cap)
                if fp > self.budget:               # a re-planned grid that can never fit
                    queue.popleft()
                    end(job, FAILED, "footprint %d B at %d intervals over the budget" % (fp, cap))
                    continue
                if used + fp > self.budget:
                    break
                queue.popleft()
                res = state if state is not None else {"Y": job.Y, "uY": None, "gains": None}
                try:
                    slot = self.batch.admit(res["Y"], (job.P.row_ptr, job.P.col, job.P.val),
                                            job.sched, it0, job.n_iter - it0, max_intervals=cap,
                                            interval_width=self.w, uY=res["uY"],
                                            gains=res["gains"])
                except Exception as e:             # this job only
                    end(job, FAILED, "admission: %s" % e)
                    continue
                if math.isnan(job.admitted):
                    job.admitted = clock() - t0
                live[slot] = (job, cap, fp)
                used += fp
            if not live:
                if pending and not queue:          # idle until the next arrival
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - (clock() - t0))))
                continue
            self.batch.tick(self.k)
            for slot in list(live):
                job, cap, fp = live[slot]
                it, st = self.batch.poll(slot)
                if st == 0 and it < job.n_iter:
                    continue
                state = self.batch.retire(slot)
                del live[slot]
                used -= fp
                if st == 4:                        # capacity: re-plan with a larger grid
                    if cap >= cap_max:
                        end(job, FAILED, "box needs more than %d intervals" % cap_max)
                        continue
                    job.replans += 1
                    queue.appendleft((job, min(cap * 2, cap_max), it, state))
                    continue
                if st != 0:
                    end(job, FAILED, "device status %d at iteration %d" % (st, it))
                    continue
                job.Y_out = state["Y"].cpu().numpy()
                end(job, OK)
        return summarize(ended, clock() - t0)


def sequential(jobs, interval_width: float = 0.75, p: int = 5, lanes_per_row: int = 32,
               device="cuda", log=None, form="A") -> dict:
    """The same trace served one job at a time with the unbatched path."""
    import torch
    from . import tsne
    dev = torch.device(device)
    t0 = time.perf_counter()
    out = []
    cap_max = max_capacity(p)
    for job in sorted(jobs, key=lambda j: j.arrival):
        now = time.perf_counter() - t0
        if job.arrival > now:
            time.sleep(job.arrival - now)
        job.admitted = time.perf_counter() - t0
        cap = min(capacity_for(job.n, interval_width), cap_max)
        it = 0
        Y = torch.from_numpy(np.ascontiguousarray(job.Y, dtype=np.float32)).to(dev)
        uY = torch.zeros_like(Y)
        gains = torch.ones_like(Y)
        rp = torch.from_numpy(job.P.row_ptr).to(dev)
        col = torch.from_numpy(job.P.col).to(dev)
        val = torch.from_numpy(job.P.val).to(dev)
        sched = job.sched if job.sched is not None else tsne.Schedule()
        job.status = OK
        while True:
            plan = tsne.Plan(job.n, 2, torch.float32, p=p, policy="fixed", form=form,
                             interval_width=interval_width, max_intervals=cap, nnz=job.P.nnz,
                             lanes_per_row=lanes_per_row, attr_slabs=1, attr_layout=1,
                             device=dev)
            plan.bind_P(rp, col, val)
            plan.run(Y, uY, gains, sched, it, job.n_iter - it)
            st = plan.query()
            if st["status"] == 0:
                break
            if st["status"] != 4 or cap >= cap_max:
                job.status, job.reason = FAILED, "device status %d" % st["status"]
                break
            it = st["iter"]
            cap = min(cap * 2, cap_max)
            job.replans += 1
        job.finished = time.perf_counter() - t0
        job.Y_out = Y.cpu().numpy()
        out.append(job)
        if log:
            log("job %d n=%d done at %.2fs" % (job.jid, job.n, job.finished))
    return summarize(out, time.perf_counter() - t0)
