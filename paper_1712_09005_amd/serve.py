"""Serving loop for t-SNE embedding jobs on one GPU: continuous batching.

Jobs arrive over time (an arrival trace), wait in a FIFO queue and are
admitted into slots of a ``tsne.Batch`` while a slot is free and the HBM
footprint of the admitted jobs stays within a budget.  Every tick runs a few
iterations of all live slots with one launch per kernel (a replayed HIP
graph); finished jobs are retired and their slot and memory are reused at the
next tick boundary, so later arrivals overlap with jobs already running.
A job whose box outgrows its grid capacity is re-admitted with twice the
capacity, resuming at the iteration it reached.

``sequential`` runs the same trace one job at a time with ``Plan.run`` (the
unbatched path), the baseline the batched server is compared with.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque

import numpy as np
import torch

from . import tsne


@dataclasses.dataclass
class Job:
    jid: int
    arrival: float                 # seconds after the start of the trace
    Y: np.ndarray                  # initial embedding [n, 2]
    P: object                      # inputs.CSR
    n_iter: int = 1000
    sched: tsne.Schedule = dataclasses.field(default_factory=tsne.Schedule)
    # filled in by the server
    admitted: float = math.nan
    finished: float = math.nan
    Y_out: np.ndarray = None
    replans: int = 0

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


def summarize(jobs, makespan: float) -> dict:
    lat = np.sort(np.array([j.latency for j in jobs]))
    k = len(lat)

    def pct(q):                                   # nearest rank
        return float(lat[min(k - 1, max(0, int(math.ceil(q / 100.0 * k)) - 1))])
    return {"jobs": k, "makespan_s": makespan, "runs_per_s": k / makespan,
            "p50_latency_s": pct(50), "p99_latency_s": pct(99),
            "mean_latency_s": float(lat.mean())}


class Server:
    def __init__(self, max_slots: int = 8, hbm_budget: int = 200 << 30, ticks_per_poll: int = 10,
                 interval_width: float = 0.75, p: int = 5, lanes_per_row: int = 32, device="cuda",
                 form="A"):
        self.device = torch.device(device)
        self.batch = tsne.Batch(max_slots, s=2, dtype=torch.float32, p=p, form=form,
                                lanes_per_row=lanes_per_row, device=self.device)
        self.form = form
        self.max_slots = max_slots
        self.budget = hbm_budget
        self.k = ticks_per_poll
        self.w = interval_width
        self.p = p

    def footprint(self, job: Job, cap: int) -> int:
        return tsne.Batch.footprint(job.n, job.P.nnz, s=2, p=self.p, max_intervals=cap,
                                    interval_width=self.w, form=self.form)

    def run(self, jobs, log=None) -> dict:
        pending = deque(sorted(jobs, key=lambda j: j.arrival))
        queue = deque()
        live = {}                                  # slot -> (job, cap, footprint, it0)
        used = 0
        t0 = time.perf_counter()
        done = []
        while pending or queue or live:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                queue.append((pending.popleft(), None, 0, None))
            # FIFO admission by slots and HBM footprint
            while queue and len(live) < self.max_slots:
                job, cap, it0, state = queue[0]
                cap = cap or capacity_for(job.n, self.w)
                fp = self.footprint(job, cap)
                if used + fp > self.budget and live:
                    break
                queue.popleft()
                res = state if state is not None else {"Y": job.Y, "uY": None, "gains": None}
                slot = self.batch.admit(res["Y"], (job.P.row_ptr, job.P.col, job.P.val), job.sched,
                                        it0, job.n_iter - it0, max_intervals=cap,
                                        interval_width=self.w, uY=res["uY"], gains=res["gains"])
                if math.isnan(job.admitted):
                    job.admitted = time.perf_counter() - t0
                live[slot] = (job, cap, fp, it0)
                used += fp
            if not live:
                if pending:                        # idle until the next arrival
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - now)))
                continue
            self.batch.tick(self.k)
            for slot in list(live):
                job, cap, fp, it0 = live[slot]
                it, st = self.batch.poll(slot)
                if st == 0 and it < job.n_iter:
                    continue
                state = self.batch.retire(slot)
                del live[slot]
                used -= fp
                if st == 4:                        # capacity: re-plan with a larger grid
                    job.replans += 1
                    queue.appendleft((job, cap * 2, it, state))
                    continue
                if st != 0:
                    raise RuntimeError("job %d failed with device status %d" % (job.jid, st))
                job.finished = time.perf_counter() - t0
                job.Y_out = state["Y"].cpu().numpy()
                done.append(job)
                if log:
                    log("job %d n=%d done at %.2fs (latency %.2fs)" % (job.jid, job.n, job.finished,
                                                                      job.latency))
        return summarize(done, time.perf_counter() - t0)


def sequential(jobs, interval_width: float = 0.75, p: int = 5, lanes_per_row: int = 32,
               device="cuda", log=None, form="A") -> dict:
    """The same trace served one job at a time with the unbatched path."""
    dev = torch.device(device)
    t0 = time.perf_counter()
    out = []
    for job in sorted(jobs, key=lambda j: j.arrival):
        now = time.perf_counter() - t0
        if job.arrival > now:
            time.sleep(job.arrival - now)
        job.admitted = time.perf_counter() - t0
        cap = capacity_for(job.n, interval_width)
        it = 0
        Y = torch.from_numpy(np.ascontiguousarray(job.Y, dtype=np.float32)).to(dev)
        uY = torch.zeros_like(Y)
        gains = torch.ones_like(Y)
        rp = torch.from_numpy(job.P.row_ptr).to(dev)
        col = torch.from_numpy(job.P.col).to(dev)
        val = torch.from_numpy(job.P.val).to(dev)
        while True:
            plan = tsne.Plan(job.n, 2, torch.float32, p=p, policy="fixed", form=form,
                             interval_width=interval_width, max_intervals=cap, nnz=job.P.nnz,
                             lanes_per_row=lanes_per_row, attr_slabs=1, attr_layout=1,
                             device=dev)
            plan.bind_P(rp, col, val)
            plan.run(Y, uY, gains, job.sched, it, job.n_iter - it)
            st = plan.query()
            if st["status"] == 0:
                break
            if st["status"] != 4:
                raise RuntimeError("job %d failed with device status %d" % (job.jid, st["status"]))
            it = st["iter"]
            cap *= 2
            job.replans += 1
        job.finished = time.perf_counter() - t0
        job.Y_out = Y.cpu().numpy()
        out.append(job)
        if log:
            log("job %d n=%d done at %.2fs" % (job.jid, job.n, job.finished))
    return summarize(out, time.perf_counter() - t0)
