"""Autotuner for the plan's launch knobs and its interval width.

Two kinds of choices are tuned.

* Launch knobs: CSR lanes per row, column slabs and layout of the attraction,
  and points per lane of the spreading kernel.  They change results only by
  summation order.  Each candidate is timed on the caller's own Y and P with
  HIP events on the plan's stream (median over repeated launches), and the
  fastest wins.
* The interval width w.  It trades accuracy for grid size: the interpolation
  error falls like w^p (Section 2.3).  The error of a width is estimated
  without any reference code: the same repulsion is computed at w and at w/2.
  The finer result is about 2^p times more accurate, so
  e(w) ~ |F(w) - F(w/2)| / |F(w/2)| (relative L2 over all components).
  The tuner returns the largest width on a ladder whose estimate, times a
  safety factor, meets the target.  The embedding given to it should be
  representative: the error grows as clusters tighten during a run.

Results are cached in a JSON file keyed by device, problem size bucket, s,
dtype and p.  The cache path is ``$TSNE_TUNE_CACHE`` or
``~/.cache/tsne_mi355x/tune.json``; ``cache=None`` disables it.
"""
from __future__ import annotations

import json
import math
import os
import statistics

import numpy as np
import torch

from . import tsne

WIDTHS = (1.6, 1.5, 1.4, 1.3, 1.2, 1.1, 1.0, 0.95, 0.9, 0.85, 0.8, 0.75, 0.7, 0.65, 0.6,
          0.55, 0.5, 0.45, 0.4, 0.35, 0.3, 0.25, 0.2)
PS = (3, 4, 5, 6)
# CSR rows at every lanes-per-row and slab count, and the row-block sweep over
# LDS column windows (layout 2, whose 64-bit fixed-point row sums give the same
# bits in any order; lanes and slabs do not apply to it)
CSR_KNOBS = [(lpr, sl, 1) for lpr in (4, 8, 16, 32, 64) for sl in (1, 2, 4, 8)] + [(0, 0, 2)]
KPTS = (4, 8, 16)


def default_cache() -> str:
    return os.environ.get("TSNE_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "tsne_mi355x",
                                       "tune.json"))


def _bucket(x: int) -> int:
    """Round to the nearest power of two (cache key granularity)."""
    return 1 << max(0, int(round(math.log2(max(1, x)))))


def _key(kind, device, n, nnz, s, dtype, p, extra=""):
    pr = torch.cuda.get_device_properties(device)
    name = "%dCU-%dGiB" % (pr.multi_processor_count, pr.total_memory >> 30)
    return "%s|%s|n%d|nnz%d|s%d|%s|p%d%s" % (kind, name, _bucket(n), _bucket(nnz), s,
                                              "f32" if dtype == torch.float32 else "f64", p, extra)


def _load(cache):
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                return json.load(f)
        except (OSError, ValueError):
            return {}
    return {}


def _store(cache, key, value):
    if not cache:
        return
    d = _load(cache)
    d[key] = value
    os.makedirs(os.path.dirname(cache) or ".", exist_ok=True)
    tmp = cache + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, cache)


def time_launches(fn, stream, reps=15, warm=2, inner=5) -> float:
    """Seconds per ``fn()``: the median over ``reps`` groups of ``inner``
    back-to-back calls, each group bracketed by HIP events recorded on
    ``stream`` (the stream the library enqueues on).  Grouping hides the host
    time between calls, which a single bracketed call would count."""
    for _ in range(warm):
        fn()
    ts = []
    for _ in range(max(1, reps // inner + 2)):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(inner):
            fn()
        e1.record(stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3 / inner)
    return statistics.median(ts)


def _device_P(P, device, dtype):
    return (torch.as_tensor(P.row_ptr, dtype=torch.int64).to(device),
            torch.as_tensor(P.col, dtype=torch.int32).to(device),
            torch.as_tensor(P.val).to(device, dtype))


def tune_attraction(Y, P, dtype=torch.float32, p=5, device="cuda:0", candidates=None,
                    reps=15, cache="default", log=None) -> dict:
    """Fastest (lanes_per_row, attr_slabs, attr_layout) for this Y and P.
    Returns {"lanes_per_row", "attr_slabs", "attr_layout", "seconds", "table"}."""
    cache = default_cache() if cache == "default" else cache
    dev = torch.device(device)
    n, s = Y.shape
    key = _key("attr", dev, n, P.nnz, s, dtype, p)
    hit = _load(cache).get(key)
    if hit is not None:
        return hit
    Yt = torch.as_tensor(np.ascontiguousarray(Y)).to(dev, dtype)
    rp, col, val = _device_P(P, dev, dtype)
    table = []
    best = None
    for lpr, sl, layout in (candidates or CSR_KNOBS):
        plan = tsne.Plan(n, s, dtype, p=p, nnz=P.nnz, lanes_per_row=lpr, attr_slabs=sl,
                         attr_layout=layout, max_intervals=16, device=dev)
        plan.bind_P(rp, col, val)
        with torch.cuda.stream(plan.stream):
            Fa = torch.empty_like(Yt)
        torch.cuda.synchronize()
        t = time_launches(lambda: plan.attractive(Yt, Fa), plan.stream, reps)
        table.append([lpr, sl, layout, t])
        if log:
            log("  attraction lanes=%d slabs=%d layout=%d: %.1f us" % (lpr, sl, layout, t * 1e6))
        if best is None or t < best[3]:
            best = (lpr, sl, layout, t)
        del plan
    out = {"lanes_per_row": best[0], "attr_slabs": best[1], "attr_layout": best[2],
           "seconds": best[3], "table": table}
    _store(cache, key, out)
    return out


def _fkey(form):
    return "" if form in ("A", tsne.FORM_A) else "|f%s" % form


def tune_spread(Y, dtype=torch.float32, p=5, interval_width=0.75, max_intervals=512,
                device="cuda:0", candidates=KPTS, reps=15, cache="default", log=None,
                form="A") -> dict:
    """Fastest points_per_lane for the spreading kernel, timed over the whole
    repulsion (box to gather) at this Y.  Returns {"points_per_lane", "seconds", "table"}."""
    cache = default_cache() if cache == "default" else cache
    dev = torch.device(device)
    n, s = Y.shape
    key = _key("spread", dev, n, 0, s, dtype, p, "|w%g" % interval_width + _fkey(form))
    hit = _load(cache).get(key)
    if hit is not None:
        return hit
    Yt = torch.as_tensor(np.ascontiguousarray(Y)).to(dev, dtype)
    table = []
    best = None
    for k in candidates:
        plan = tsne.Plan(n, s, dtype, p=p, interval_width=interval_width, form=form,
                         max_intervals=max_intervals, points_per_lane=k, device=dev)
        with torch.cuda.stream(plan.stream):
            F = torch.empty_like(Yt)
            Z = torch.empty(1, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t = time_launches(lambda: plan.repulsive(Yt, F, Z), plan.stream, reps)
        if plan.query()["status"] != 0:
            raise RuntimeError("repulsion failed while tuning (box larger than max_intervals?)")
        table.append([k, t])
        if log:
            log("  repulsion points_per_lane=%d: %.1f us" % (k, t * 1e6))
        if best is None or t < best[1]:
            best = (k, t)
        del plan
    out = {"points_per_lane": best[0], "seconds": best[1], "table": table}
    _store(cache, key, out)
    return out


def estimate_error(Y, interval_width, dtype=torch.float32, p=5, device="cuda:0",
                   max_intervals=4096, form="A") -> float:
    """Estimated relative L2 error of F_rep at ``interval_width``: the
    difference to the same computation at half the width (in FP64, so that
    FP32 rounding does not mask the interpolation error)."""
    dev = torch.device(device)
    n, s = Y.shape
    Yt = torch.as_tensor(np.ascontiguousarray(Y)).to(dev, torch.float64)
    out = []
    for w in (interval_width, 0.5 * interval_width):
        L = float(np.max(Y.max(0) - Y.min(0)))
        need = int(math.ceil(max(L, 1e-6) / w)) + 1
        if need > max_intervals:
            raise ValueError("box of side %.3g needs %d intervals at width %g" % (L, need, w))
        plan = tsne.Plan(n, s, torch.float64, p=p, interval_width=w, max_intervals=need,
                         form=form, device=dev)
        F, _ = plan.repulsive(Yt)
        torch.cuda.synchronize()
        if plan.query()["status"] != 0:
            raise RuntimeError("repulsion failed while estimating the error")
        out.append(F.cpu().numpy())
        del plan
    coarse, fine = out
    return float(np.linalg.norm(coarse - fine) / np.linalg.norm(fine))


def tune_width(Y, target=1e-3, safety=2.0, p=5, device="cuda:0", widths=WIDTHS,
               cache="default", log=None, form="A") -> dict:
    """Largest width on the ladder with safety * estimated error <= target.
    Returns {"interval_width", "estimate", "table"}."""
    cache = default_cache() if cache == "default" else cache
    dev = torch.device(device)
    n, s = Y.shape
    L = float(np.max(Y.max(0) - Y.min(0)))
    key = _key("width", dev, n, 0, s, torch.float64, p,
               "|L%d|t%g|k%g" % (_bucket(int(L)), target, safety) + _fkey(form))
    hit = _load(cache).get(key)
    if hit is not None:
        return hit
    table = []
    chosen = None
    for w in sorted(widths, reverse=True):
        try:
            e = estimate_error(Y, w, p=p, device=dev, form=form)
        except (ValueError, tsne.TsneError) as ex:   # the half-width grid no longer fits
            if log:
                log("  width %.3g: not evaluated (%s)" % (w, ex))
            break
        table.append([w, e])
        if log:
            log("  width %.3g: estimated error %.2e" % (w, e))
        if safety * e <= target:
            chosen = (w, e)
            break
    if chosen is None:
        raise RuntimeError("no width on the ladder meets the target %g" % target)
    out = {"interval_width": chosen[0], "estimate": chosen[1], "table": table}
    _store(cache, key, out)
    return out


def max_capacity(p: int) -> int:
    """Largest interval count a plan accepts at p nodes per interval (the
    circulant of 2 N_int p nodes stays within 12288-point transforms)."""
    return 12288 // (2 * p)


def tune_interp(Y, target=1e-3, safety=2.5, ps=PS, max_intervals=512, device="cuda:0",
                reps=10, cache="default", log=None, forms=("A",)) -> dict:
    """Form, nodes per interval p and interval width together: for each
    (form, p) the widest width meeting the accuracy target (tune_width), then
    the choice whose FP32 repulsion at this Y is fastest.  A choice whose box
    needs more than max_intervals intervals is timed at the capacity it needs
    (up to the library's largest).  Returns {"form", "p", "interval_width",
    "estimate", "max_intervals", "seconds", "table"}; every (form, p) has a
    table row {"form", "p", "interval_width", "estimate", "max_intervals",
    "seconds", "note"} (seconds None when it was not timed, with the reason)."""
    cache = default_cache() if cache == "default" else cache
    dev = torch.device(device)
    n, s = Y.shape
    L = float(np.max(Y.max(0) - Y.min(0)))
    key = _key("interp", dev, n, 0, s, torch.float32, 0,
               "|L%d|t%g|k%g|p%s" % (_bucket(int(L)), target, safety, "-".join(map(str, ps)))
               + ("" if tuple(forms) == ("A",) else "|f" + "".join(forms)))
    hit = _load(cache).get(key)
    if hit is not None:
        return hit
    Yt = torch.as_tensor(np.ascontiguousarray(Y)).to(dev, torch.float32)
    table = []
    best = None
    for form, p in [(f, p) for f in forms for p in ps]:
        row = {"form": form, "p": p, "interval_width": None, "estimate": None,
               "max_intervals": None, "seconds": None, "note": ""}
        table.append(row)
        try:
            tw = tune_width(Y, target=target, safety=safety, p=p, device=dev, cache=cache, log=log,
                            form=form)
        except RuntimeError as e:
            row["note"] = str(e)
            if log:
                log("  form %s p=%d: %s" % (form, p, e))
            continue
        w = tw["interval_width"]
        row.update(interval_width=w, estimate=tw["estimate"])
        need = int(math.ceil(L / w)) + 1
        cap = max(max_intervals, need)
        if cap > max_capacity(p):
            row["note"] = "needs %d intervals, above the largest capacity %d" % (need, max_capacity(p))
            if log:
                log("  form %s p=%d width %.3g: %s" % (form, p, w, row["note"]))
            continue
        row["max_intervals"] = cap
        plan = tsne.Plan(n, s, torch.float32, p=p, interval_width=w, max_intervals=cap,
                         form=form, device=dev)
        with torch.cuda.stream(plan.stream):
            F = torch.empty_like(Yt)
            Z = torch.empty(1, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t = time_launches(lambda: plan.repulsive(Yt, F, Z), plan.stream, reps)
        if plan.query()["status"] != 0:
            row["note"] = "repulsion latched a device status"
            continue
        row["seconds"] = t
        if log:
            log("  form %s p=%d width %.3g (estimate %.2e, %d intervals): repulsion %.1f us"
                % (form, p, w, tw["estimate"], cap, t * 1e6))
        if best is None or t < best["seconds"]:
            best = row
        del plan
    if best is None:
        raise RuntimeError("no (form, p, width) meets the target %g" % target)
    out = {"form": best["form"], "p": best["p"], "interval_width": best["interval_width"],
           "estimate": best["estimate"], "max_intervals": best["max_intervals"],
           "seconds": best["seconds"], "table": table}
    _store(cache, key, out)
    return out


def tune_batch_lanes(jobs, p=5, device="cuda:0", candidates=(4, 8, 16, 32, 64), reps=10,
                     cache="default", log=None) -> dict:
    """Lanes per row for a batch's shared attraction launch: the candidate with
    the least summed attraction time over a sample of jobs [(Y, P), ...]."""
    cache = default_cache() if cache == "default" else cache
    dev = torch.device(device)
    n_tot = sum(y.shape[0] for y, _ in jobs)
    nnz_tot = sum(P.nnz for _, P in jobs)
    key = _key("batch_lanes", dev, n_tot, nnz_tot, jobs[0][0].shape[1], torch.float32, p,
               "|j%d" % len(jobs))
    hit = _load(cache).get(key)
    if hit is not None:
        return hit
    table = []
    for lpr in candidates:
        t = 0.0
        for Y, P in jobs:
            r = tune_attraction(Y, P, p=p, device=dev, candidates=[(lpr, 1, 1)], reps=reps,
                                cache=None)
            t += r["seconds"]
        table.append([lpr, t])
        if log:
            log("  batch lanes=%d: %.1f us over %d jobs" % (lpr, t * 1e6, len(jobs)))
    best = min(table, key=lambda r: r[1])
    out = {"lanes_per_row": best[0], "seconds": best[1], "table": table}
    _store(cache, key, out)
    return out
