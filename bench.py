#!/usr/bin/env python3
"""Throughput of one t-SNE gradient iteration on one MI355X.

Workload: N = 1,000,000 points in 2-D drawn from 50 Gaussian clusters (centres
uniform in [-95, 95]^2, sd 2) with a random 90-neighbour P (about 9e7
non-zeros), FP32, p = 5 Lagrange nodes per interval; the interval width and
the launch knobs come from the autotuner (accuracy target 1e-3).  A step is
one full iteration: box, binning, spreading, FFT convolution, gather and Z,
attraction and the descent update, replayed from a captured HIP graph.

Prints one JSON line: iterations/s, the roofline of the dominant kernel (the
CSR attraction, timed with HIP events on the plan's stream; its measured HBM
traffic comes from the committed counter summary when that summary was taken
on the same kernel source and launch knobs) and the CPU oracle timed on a
bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 (vector and matrix)
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_attr_traffic_n1e6_2d.txt")
ATTR_SOURCES = [os.path.join(ROOT, "paper_1712_09005_amd", "csrc", f)
                for f in ("k_attr.hip", "tsne_dev.h", "launch.h")]


def measured_traffic(knobs):
    """HBM bytes per attraction launch from the counter summary (FETCH_SIZE
    and WRITE_SIZE, scaled by a plain copy of known size), or None if the
    summary is missing or was taken on another kernel source or knobs."""
    try:
        fields = {}
        with open(TRAFFIC_SUMMARY) as f:
            for line in f:
                if ":" in line and not line.startswith(" "):
                    k, v = line.split(":", 1)
                    fields[k.strip()] = v.strip()
        h = hashlib.sha256()
        for path in ATTR_SOURCES:
            with open(path, "rb") as f:
                h.update(f.read())
        sha = h.hexdigest()
        if fields.get("source_sha256") != sha:
            return None
        want = "lanes_per_row=%d attr_slabs=%d attr_layout=%d" % (
            knobs.get("lanes_per_row", 0), knobs.get("attr_slabs", 0), knobs.get("attr_layout", 0))
        if fields.get("knobs") != want:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--p", type=int, default=None,
                    help="Lagrange nodes per interval (default: autotuned with the width for "
                         "the 2-D step benchmark, else 5)")
    ap.add_argument("--width", type=float, default=None,
                    help="interval width (default: autotuned for the 2-D step benchmark, "
                         "0.75 for the other 2-D workloads, 0.5 in 1-D)")
    ap.add_argument("--no-tune", action="store_true",
                    help="2-D step benchmark: skip the autotuner (default knobs, width 0.75)")
    ap.add_argument("--form", default=None, choices=["A", "B", "V"],
                    help="charge/kernel form of the repulsion (default: autotuned between A and V)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-pca", action="store_true", help="skip the randomised-PCA workload")
    ap.add_argument("--pca-m", type=int, default=1_000_000)
    ap.add_argument("--pca-n", type=int, default=30_000)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--workload", default="c3", choices=["c3", "c4", "c2", "serve"],
                    help="c3: N=1e6 2-D step throughput (default); c4: N=1e6 1-D 750-iteration "
                         "run; c2: N=1e5 2-D 1000-iteration run from a 50-d mixture; serve: "
                         "64-job continuous-batching server vs sequential runs")
    ap.add_argument("--jobs", type=int, default=64)
    ap.add_argument("--slots", type=str, default="8",
                    help="serving: batch slots (jobs live at once); a comma list runs the "
                         "batched server once per value and reports each")
    ap.add_argument("--copy-ref", action="store_true",
                    help="after the benchmark, copy a 512 MiB buffer three times (a plain copy "
                         "kernel of known size that scales HBM counters under a profiler)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload != "c3":
        if args.form is None:
            args.form = "V"
        if args.p is None:
            args.p = 5
        if args.width is None:
            # serving with form V: 0.65 gives the final embeddings the error form A
            # has at 0.75 (about 3e-4 on the smallest jobs)
            if args.workload == "c4":
                args.width = 0.5
            elif args.workload == "serve" and args.form == "V":
                args.width = 0.65
            else:
                args.width = 0.75
        return other_workloads(args)

    import numpy as np
    import torch
    from paper_1712_09005_amd import inputs, tsne

    dev = torch.device("cuda:0")
    n, s = args.n, 2
    t0 = time.time()
    Y = inputs.mixture_embedding(n, s, 50, -95.0, 95.0, 2.0, seed=0)
    P = inputs.random_graph_P(n, 90, seed=1)
    log("inputs: n=%d nnz=%d (%.1f s)" % (n, P.nnz, time.time() - t0))

    max_int = 512                     # grid capacity (intervals per dimension)
    knobs = {}
    tuned = None
    if not args.no_tune:
        # autotuner: interval width for the accuracy target, then launch knobs
        from paper_1712_09005_amd import autotune
        t0 = time.time()
        if args.width is None and args.p is None:
            forms = (args.form,) if args.form else ("A", "V")
            ti = autotune.tune_interp(Y, target=1e-3, safety=2.5, max_intervals=max_int,
                                      device=dev, log=log, forms=forms)
            args.form, args.p, args.width = ti["form"], ti["p"], ti["interval_width"]
        elif args.width is None:
            args.form = args.form or "A"
            tw = autotune.tune_width(Y, target=1e-3, safety=2.5, p=args.p, device=dev, log=log,
                                     form=args.form)
            args.width = tw["interval_width"]
    if args.form is None:
        args.form = "A"
    if args.p is None:
        args.p = 5
    if args.width is None:
        args.width = 0.75
    if not args.no_tune:
        ta = autotune.tune_attraction(Y, P, p=args.p, device=dev, log=log)
        tsp = autotune.tune_spread(Y, p=args.p, interval_width=args.width, max_intervals=max_int,
                                   device=dev, log=log, form=args.form)
        knobs = dict(lanes_per_row=ta["lanes_per_row"], attr_slabs=ta["attr_slabs"],
                     attr_layout=ta["attr_layout"], points_per_lane=tsp["points_per_lane"])
        tuned = dict(knobs, form=args.form, p=args.p, interval_width=args.width,
                     seconds=round(time.time() - t0, 1))
        log("autotuned: %s" % tuned)
    plan = tsne.Plan(n, s, torch.float32, p=args.p, policy="fixed", interval_width=args.width,
                     form=args.form, max_intervals=max_int, nnz=P.nnz, device=dev, **knobs)
    st_ = plan.stream
    with torch.cuda.stream(st_):
        Yt = torch.from_numpy(Y).to(dev)
        uY = torch.zeros_like(Yt)
        gains = torch.ones_like(Yt)
        rp = torch.from_numpy(P.row_ptr).to(dev)
        col = torch.from_numpy(P.col).to(dev)
        val = torch.from_numpy(P.val).to(dev)
    torch.cuda.synchronize()
    plan.bind_P(rp, col, val)
    sched = tsne.Schedule()          # early exaggeration phase: alpha = 12

    # warm-up (builds the kernel spectra, captures the graph)
    plan.run(Yt, uY, gains, sched, 0, max(1, args.warmup))
    torch.cuda.synchronize()
    q = plan.query()
    if q["status"] != 0:
        raise SystemExit("device status %d after warm-up" % q["status"])
    log("warm-up done: n_int=%d nodes=%d M=%d" % (q["n_int"], q["n_nodes"], q["fft_len"]))

    # timed region: exactly K iterations
    K = args.steps
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.run(Yt, uY, gains, sched, args.warmup, K)
    st_.synchronize()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    elapsed = t2 - t1
    q = plan.query()
    if q["status"] != 0:
        raise SystemExit("device status %d in the timed region" % q["status"])
    ips = K / elapsed
    log("timed: %d iterations in %.4f s -> %.1f it/s" % (K, elapsed, ips))

    # dominant kernel: the attraction step (k_attr, plus k_asum summing the
    # column-slab partials when slabs > 1), timed with HIP events on the
    # plan's stream over R back-to-back calls through the C ABI
    import ctypes
    R = 50
    with torch.cuda.stream(st_):
        Fa = torch.empty_like(Yt)
    plan.attractive(Yt, Fa)
    st_.synchronize()
    fn = tsne.lib().tsne_attractive
    yp, fp = ctypes.c_void_p(Yt.data_ptr()), ctypes.c_void_p(Fa.data_ptr())
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(st_)
    for _ in range(R):
        rc = fn(plan._h, yp, fp)
        if rc != 0:
            raise SystemExit("tsne_attractive failed with status %d" % rc)
    ev1.record(st_)
    ev1.synchronize()
    t_attr = ev0.elapsed_time(ev1) / 1e3 / R
    alg_bytes = 8 * (n + 1) + 8 * P.nnz + 3 * 8 * n   # row_ptr, col+val, own y, y_j once, F
    achieved = alg_bytes / t_attr / 1e9
    log("attraction: %.1f us per launch, %.1f GB/s algorithmic" % (t_attr * 1e6, achieved))

    # KL divergence at the final Y: the repulsion chain for Z plus one pass
    # over P (not part of a step), timed the same way
    with torch.cuda.stream(st_):
        klv = torch.empty(1, dtype=torch.float64, device=dev)
    fnk = tsne.lib().tsne_kl_divergence
    kp = ctypes.c_void_p(klv.data_ptr())
    if fnk(plan._h, yp, kp) != 0:
        raise SystemExit("tsne_kl_divergence failed")
    ev0.record(st_)
    for _ in range(20):
        fnk(plan._h, yp, kp)
    ev1.record(st_)
    ev1.synchronize()
    kl_info = {"value": float(klv.item()), "ms_per_call": ev0.elapsed_time(ev1) / 20}
    log("KL divergence %.6f, %.3f ms per call" % (kl_info["value"], kl_info["ms_per_call"]))

    pca_info = None if args.no_pca else pca_leg(args, dev)

    # accuracy on sampled rows against the direct sum (repulsion numerators)
    rel_err = None
    cpu = None
    if not args.no_cpu:
        import oracle
        rng = np.random.default_rng(123)
        rows = np.sort(rng.choice(n, 512, replace=False))
        Fr, Z = plan.repulsive(Yt)
        torch.cuda.synchronize()
        Rnum = np.frombuffer(plan.export(2), np.float32).reshape(n, s)[rows].astype(np.float64)
        Yd = Yt.cpu().numpy().astype(np.float64)
        h1, num = oracle.direct_sums(Yd, rows)
        rel_err = float(np.linalg.norm(Rnum - num) / np.linalg.norm(num))
        log("sampled repulsion numerators vs direct sum: rel err %.2e" % rel_err)
        # CPU oracle baseline: direct per-row sums on a sample of rows, plus the
        # full attraction and update, scaled to one iteration
        Pd = inputs.CSR(P.row_ptr, P.col, P.val.astype(np.float64))
        ta = time.perf_counter()
        Fa_ref = oracle.attr(Yd, Pd)
        t_attr_cpu = time.perf_counter() - ta
        nrow = 256
        while True:
            sample = rng.choice(n, nrow, replace=False)
            tb = time.perf_counter()
            oracle.direct_sums(Yd, sample)
            t_rows = time.perf_counter() - tb
            if t_rows > args.cpu_seconds / 4 or nrow >= n:
                break
            nrow = min(n, int(nrow * max(2.0, (args.cpu_seconds / 4) / max(t_rows, 1e-3))))
        tu = time.perf_counter()
        oracle.update(Yd, np.zeros_like(Yd), np.ones_like(Yd), Fa_ref, np.zeros_like(Yd),
                      12.0, 0.5, 200.0)
        t_upd = time.perf_counter() - tu
        t_iter = t_rows * n / nrow + t_attr_cpu + t_upd
        cpu = {"value": 1.0 / t_iter, "unit": "iterations/s", "cores": oracle.threads(),
               "kind": "oracle",
               "sample": "direct O(N^2) repulsion for %d sampled rows (%.1f s, scaled by N/rows) "
                         "+ full attraction (%.2f s) + update (%.2f s); FP64" %
                         (nrow, t_rows, t_attr_cpu, t_upd)}
        log("cpu oracle: %.3g s per iteration on %d threads" % (t_iter, oracle.threads()))

    out = {
        "metric": "t-SNE iters/s at N=1M 2D (rel err<=1e-3)",
        "value": ips,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "N=1e6 2-D, 50-cluster Gaussian mixture on [-95,95]^2 sd 2, "
                               "random 90-neighbour P",
                   "n": n, "s": s, "nnz": int(P.nnz), "p": args.p, "interval_width": args.width,
                   "n_int": q["n_int"], "fft_len": q["fft_len"], "max_intervals": max_int,
                   "form": args.form,
                   "autotuned": tuned, "kl_divergence": kl_info, "pca": pca_info,
                   "rel_err_rep_numerators_sampled": rel_err},
        "roofline": {"bound": "hbm", "kernel": "attraction step: k_attr (+ k_asum when "
                                               "attr_slabs > 1)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(knobs),
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_us": t_attr * 1e6},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if args.copy_ref:
        copy_reference()


def pca_leg(args, dev, rank=50, k=50, l=52, its=2, reps=2):
    """Randomised PCA (Section 6, Algorithm 2) of a planted rank-50 FP64
    matrix, by default the section's 1,000,000 x 30,000 (240 GB, resident in
    HBM): seconds per call, FP64 rate of its big products, error of the
    singular values against the planted ones, and the oracle's time on a
    row sample of the same matrix."""
    import numpy as np
    import torch
    from paper_1712_09005_amd import inputs, pca
    m, n = args.pca_m, args.pca_n
    info = {"workload": "%d x %d FP64, planted rank %d (cosine factors, singular values 1 .. 1e-2), "
                        "A in HBM" % (m, n, rank), "m": m, "n": n, "k": k, "l": l, "its": its}
    try:
        torch.cuda.empty_cache()
        U0, s0, V0 = inputs.low_rank_factors(m, n, rank, seed=30)
        A = (torch.from_numpy(U0).to(dev) * torch.from_numpy(s0).to(dev)) @ \
            torch.from_numpy(V0).to(dev).T.contiguous()
        om = inputs.pca_omega(n, l, seed=31)
        U, s, V = pca.oocpca(A, om, k=k, its=its)     # warm-up (workspace, code objects)
        torch.cuda.synchronize()
        st_ = torch.cuda.current_stream()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(st_)
        for _ in range(reps):
            U, s, V = pca.oocpca(A, om, k=k, its=its)
        ev1.record(st_)
        ev1.synchronize()
        sec = ev0.elapsed_time(ev1) / 1e3 / reps
        gemms = 2 * its + 2
        flops = gemms * 2.0 * m * n * l
        info.update({"seconds_per_call": sec, "passes_over_A": its + 2, "big_products": gemms,
                     "tflops": flops / sec / 1e12, "fp64_peak_tflops": FP64_PEAK_TFLOPS,
                     "frac": flops / sec / 1e12 / FP64_PEAK_TFLOPS,
                     "max_rel_err_sigma": float(np.max(np.abs(s.cpu().numpy() - s0) / s0))})
        log("pca %d x %d: %.3f s per call, %.1f TFLOP/s FP64" % (m, n, sec, flops / sec / 1e12))
        del A, U, s, V
        torch.cuda.empty_cache()
        # out of core: a tenth of the rows in pinned host memory, streamed to
        # the device in 16,384-row blocks once per pass
        mh = m // 10
        Ah = torch.empty((mh, n), dtype=torch.float64, pin_memory=True)
        Ah.copy_(torch.from_numpy((U0[:mh] * s0) @ V0.T))
        An = Ah.numpy()
        pca.oocpca(An, om, k=k, its=its)
        t0 = time.perf_counter()
        pca.oocpca(An, om, k=k, its=its)
        torch.cuda.synchronize()
        th = time.perf_counter() - t0
        info["host_streamed"] = {"m": mh, "b": 16384, "seconds_per_call": th, "passes_over_A": its + 2,
                                 "stream_GBps": (its + 2) * mh * n * 8 / th / 1e9,
                                 "note": "A in pinned host memory, copied to the device in b-row "
                                         "blocks; wall time of one call"}
        log("pca out of core, %d rows: %.3f s per call, %.1f GB/s streamed" %
            (mh, th, (its + 2) * mh * n * 8 / th / 1e9))
        del Ah, An
        if not args.no_cpu:
            from oracle import pca as opca
            ms = 20_000
            Us = U0[:ms]
            As = (Us * s0) @ V0.T
            t0 = time.perf_counter()
            opca.oocpca(As, om, k=k, its=its, b=4096)
            tc = time.perf_counter() - t0
            info["cpu_oracle"] = {"seconds_scaled": tc * m / ms, "sample_rows": ms,
                                  "sample_seconds": tc, "kind": "oracle",
                                  "note": "the first %d rows of the same matrix; time scaled by m / rows" % ms}
            log("pca oracle on %d rows: %.2f s" % (ms, tc))
    except (RuntimeError, MemoryError) as e:
        info["error"] = str(e)[:200]
        torch.cuda.empty_cache()
    return info


def copy_reference(nbytes=512 << 20, reps=3):
    """Device-to-device copies of ``nbytes`` (reads and writes nbytes each)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copy reference: %d x %d bytes" % (reps, nbytes))


def sampled_error(plan, Yt, n, s, rows=512, seed=123):
    """Relative L2 error of the repulsion numerators on sampled rows against
    the direct sum (the normalisation Z cancels out of the comparison)."""
    import numpy as np
    import oracle
    import torch
    rng = np.random.default_rng(seed)
    r = np.sort(rng.choice(n, min(rows, n), replace=False))
    plan.repulsive(Yt)
    torch.cuda.synchronize()
    Rn = np.frombuffer(plan.export(2), np.float32).reshape(n, s)[r].astype(np.float64)
    Yd = Yt.cpu().numpy().astype(np.float64)
    _, num = oracle.direct_sums(Yd, r)
    return float(np.linalg.norm(Rn - num) / np.linalg.norm(num))


def timed_run(plan, Yt, uY, gains, sched, n_iter, checkpoints, n, s):
    """Run n_iter iterations from iteration 0, stopping at the checkpoints to
    measure the sampled repulsion error; returns (seconds of GPU work, errors)."""
    import torch
    errs = {}
    t = 0.0
    it = 0
    for c in sorted(set(checkpoints) | {n_iter}):
        if c > it:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.run(Yt, uY, gains, sched, it, c - it)
            plan.stream.synchronize()
            torch.cuda.synchronize()
            t += time.perf_counter() - t0
            q = plan.query()
            if q["status"] != 0:
                raise SystemExit("device status %d at iteration %d" % (q["status"], c))
            it = c
        if c in checkpoints:
            errs[str(c)] = sampled_error(plan, Yt, n, s)
    return t, errs


def other_workloads(args):
    import numpy as np
    import torch
    from paper_1712_09005_amd import inputs, tsne
    dev = torch.device("cuda:0")
    if args.workload in ("c4", "c2"):
        if args.workload == "c4":
            n, s, n_iter = 1_000_000, 1, 750
            Y = inputs.mixture_embedding(n, 1, 30, -195.0, 195.0, 1.5, seed=0)
            P = inputs.random_graph_P(n, 90, seed=1)
            sched = tsne.Schedule(ee_alpha=1.0, ee_stop=0, le_alpha=4.0, le_start=500)
            checks = [0, 500, 749]
            cap = 1024
            extra = {}
            desc = "N=1e6 1-D, 30 clusters on [-195,195] sd 1.5, random 90-neighbour P, 750 " \
                   "iterations, late exaggeration 4 from iteration 500"
        else:
            n, s, n_iter = 100_000, 2, 1000
            x = inputs.mixture_highdim(n, 50, 20, 5.0, seed=0)
            # affinities on the device: exact 90-NN, perplexity 30, symmetrised
            Xt = torch.from_numpy(x).to(dev)
            torch.cuda.synchronize()
            ta0 = time.perf_counter()
            rp_d, col_d, val_d = tsne.affinities(Xt, 90, 30.0)
            torch.cuda.synchronize()
            t_aff = time.perf_counter() - ta0
            P = inputs.CSR(rp_d.cpu().numpy(), col_d.cpu().numpy(), val_d.cpu().numpy())
            log("c2 inputs: exact 90-NN perplexity-30 P on the device in %.1f ms, nnz=%d"
                % (1e3 * t_aff, P.nnz))
            rng = np.random.default_rng(2)
            Y = (1e-2 * rng.standard_normal((n, 2))).astype(np.float32)
            sched = tsne.Schedule()
            checks = [0, 250, 500, 999]
            cap = 512
            desc = "N=1e5 2-D from a 20-cluster 50-d mixture, exact 90-NN perplexity-30 P, " \
                   "1000 iterations, early exaggeration 12 for 250"
            extra = {"affinities_ms": 1e3 * t_aff}
        plan = tsne.Plan(n, s, torch.float32, p=args.p, policy="fixed", interval_width=args.width,
                         form=args.form, max_intervals=cap, nnz=P.nnz, device=dev)
        with torch.cuda.stream(plan.stream):
            Yt = torch.from_numpy(np.ascontiguousarray(Y)).to(dev)
            uY = torch.zeros_like(Yt)
            gains = torch.ones_like(Yt)
            rp = torch.from_numpy(P.row_ptr).to(dev)
            col = torch.from_numpy(P.col).to(dev)
            val = torch.from_numpy(P.val).to(dev)
        torch.cuda.synchronize()
        plan.bind_P(rp, col, val)
        secs, errs = timed_run(plan, Yt, uY, gains, sched, n_iter, checks, n, s)
        q = plan.query()
        out = {"metric": "t-SNE iterations/s over a full run", "value": n_iter / secs,
               "unit": "iterations/s", "n_gpus": 1, "steps": n_iter, "warmup": 0,
               "ms_per_step": 1e3 * secs / n_iter, "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "f32", "data": "synthetic",
               "config": {"workload": desc, "n": n, "s": s, "nnz": int(P.nnz), "p": args.p,
                          "interval_width": args.width, "form": args.form,
                          "final_n_int": q["n_int"],
                          "final_fft_len": q["fft_len"],
                          "rel_err_rep_numerators_sampled_at": errs, **extra}}
        print(json.dumps(out), flush=True)
        return
    # serving: 64 jobs, Poisson arrivals at twice the sequential rate
    from paper_1712_09005_amd import serve
    t0 = time.time()
    raw = inputs.serving_jobs(args.jobs)
    specs = []
    t_aff = 0.0
    for y, x in raw:                       # affinities on the device, before the clock
        Xt = torch.from_numpy(x).to(dev)
        torch.cuda.synchronize()
        ta0 = time.perf_counter()
        rp_d, col_d, val_d = tsne.affinities(Xt, 90, 30.0)
        torch.cuda.synchronize()
        t_aff += time.perf_counter() - ta0
        specs.append((y, inputs.CSR(rp_d.cpu().numpy(), col_d.cpu().numpy(), val_d.cpu().numpy())))
    del raw
    log("serving inputs: %d jobs, N from %d to %d (%.1f s; device affinities %.2f s in all)" % (
        len(specs), min(y.shape[0] for y, _ in specs), max(y.shape[0] for y, _ in specs),
        time.time() - t0, t_aff))

    def jobs_at(arrivals):
        return [serve.Job(j, float(a), y, P) for j, ((y, P), a) in enumerate(zip(specs, arrivals))]

    # autotuner: lanes per row of the shared attraction launch, over a sample of jobs
    lanes = 32
    if not args.no_tune:
        from paper_1712_09005_amd import autotune
        lanes = autotune.tune_batch_lanes(specs[::8], p=args.p, device=dev, log=log)["lanes_per_row"]
        log("autotuned lanes per row: %d" % lanes)
    back_to_back = serve.sequential(jobs_at(np.zeros(len(specs))), interval_width=args.width,
                                    p=args.p, lanes_per_row=lanes, device=dev, form=args.form)
    rate = 2.0 * back_to_back["runs_per_s"]
    arr = inputs.poisson_arrivals(len(specs), rate, seed=7)
    log("sequential back-to-back: %.2f runs/s; Poisson rate %.2f/s" % (back_to_back["runs_per_s"], rate))
    slot_list = [int(x) for x in args.slots.split(",")]
    runs = {}
    for k in slot_list:
        srv = serve.Server(max_slots=k, hbm_budget=200 << 30, ticks_per_poll=10,
                           interval_width=args.width, p=args.p, lanes_per_row=lanes, device=dev,
                           form=args.form)
        jobs_k = jobs_at(arr)
        runs[k] = (srv.run(jobs_k), jobs_k)
        log("batched, %d slots: %s" % (k, runs[k][0]))
        del srv
    batched, batched_jobs = runs[slot_list[0]]
    seq_jobs = jobs_at(arr)
    seq = serve.sequential(seq_jobs, interval_width=args.width, p=args.p, lanes_per_row=lanes,
                           device=dev, form=args.form)
    log("sequential: %s" % seq)
    # equal accuracy: repulsion error of the final embeddings of the smallest jobs
    import oracle
    acc = []
    for jb, js in sorted(zip(batched_jobs, seq_jobs), key=lambda t: t[0].n)[:3]:
        errs = []
        for Yo in (jb.Y_out, js.Y_out):
            plan = tsne.Plan(jb.n, 2, torch.float32, p=args.p, interval_width=args.width,
                             form=args.form, max_intervals=serve.capacity_for(jb.n, args.width) * 2,
                             device=dev)
            Yt = torch.from_numpy(np.ascontiguousarray(Yo)).to(dev)
            F, Z = plan.repulsive(Yt)
            torch.cuda.synchronize()
            Fd, Zd = oracle.direct_rep(Yo.astype(np.float64))
            errs.append(float(np.linalg.norm(F.cpu().numpy() - Fd) / np.linalg.norm(Fd)))
        acc.append({"job": jb.jid, "n": jb.n, "rel_err_batched": errs[0], "rel_err_sequential": errs[1]})
    out = {"metric": "served t-SNE runs/s (64 jobs, 1000 iterations each)", "value": batched["runs_per_s"],
           "unit": "runs/s", "n_gpus": 1, "steps": len(specs), "warmup": 0,
           "ms_per_step": 1e3 * batched["makespan_s"] / len(specs), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "64 jobs, N log-uniform [5e3, 2e5], 5-30 cluster 50-d mixtures, "
                                  "exact 90-NN perplexity-30 P, Poisson arrivals at 2x the "
                                  "sequential rate", "batched": batched, "sequential_same_trace": seq,
                      "sequential_back_to_back": back_to_back, "lanes_per_row": lanes,
                      "form": args.form, "p": args.p, "interval_width": args.width,
                      "slots": slot_list[0],
                      "batched_by_slots": {str(k): v[0] for k, v in runs.items()},
                      "speedup_runs_per_s": batched["runs_per_s"] / seq["runs_per_s"],
                      "accuracy_final_embeddings": acc}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
