#!/usr/bin/env python3
"""Throughput of one t-SNE gradient iteration on one MI355X.

Workload: N = 1,000,000 points in 2-D drawn from 50 Gaussian clusters (centres
uniform in [-95, 95]^2, sd 2) with a random 90-neighbour P (about 9e7
non-zeros), FP32, p = 5 Lagrange nodes per interval of width 0.75.  A step is
one full iteration: box, binning, spreading, FFT convolution, gather and Z,
attraction and the descent update, replayed from a captured HIP graph.

Prints one JSON line: iterations/s, the roofline of the dominant kernel (the
CSR attraction, timed with HIP events on the plan's stream) and the CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--p", type=int, default=5)
    ap.add_argument("--width", type=float, default=0.75)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1712_09005_amd import inputs, tsne

    dev = torch.device("cuda:0")
    n, s = args.n, 2
    t0 = time.time()
    Y = inputs.mixture_embedding(n, s, 50, -95.0, 95.0, 2.0, seed=0)
    P = inputs.random_graph_P(n, 90, seed=1)
    log("inputs: n=%d nnz=%d (%.1f s)" % (n, P.nnz, time.time() - t0))

    max_int = 512
    plan = tsne.Plan(n, s, torch.float32, p=args.p, policy="fixed", interval_width=args.width,
                     max_intervals=max_int, nnz=P.nnz, device=dev)
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

    # dominant kernel: CSR attraction, HIP events on the plan's stream
    R = 50
    with torch.cuda.stream(st_):
        Fa = torch.empty_like(Yt)
    plan.attractive(Yt, Fa)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(st_)
    for _ in range(R):
        plan.attractive(Yt, Fa)
    ev1.record(st_)
    ev1.synchronize()
    t_attr = ev0.elapsed_time(ev1) / 1e3 / R
    alg_bytes = 8 * (n + 1) + 8 * P.nnz + 3 * 8 * n   # row_ptr, col+val, own y, y_j once, F
    achieved = alg_bytes / t_attr / 1e9
    log("attraction: %.1f us per launch, %.1f GB/s algorithmic" % (t_attr * 1e6, achieved))

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
                   "n_int": q["n_int"], "fft_len": q["fft_len"], "form": "A",
                   "rel_err_rep_numerators_sampled": rel_err},
        "roofline": {"bound": "hbm", "kernel": "k_attr (CSR attraction)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_us": t_attr * 1e6},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
