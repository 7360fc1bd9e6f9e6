"""Benchmark of the greedy blue-noise ordering on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one full ordering of one synthetic object: input validation,
every greedy step (select + min-distance update) and the emitted order and
radii, with the candidates already resident in HBM.  The default workload is
one CAD-like part: the union boundary of 200 random boxes/cylinders, 4,194,304
binary32 candidates, ordered to k = 262,144.

Prints one JSON line (metric, value = ordered surfels/s, roofline of the
dominant kernel measured with HIP events on the launch stream, and the CPU
oracle timed on a bounded sample on this host).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (n, k, seed, generator)
    "cad_part": (4194304, 262144, 2, "cad_part"),
    "sphere_box": (16384, 16384, 1, "sphere_and_box"),
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def make_points(gen, n, seed, device):
    import synth
    if gen == "cad_part":
        return synth.cad_part(n, seed=seed, device=device)
    return synth.sphere_and_box(n=n, seed=seed, device=device)


def algorithmic_bytes_full_scan(n, k):
    """16 B (xyz + min-distance) read per live candidate per update; the
    update after pick t-1 (t = 1..k-1) runs over n - t live candidates."""
    if k < 2:
        return 0
    live = (k - 1) * n - (k * (k - 1)) // 2
    return 16 * live


def cpu_baseline(points_host, k, start, budget_s=30.0):
    """Oracle timed on this host on a bounded sample of the workload."""
    import numpy as np
    import oracle
    P = np.ascontiguousarray(points_host)
    n = P.shape[0]
    # grid-accelerated exact oracle (single thread) on the full workload if it
    # fits the budget, else on a prefix of the steps
    kk = k
    t0 = time.perf_counter()
    order, radius = oracle.greedy32_grid(P, kk, start)
    dt = time.perf_counter() - t0
    return {"value": kk / dt, "unit": "ordered surfels/s", "cores": 1, "kind": "oracle",
            "sample": "exact grid oracle (bs_oracle.c, 1 thread), full workload n=%d k=%d, %.1f s" % (n, kk, dt)}, order


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cad_part", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel", type=int, default=0)
    ap.add_argument("--per-thread", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build orders each object on a single MI355X; "
              "--gpus %d is not supported (see the sharding note in DESIGN.md)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1904_08225_amd as bs

    n, k, seed, gen = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    surf = make_points(gen, n, seed, dev)
    pts = surf.points.contiguous()
    torch.cuda.synchronize()
    log("generated %s n=%d in %.1fs" % (args.workload, n, time.time() - t0))

    tune = bs.tuning(kernel=args.kernel, block=args.block, per_thread=args.per_thread)
    ws = torch.empty(max(bs.workspace_size(n, k, tune), 1), dtype=torch.uint8, device=dev)
    out_o = torch.empty(k, dtype=torch.int32, device=dev)
    out_r = torch.empty(k, dtype=torch.float32, device=dev)
    start = bs.start_index(seed, n)
    stream = torch.cuda.current_stream()

    def step():
        bs.order(pts, k, seed=seed, normals=surf.normals, colors=surf.colors, tune=tune, workspace=ws,
                 out_order=out_o, out_radius=out_r, check=False)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log("warmup %d done" % i)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    kern_ms = ev0.elapsed_time(ev1) / args.steps
    ms = wall * 1000.0 / args.steps
    log("timed %d steps: %.3f ms/step wall, %.3f ms/step events" % (args.steps, ms, kern_ms))

    value = k / (ms / 1000.0)
    abytes = algorithmic_bytes_full_scan(n, k)
    achieved = abytes / (kern_ms / 1000.0) / 1e9
    kernel = bs.auto_kernel(n, k) if args.kernel == 0 else args.kernel
    rec = {
        "metric": "ordered surfels/sec (exact greedy blue-noise ordering)",
        "value": value,
        "unit": "ordered surfels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "k": k, "seed": seed, "kernel": kernel,
                   "per_step_us": kern_ms * 1000.0 / max(k - 1, 1)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
    }
    if not args.no_cpu_baseline:
        host = pts.cpu().numpy()
        cb, eo = cpu_baseline(host, k, start)
        rec["cpu_baseline"] = cb
        got = out_o.cpu().numpy()
        rec["config"]["matches_oracle"] = bool(np.array_equal(got, eo))
        log("cpu baseline: %s" % cb["sample"])
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
