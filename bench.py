"""Benchmark of the greedy blue-noise ordering on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-batch] [--no-scene]
                [--no-serve] [--no-cpu-baseline] [--no-full-scan]
                [--copy-calibration BYTES] [--profile-leg batch|serve]

A step is one full ordering of one synthetic CAD-like part -- the union
boundary of 200 random boxes/cylinders, 4,194,304 binary32 candidates,
ordered to k = 262,144 -- through the library's automatic kernel choice
(autotuned for this size before the timed steps): input validation, Morton
sort, every greedy step (select + min-distance update; at this size the
cooperative scan over all CUs with the candidates in VGPRs, several exact
picks per step) and the emitted order and radii, with the candidates
already resident in HBM.  `value` is ordered surfels per second of that step.

The same JSON line also carries
  roofline      the dominant kernel (the ordering kernel) against HBM, with
                its algorithmic bytes (16 B per candidate inside the
                covering-radius ball over its steps, counted by the CPU
                oracle on the same points) over its duration (HIP events on
                the launch stream) and the HBM traffic measured by counters
                (profiles/); the plain-definition rate (16 B per live
                candidate per step) beside it;
  lead_scan     when the grid kernel is chosen: the leading cooperative full
                scan of the same step (picks, duration, algorithmic bytes);
  latency       per-step p50 / p99 of the ordering kernel from device
                timestamps (a step emits several exact picks);
  full_scan     the cooperative register-resident full scan on the same
                input (16 B per live candidate per step);
  batched       1,000 parts of the same kind, n log-uniform 2,048..2,097,152,
                k = n/4, in one graph-captured persistent launch (cell
                occupancy autotuned), against a plain loop of one ordering
                launch per object (sampled);
  scene_batched the heterogeneous scene: 10,000 objects (thin sheets, tori,
                small-box clusters), 1.5e9 candidates, k = 12% of n;
  served        a Poisson stream (mean 200 requests/s) of jobs with n
                log-uniform 1e4..4e6, k = n/8, under an 80 GB budget:
                p50 / p99 latency and throughput, against the plain loop;
                and the same requests queued at once (capacity);
  cpu_baseline  the exact CPU oracle (grid-accelerated, one thread) on the
                same points.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_MAIN, K_MAIN, SEED_MAIN = 4194304, 262144, 2


TRAFFIC_FILES = {"grid": os.path.join(ROOT, "profiles", "grid_cad_part_4M_hbm_counters.txt"),
                 "scan_mp": os.path.join(ROOT, "profiles", "scan_mp_cad_part_4M_hbm_counters.txt")}


def measured_traffic(which):
    """HBM bytes per launch of the ordering kernel (`which`: "grid" or
    "scan_mp") from the committed FETCH_SIZE / WRITE_SIZE counter summary, or
    None when the kernel's sources have changed since the counters were taken."""
    import hashlib
    try:
        fields = dict(l.split(": ", 1) for l in open(TRAFFIC_FILES[which]).read().splitlines() if ": " in l)
        h = hashlib.sha256()
        for src in fields["kernel_sources"].split():
            h.update(open(os.path.join(ROOT, src), "rb").read())
        if h.hexdigest() != fields["kernel_source_sha256"].strip():
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def ordering_kernel_seconds(bs, pts, k, start, tune, lead=0):
    """Duration of the ordering loop from the device clock (first to last pick)
    and per-step latencies.  With a leading full scan of `lead` picks, the
    round statistics cover the grid kernel's picks (lead onward) and the
    scan's steps are reported apart."""
    import torch
    o, r, t = bs.order_profile(pts, k, start=start, tune=tune)
    torch.cuda.synchronize()
    import numpy as np
    tk = t.cpu().numpy().astype("float64")
    hz = bs.wall_clock_hz()
    lead = lead if lead >= 2 else 0
    g = tk[lead:] if lead else tk
    # picks of one round share a timestamp: latencies are per round
    rt = np.unique(g)
    d = (rt[1:] - rt[:-1]) / hz * 1e6 if rt.shape[0] > 1 else np.zeros(1)
    span = (g[-1] - g[0]) / hz
    lat = {"p50_us": float(np.percentile(d, 50)), "p99_us": float(np.percentile(d, 99)),
           "mean_us": float(d.mean()), "rounds": int(rt.shape[0]),
           "picks_per_round": float(g.shape[0] / rt.shape[0]),
           "mean_us_per_pick": float(span * 1e6 / max(1, g.shape[0] - 1))}
    if lead:
        ds = (tk[1:lead] - tk[:lead - 1]) / hz * 1e6
        lat["lead_picks"] = lead
        lat["lead_seconds"] = float((tk[lead - 1] - tk[0]) / hz)
        lat["lead_step_p50_us"] = float(np.percentile(ds, 50))
        lat["lead_step_p99_us"] = float(np.percentile(ds, 99))
    return span, lat, o


def bench_main(args, bs, torch, np):
    import synth
    dev = torch.device("cuda:0")
    t0 = time.time()
    surf = synth.cad_part(N_MAIN, seed=SEED_MAIN, device=dev)
    pts = surf.points.contiguous()
    torch.cuda.synchronize()
    log("generated cad_part n=%d in %.1fs" % (N_MAIN, time.time() - t0))
    n, k = N_MAIN, K_MAIN
    t0 = time.time()
    force = bs.tuning(kernel=bs.KERNEL_GRID) if args.plan == "grid" else None
    if args.no_autotune or force is not None:
        tuned = bs.Tuning()
    else:
        tuned = bs.autotune(pts, k, seed=SEED_MAIN)  # recorded for this size; untimed
    plan = bs.plan_describe(n, k, force)  # the plan the timed calls follow (automatic choices resolved)
    lead = int(plan.lead_picks) if plan.kernel == bs.KERNEL_GRID and plan.lead_picks > 0 else 0
    log("autotune: kernel %d block %d cells %g picks %d lead %d in %.1fs"
        % (plan.kernel, plan.block, plan.cell_points, plan.picks, lead, time.time() - t0))
    kernel = int(plan.kernel)
    ws = torch.empty(max(bs.workspace_size(n, k, force), 1), dtype=torch.uint8, device=dev)
    out_o = torch.empty(k, dtype=torch.int32, device=dev)
    out_r = torch.empty(k, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    start = bs.start_index(SEED_MAIN, n)

    def new_event():
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(stream)  # creates the handle the library records into
        return ev

    def step(events=None):
        # the same kernels as bs_order; the events bracket the ordering kernel
        bs.order_profile(pts, k, start=start, tune=force, stream=stream, ticks=False, events=events,
                         workspace=ws, out_order=out_o, out_radius=out_r)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log("warmup %d done" % i)
    kev = [(new_event(), new_event()) for _ in range(args.steps)]
    ev0, ev1 = new_event(), new_event()
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        step(kev[i])
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ev_ms = ev0.elapsed_time(ev1) / args.steps
    kern_ms = sum(b.elapsed_time(e) for b, e in kev) / args.steps
    ms = wall * 1000.0 / args.steps
    log("timed %d steps: %.1f ms/step wall, %.1f ms/step events, ordering kernel %.1f ms"
        % (args.steps, ms, ev_ms, kern_ms))
    _, lat, _ = ordering_kernel_seconds(bs, pts, k, start, force, lead)
    log("rounds %d (%.2f picks each), per-round p50 %.2f us, %.2f us per pick (device clock)"
        % (lat["rounds"], lat["picks_per_round"], lat["p50_us"], lat["mean_us_per_pick"]))
    if lead:
        log("leading full scan: %d picks in %.1f ms, p50 %.2f us per step"
            % (lead, lat["lead_seconds"] * 1e3, lat["lead_step_p50_us"]))
    return pts, surf, out_o, ms, ev_ms, kern_ms / 1e3, lat, kernel, plan, lead


def bench_emit(bs, torch, surf, pts, order):
    """The ordered 20-byte surfel records of the headline ordering (gather of
    position, normal, colour; 51 algorithmic bytes per record: 4 B index,
    12 + 12 + 3 B read, 20 B written) and r_m over the first 1000 picks."""
    nrm = surf.normals.contiguous()
    col = surf.colors.contiguous()
    k = int(order.shape[0])
    out = torch.empty((k, 20), dtype=torch.uint8, device=pts.device)
    stream = torch.cuda.current_stream()
    bs.emit_surfels(pts, order, nrm, col, out=out)
    reps = 50
    b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.record(stream)
    for _ in range(reps):
        bs.emit_surfels(pts, order, nrm, col, out=out)
    e.record(stream)
    torch.cuda.synchronize()
    secs = b.elapsed_time(e) / 1e3 / reps
    rm_b, rm_e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rm_b.record(stream)
    r_m = bs.prefix_median_nn(pts, order, 1000)
    rm_e.record(stream)
    torch.cuda.synchronize()
    abytes = 51 * k
    return {"records": k, "record_bytes": 20, "seconds": secs, "algorithmic_bytes": abytes,
            "achieved_GBs": abytes / secs / 1e9, "frac_of_hbm_peak": abytes / secs / 1e9 / HBM_PEAK_GBS,
            "median_nn_p_m": 1000, "r_m": r_m, "median_nn_seconds": rm_b.elapsed_time(rm_e) / 1e3,
            "note": "one launch of 1,024 workgroups: at this size launch latency, not HBM, bounds it"}


def bench_config1(bs, torch, np, cpu=True):
    """The small single-object workload: unit sphere + 1 x 0.5 x 0.25 box,
    16,384 candidates (seed 1), ordered completely (k = n) by the automatic
    plan; ms per ordering (HIP events around the whole call, inputs
    resident), per-step p50 / p99 from device timestamps, and the plain CPU
    oracle's time on the same points."""
    import synth
    n = 16384
    s = synth.sphere_and_box(n=n, seed=1)
    dev = torch.device("cuda:0")
    pts = s.points.to(dev).contiguous()
    start = bs.start_index(1, n)
    plan = bs.plan_describe(n, n)
    ws = torch.empty(max(bs.workspace_size(n, n), 1), dtype=torch.uint8, device=dev)
    oo = torch.empty(n, dtype=torch.int32, device=dev)
    rr = torch.empty(n, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def one():
        bs.order_profile(pts, n, start=start, stream=stream, ticks=False, workspace=ws, out_order=oo, out_radius=rr)

    for _ in range(3):
        one()
    torch.cuda.synchronize()
    reps = 20
    b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    b.record(stream)
    for _ in range(reps):
        one()
    e.record(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / reps
    ev_ms = b.elapsed_time(e) / reps
    _, lat, o = ordering_kernel_seconds(bs, pts, n, start, None)
    rec = {"workload": "sphere_and_box n=16,384 k=n=16,384 (seed 1)", "n": n, "k": n,
           "plan": {"kernel": int(plan.kernel), "block": int(plan.block), "per_thread": int(plan.per_thread),
                    "groups": int(plan.groups), "picks": int(plan.picks)},
           "ms_per_ordering": ev_ms, "wall_ms_per_ordering": wall_ms,
           "ordered_surfels_per_s": n / (ev_ms / 1e3),
           "per_step_p50_us": lat["p50_us"], "per_step_p99_us": lat["p99_us"], "steps": lat["rounds"],
           "picks_per_step": lat["picks_per_round"],
           "time_source": "HIP events around %d back-to-back orderings (validation, Morton sort, ordering) on "
                          "resident inputs; steps from the device wall clock at each pick's emission" % reps}
    if cpu:
        import oracle
        t0 = time.perf_counter()
        eo, er = oracle.greedy32(s.points.numpy(), n, start)
        cs = time.perf_counter() - t0
        rec["matches_oracle"] = bool(np.array_equal(o.cpu().numpy(), eo))
        rec["cpu_oracle"] = {"kind": "oracle", "cores": 1, "seconds": cs, "ordered_surfels_per_s": n / cs,
                             "sample": "plain binary32 oracle (oracle/bs_oracle.c, 1 thread), the whole workload"}
    return rec


def prefix_quality(bs, torch, pts, orders, prefixes=(1000, 5000, 10000)):
    """Sec. 3.3's measure: each prefix surfel's distance to its nearest other
    surfel of the prefix (bs_prefix_nn), min / median / mean relative to the
    part's bounding-box diagonal, per ordering and prefix length."""
    lo = pts.min(0).values
    hi = pts.max(0).values
    diag = float(torch.linalg.vector_norm((hi - lo).double()))
    out = {}
    for name, o in orders.items():
        rows = {}
        for p in prefixes:
            if p > o.shape[0]:
                continue
            nn = bs.prefix_nn(pts, o, p).double() / diag
            rows[str(p)] = {"min": float(nn.min()), "median": float(nn.median()), "mean": float(nn.mean())}
        out[name] = rows
    return {"bbox_diagonal": diag, "relative_nn_distance": out,
            "note": "nearest-neighbour distance inside each prefix / bounding-box diagonal (Sec. 3.3 compares "
                    "orderings by the minimum relative point distances of their prefixes)"}


def bench_sampler(bs, torch, np, pts, exact_order, cpu=True):
    """The paper's randomized sampler (Sec. 3.2, 200 samples per round, one
    more pick every 500 rounds) on the headline part, k = 262,144: ms per
    run (HIP events, inputs resident), and its prefixes against the exact
    ordering's and a random subset's (Sec. 3.3)."""
    n = int(pts.shape[0])
    k = int(exact_order.shape[0])
    dev = pts.device
    seed = SEED_MAIN
    ws = torch.empty(max(bs.load().bs_sample_workspace_size(n), 1), dtype=torch.uint8, device=dev)
    oo = torch.empty(k, dtype=torch.int32, device=dev)
    rr = torch.empty(k, dtype=torch.float32, device=dev)
    o, r, c = bs.sample(pts, k, seed=seed, workspace=ws, out_order=oo, out_radius=rr)  # warm-up
    stream = torch.cuda.current_stream()
    b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 2
    b.record(stream)
    for _ in range(reps):
        bs.sample(pts, k, seed=seed, workspace=ws, out_order=oo, out_radius=rr, check=False)
    e.record(stream)
    torch.cuda.synchronize()
    secs = b.elapsed_time(e) / 1e3 / reps
    g = torch.Generator(device=dev)
    g.manual_seed(12345)
    rnd = torch.randperm(n, generator=g, device=dev)[:k].to(torch.int32)
    rec = {"workload": "cad_part n=4,194,304 k=262,144 (the headline part), seed %d" % seed,
           "params": {"sample_size": 200, "growth_rounds": 500, "vicinity": 0.0},
           "seconds": secs, "ordered_surfels_per_s": k / secs, "picks_made": int(c),
           "exact_ordering_seconds": None,
           "kernel": "sample_single_kernel<1024,1024>: one workgroup, grid-pruned exact distances, one update "
                     "pass per pick",
           "quality": prefix_quality(bs, torch, pts, {"greedy_permutation": exact_order, "sampler": oo,
                                                      "random": rnd})}
    if cpu:
        import oracle
        host = pts.cpu().numpy()
        kk = 1500
        t0 = time.perf_counter()
        eo, _, _ = oracle.sample32(host, kk, seed, bs.start_index(seed, n))
        cs = time.perf_counter() - t0
        rec["matches_oracle_prefix"] = bool(np.array_equal(eo, oo[:kk].cpu().numpy()))
        rec["cpu_oracle"] = {"kind": "oracle", "cores": 1, "value": kk / cs, "unit": "ordered surfels/s",
                             "sample": "oracle/bs_oracle.c oracle_sample32 (plain O(n) distance update per pick, "
                                       "1 thread): the first %d picks of the same run, %.1f s" % (kk, cs)}
    return rec


def bench_capture(bs, torch, np, cpu=True):
    """Sec. 3.1 + 3.2/3.3 as one preprocessing pipeline on the device: the
    visible surface of a CAD-like part (200 boxes / cylinders, seed 2) from
    the eight bounding-box corners at 1024^2 pixels per view, then the exact
    ordering of the captured candidates to k = 262,144 (or all of them)."""
    import synth
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    prims = synth.cad_primitives(2, count=200)
    kind = prims.kind.numpy().astype(np.int32)
    center = prims.center.numpy().astype(np.float32)
    rot = prims.rot.numpy().astype(np.float32)
    prm = prims.prm.numpy().astype(np.float32)
    rgb = prims.color.numpy().astype(np.uint8)
    ext = np.where(kind[:, None] == 0, prm[:, :1].repeat(3, 1),
                   np.where(kind[:, None] == 1, prm, np.stack([prm[:, 0], prm[:, 0], prm[:, 1]], 1)))
    half = (np.abs(rot.astype(np.float64)) @ ext.astype(np.float64)[:, :, None])[:, :, 0]
    lo = (center - half).min(0).astype(np.float32)
    hi = (center + half).max(0).astype(np.float32)
    rec = bs.primitive_records(kind, center, rot, prm, rgb)
    R = 1024
    pts, nrm, col = bs.capture(rec, lo, hi, R)  # warm-up
    stream = torch.cuda.current_stream()
    lib = bs.load()
    raw = torch.from_numpy(rec.view(np.uint8).copy()).cuda()
    cap = 8 * R * R
    P = torch.empty((cap, 3), dtype=torch.float32, device="cuda")
    N = torch.empty((cap, 3), dtype=torch.float32, device="cuda")
    C = torch.empty((cap, 3), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(int(lib.bs_capture_workspace_size(R)), dtype=torch.uint8, device="cuda")
    import ctypes
    reps = 10
    b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.record(stream)
    for _ in range(reps):
        rc = lib.bs_capture(ctypes.c_void_p(raw.data_ptr()), int(rec.shape[0]), lo.ctypes.data_as(ctypes.c_void_p),
                            hi.ctypes.data_as(ctypes.c_void_p), R, ctypes.c_void_p(P.data_ptr()),
                            ctypes.c_void_p(N.data_ptr()), ctypes.c_void_p(C.data_ptr()),
                            ctypes.c_void_p(cnt.data_ptr()), ctypes.c_void_p(ws.data_ptr()), int(ws.numel()),
                            ctypes.c_void_p(stream.cuda_stream))
        assert rc == 0
    e.record(stream)
    torch.cuda.synchronize()
    cap_s = b.elapsed_time(e) / 1e3 / reps
    n = int(cnt.cpu()[0])
    k = min(262144, n)
    cand = P[:n]
    o, r = bs.order(cand, k, seed=2)  # warm-up
    b2, e2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b2.record(stream)
    o, r = bs.order(cand, k, seed=2, check=False)
    e2.record(stream)
    torch.cuda.synchronize()
    ord_s = b2.elapsed_time(e2) / 1e3
    tests = 8 * R * R * int(rec.shape[0])
    rec_out = {"workload": "cad_primitives seed 2 (200 boxes / cylinders), 8 views x 1024^2 pixels",
               "candidates": n, "capture_seconds": cap_s, "ray_primitive_tests_per_s": tests / cap_s,
               "gbuffer_bytes": 8 * R * R * 32, "order_k": k, "order_seconds": ord_s,
               "pipeline_seconds": cap_s + ord_s,
               "note": "capture kernel (ray cast, G-buffer) + scan + scatter, then bs_order on the captured "
                       "candidates on the device: the paper's render-to-texture, initial-set and sampling stages "
                       "without a host round trip"}
    if cpu:
        import oracle
        Rs = 256
        t0 = time.perf_counter()
        ep, _, _ = oracle.capture32(kind, center, rot, prm, rgb, lo, hi, Rs)
        cs = time.perf_counter() - t0
        gp, _, _ = bs.capture(rec, lo, hi, Rs)
        rec_out["matches_oracle_at_256"] = bool(np.array_equal(gp.cpu().numpy().view(np.uint32),
                                                               ep.view(np.uint32)))
        rec_out["cpu_oracle"] = {"kind": "oracle", "cores": 1, "seconds": cs,
                                 "ray_primitive_tests_per_s": 8 * Rs * Rs * int(rec.shape[0]) / cs,
                                 "sample": "oracle_capture32 (1 thread) at 256^2 pixels per view"}
    return rec_out


def bench_full_scan(bs, torch, pts, k):
    tune = bs.tuning(kernel=bs.KERNEL_COOP, block=1024, per_thread=16)
    n = int(pts.shape[0])
    start = bs.start_index(SEED_MAIN, n)
    _, lat, _ = ordering_kernel_seconds(bs, pts, k, start, tune)
    stream = torch.cuda.current_stream()
    b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.record(stream)
    e.record(stream)
    o, _, _ = bs.order_profile(pts, k, start=start, tune=tune, stream=stream, ticks=False, events=(b, e))
    torch.cuda.synchronize()
    secs = b.elapsed_time(e) / 1e3
    live = (k - 1) * n - (k * (k - 1)) // 2
    abytes = 16 * live
    return {"kernel": "resident cooperative full scan (256 workgroups x 16K candidates in VGPRs)",
            "seconds": secs, "ordered_surfels_per_s": k / secs, "per_step_p50_us": lat["p50_us"],
            "picks_per_round": lat["picks_per_round"],
            "algorithmic_bytes": abytes, "achieved_GBs": abytes / secs / 1e9,
            "frac_of_hbm_peak": abytes / secs / 1e9 / HBM_PEAK_GBS}, o


def bench_batched(bs, torch, np, cpu=True):
    import synth
    dev = torch.device("cuda:0")
    m = 1000
    sizes = synth.log_uniform_sizes(m, 2048, 2097152, seed=3)
    ks = [s // 4 for s in sizes]
    seeds = [3 * 1000003 + j for j in range(m)]
    t0 = time.time()
    pts, offs = synth.cad_parts_batch(sizes, seed=3, count=200, device=dev)
    torch.cuda.synchronize()
    log("generated batch: %d objects, %d candidates in %.1fs" % (m, pts.shape[0], time.time() - t0))
    t0 = time.time()
    tune = bs.batch_autotune(pts, offs, ks, seeds)
    log("batch autotune: cell target %g, %d wide workgroups in %.1fs" % (tune.cell_points, tune.groups,
                                                                         time.time() - t0))
    plan = bs.BatchPlan(offs, ks, seeds, tune=tune)
    out_o = torch.empty(plan.total_k, dtype=torch.int32, device=dev)
    out_r = torch.empty(plan.total_k, dtype=torch.float32, device=dev)
    plan.execute(pts, out_o, out_r)
    torch.cuda.synchronize()
    reps = 2
    t = time.perf_counter()
    for _ in range(reps):
        plan.execute(pts, out_o, out_r)
    torch.cuda.synchronize()
    batch_s = (time.perf_counter() - t) / reps
    log("batched: %.3f s for sum k = %d" % (batch_s, plan.total_k))
    # the same objects through the paper's randomized sampler (one persistent launch)
    so, sr, sc = plan.execute_sample(pts)
    torch.cuda.synchronize()
    t = time.perf_counter()
    so, sr, sc = plan.execute_sample(pts)
    torch.cuda.synchronize()
    sample_s = time.perf_counter() - t
    log("batched sampler: %.3f s for sum k = %d" % (sample_s, int(sc.sum())))
    sampler_rec = {"seconds": sample_s, "ordered_surfels_per_s": int(sc.sum()) / sample_s,
                   "params": {"sample_size": 200, "growth_rounds": 500, "vicinity": 0.0},
                   "kernel": "sample_batch_kernel: objects largest k first, the longest chains on 1024-thread workgroups, the others on 256-thread ones"}
    del so, sr, sc
    # plain loop: one ordering launch per object, sampled across the size range
    order_idx = sorted(range(m), key=lambda j: sizes[j])
    sample = order_idx[:: max(1, m // 24)]
    sk = 0
    torch.cuda.synchronize()
    t = time.perf_counter()
    for j in sample:
        a, b = offs[j], offs[j + 1]
        bs.order(pts[a:b], ks[j], seed=seeds[j], check=False)
        sk += ks[j]
    torch.cuda.synchronize()
    sample_s = time.perf_counter() - t
    plain_rate = sk / sample_s
    plain_est_s = plan.total_k / plain_rate
    # spot check: three objects equal ordering them alone
    same = True
    for j in (order_idx[0], order_idx[m // 2], order_idx[-1]):
        a, b = offs[j], offs[j + 1]
        so, _ = bs.order(pts[a:b], ks[j], seed=seeds[j])
        oa, ob = plan.out_offsets[j], plan.out_offsets[j + 1]
        same &= bool(torch.equal(so, out_o[oa:ob]))
    plan.close()
    cpu_rec = cpu_oracle_objects(pts, offs, ks, seeds, order_idx, plan.total_k, batch_s) if cpu else None
    return {"objects": m, "candidates": int(pts.shape[0]), "sum_k": int(plan.total_k),
            "cell_target": float(tune.cell_points), "wide_workgroups": int(tune.groups),
            "seconds": batch_s, "ordered_surfels_per_s": plan.total_k / batch_s,
            "plain_loop_ordered_surfels_per_s": plain_rate,
            "plain_loop_sample": "%d objects spread over the size range, %d picks, %.1f s" % (len(sample), sk, sample_s),
            "plain_loop_estimated_seconds": plain_est_s, "speedup_vs_plain": plain_est_s / batch_s,
            "largest_object_k": max(ks), "spot_check_equal_alone": same, "cpu_oracle": cpu_rec,
            "randomized_sampler": sampler_rec}


def bench_scene(bs, torch, np, cpu=True):
    """Heterogeneous scene: 10,000 objects (thin sheets, tori, small-box
    clusters), 1.5e9 candidates, k_j = 12% of n_j, one batched launch."""
    import synth
    dev = torch.device("cuda:0")
    m = 10000
    sizes = synth.scene_sizes(m, 1_500_000_000, seed=5)
    ks = [int(0.12 * s) for s in sizes]
    seeds = [5 * 1000003 + j for j in range(m)]
    t0 = time.time()
    pts, offs = synth.scene_batch(sizes, seed=5, device=dev)
    torch.cuda.synchronize()
    log("generated scene: %d objects, %d candidates in %.1fs" % (m, pts.shape[0], time.time() - t0))
    t0 = time.time()
    tune = bs.batch_autotune(pts, offs, ks, seeds)
    log("batch autotune: cell target %g in %.1fs" % (tune.cell_points, time.time() - t0))
    plan = bs.BatchPlan(offs, ks, seeds, tune=tune)
    out_o = torch.empty(plan.total_k, dtype=torch.int32, device=dev)
    out_r = torch.empty(plan.total_k, dtype=torch.float32, device=dev)
    plan.execute(pts, out_o, out_r)
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan.execute(pts, out_o, out_r)
    torch.cuda.synchronize()
    batch_s = time.perf_counter() - t
    log("scene batched: %.3f s for sum k = %d" % (batch_s, plan.total_k))
    order_idx = sorted(range(m), key=lambda j: sizes[j])
    sample = order_idx[:: max(1, m // 20)]
    sk = 0
    torch.cuda.synchronize()
    t = time.perf_counter()
    for j in sample:
        bs.order(pts[offs[j]:offs[j + 1]], ks[j], seed=seeds[j], check=False)
        sk += ks[j]
    torch.cuda.synchronize()
    sample_s = time.perf_counter() - t
    plain_rate = sk / sample_s
    same = True
    for j in (order_idx[0], order_idx[m // 2], order_idx[-1]):
        so, _ = bs.order(pts[offs[j]:offs[j + 1]], ks[j], seed=seeds[j])
        oa, ob = plan.out_offsets[j], plan.out_offsets[j + 1]
        same &= bool(torch.equal(so, out_o[oa:ob]))
    plan.close()
    plan._ws = None  # the scene plan's 99 GB workspace, before the hierarchy takes its own
    torch.cuda.empty_cache()
    hier = bench_hierarchy(bs, torch, np, pts, offs, sizes, ks, seeds)
    res = {"objects": m, "candidates": int(pts.shape[0]), "sum_k": int(plan.total_k),
           "workspace_bytes": int(plan.workspace_bytes), "cell_target": float(tune.cell_points),
           "seconds": batch_s, "ordered_surfels_per_s": plan.total_k / batch_s,
           "plain_loop_ordered_surfels_per_s": plain_rate,
           "plain_loop_sample": "%d objects spread over the size range, %d picks, %.1f s" % (len(sample), sk, sample_s),
           "speedup_vs_plain": (plan.total_k / plain_rate) / batch_s, "spot_check_equal_alone": same,
           "hierarchy": hier}
    res["cpu_oracle"] = cpu_oracle_objects(pts, offs, ks, seeds, order_idx, res["sum_k"], batch_s) if cpu else None
    return res


def bench_hierarchy(bs, torch, np, pts, offs, sizes, ks, seeds):
    """Sec. 3.4 bottom-up generation over the scene: its 10,000 objects are
    leaves placed in 20 clusters of 500 (an 8^3 lattice of 2.5-unit spacing
    per cluster, clusters on a 3^3 lattice 30 units apart); each cluster node
    orders the surfels its objects chose, and the root the clusters' surfels.
    Leaf k = 12% of n; an inner node keeps min(200,000, half its candidates)
    (the paper's bound for a subtree, with its children's surfels standing in
    for its triangles)."""
    m = len(sizes)
    per = 500
    nc = (m + per - 1) // per
    j = torch.arange(m, device=pts.device)
    cl = j // per
    w = j % per
    ctr = torch.stack([(cl % 3), (cl // 3) % 3, cl // 9], 1).double() * 30.0
    loc = torch.stack([w % 8, (w // 8) % 8, w // 64], 1).double() * 2.5
    shift = (ctr + loc).float()
    counts = torch.tensor([offs[i + 1] - offs[i] for i in range(m)], device=pts.device)
    pts += torch.repeat_interleave(shift, counts, 0)
    parents = [m + i // per for i in range(m)] + [m + nc] * nc + [-1]
    leaf_offs = list(offs) + [offs[-1]] * (nc + 1)
    kk = list(ks)
    for c in range(nc):
        kk.append(min(200000, sum(ks[c * per:(c + 1) * per]) // 2))
    kk.append(min(200000, sum(kk[m:m + nc]) // 2))
    sd = list(seeds) + [77 + c for c in range(nc)] + [99]
    plan = bs.HierPlan(parents, leaf_offs, kk, sd)
    o, r, s = plan.execute(pts)
    torch.cuda.synchronize()
    t = time.perf_counter()
    o, r, s = plan.execute(pts)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t
    root = plan.out_offsets[-2]
    res = {"nodes": len(parents), "levels": 3, "leaves": m, "cluster_nodes": nc,
           "sum_k": int(plan.total_k), "cluster_k": kk[m], "root_k": kk[-1], "seconds": secs,
           "ordered_surfels_per_s": plan.total_k / secs, "workspace_bytes": int(plan.workspace_bytes),
           "root_sources_valid": bool((s[root:] >= 0).all())}
    plan.close()
    pts -= torch.repeat_interleave(shift, counts, 0)
    log("hierarchy: %d nodes, sum k %d in %.3f s" % (len(parents), plan.total_k, secs))
    return res


def bench_served(bs, torch, np):
    import synth
    dev = torch.device("cuda:0")
    pool_m = 64
    sizes = synth.log_uniform_sizes(pool_m, 10000, 4000000, seed=4)
    pts, offs = synth.cad_parts_batch(sizes, seed=4, count=200, device=dev)
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    nreq = 2000
    arrivals = synth.poisson_arrivals(nreq, 200.0, seed=4)
    picks = rng.integers(0, pool_m, nreq)
    seeds = rng.integers(0, 2**62, nreq)
    ks = [sizes[p] // 8 for p in picks]
    total_k = int(sum(ks))
    out_o = torch.empty(total_k, dtype=torch.int32, device=dev)
    out_r = torch.empty(total_k, dtype=torch.float32, device=dev)
    views = [pts[offs[p]:offs[p + 1]] for p in range(pool_m)]
    # warm-up server (loads kernels)
    warm = bs.Server(hbm_budget_bytes=80_000_000_000)
    for i in range(8):
        p = int(picks[i])
        warm.submit(views[p], min(ks[i], 1000), int(seeds[i]), out_o[:1000], out_r[:1000])
    warm.drain()
    warm.close()
    srv = bs.Server(hbm_budget_bytes=80_000_000_000, max_jobs_per_batch=256, poll_us=20)
    off = 0
    t0 = time.perf_counter()
    for i in range(nreq):
        now = time.perf_counter() - t0
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        p = int(picks[i])
        srv.submit(views[p], ks[i], int(seeds[i]), out_o[off:off + ks[i]], out_r[off:off + ks[i]])
        off += ks[i]
        if (i + 1) % 500 == 0:
            st = srv.stats()
            log("served: %d submitted, %d completed" % (i + 1, st["completed"]))
    srv.drain()
    st = srv.stats()
    srv.close()
    log("served: p50 %.1f ms p99 %.1f ms, %.3g surfels/s, %d worker launches, %d stall stops"
        % (st["p50_us"] / 1e3, st["p99_us"] / 1e3, st["surfels_per_s"], st["worker_launches"], st["stall_stops"]))
    # capacity: the same requests all queued at once (the offered rate above
    # caps the served rate, so this is what compares with the plain loop)
    sat = bs.Server(hbm_budget_bytes=80_000_000_000, max_jobs_per_batch=256, poll_us=20)
    off = 0
    for i in range(nreq):
        p = int(picks[i])
        sat.submit(views[p], ks[i], int(seeds[i]), out_o[off:off + ks[i]], out_r[off:off + ks[i]])
        off += ks[i]
    sat.drain()
    st2 = sat.stats()
    sat.close()
    log("served, saturated: %.3g surfels/s in %.2f s" % (st2["surfels_per_s"], st2["elapsed_s"]))
    # plain loop: one ordering launch per request, back to back, sampled
    sample = list(range(0, nreq, nreq // 20))[:20]
    sk = 0
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in sample:
        bs.order(views[int(picks[i])], ks[i], seed=int(seeds[i]), check=False)
        sk += ks[i]
    torch.cuda.synchronize()
    plain_rate = sk / (time.perf_counter() - t)
    offered = total_k / arrivals[-1]
    return {"requests": nreq, "rate_hz": 200.0, "offered_surfels_per_s": offered,
            "p50_latency_ms": st["p50_us"] / 1e3, "p99_latency_ms": st["p99_us"] / 1e3,
            "max_latency_ms": st["max_us"] / 1e3, "served_surfels_per_s": st["surfels_per_s"],
            "elapsed_s": st["elapsed_s"], "batches": st["batches"], "hbm_peak_bytes": st["hbm_peak"],
            "worker_launches": st["worker_launches"], "stall_stops": st["stall_stops"],
            "plain_loop_ordered_surfels_per_s": plain_rate,
            "speedup_vs_plain": st["surfels_per_s"] / plain_rate,
            "speedup_bound_by_offered_load": offered / plain_rate,
            "saturated": {"surfels_per_s": st2["surfels_per_s"], "elapsed_s": st2["elapsed_s"],
                          "batches": st2["batches"], "hbm_peak_bytes": st2["hbm_peak"],
                          "worker_launches": st2["worker_launches"], "stall_stops": st2["stall_stops"],
                          "speedup_vs_plain": st2["surfels_per_s"] / plain_rate,
                          "note": "the same 2,000 requests queued at once: the serving path's capacity"},
            "plain_loop_sample": "%d requests back to back" % len(sample)}


def cpu_baseline(points_host, k, start):
    """The exact CPU oracle on the same points (bounded: about 10-20 s)."""
    import oracle
    t0 = time.perf_counter()
    order, radius, st = oracle.greedy32_grid(points_host, k, start, stats=True)
    dt = time.perf_counter() - t0
    return {"value": k / dt, "unit": "ordered surfels/s", "cores": 1, "kind": "oracle",
            "sample": "exact grid-accelerated oracle (oracle/bs_oracle.c, 1 thread) on the full "
                      "workload n=%d k=%d, %.1f s" % (points_host.shape[0], k, dt)}, order, st["n_ball"]


def cpu_oracle_objects(pts, offs, ks, seeds, order_idx, sum_k_total, gpu_seconds,
                       max_k=300_000, budget_k=3_000_000, count=24):
    """The exact CPU oracle on a bounded sample of a batch's objects (those
    with k <= max_k, spread over their size range, at most budget_k picks),
    object-parallel on a thread pool over the host's cores (the oracle's C
    calls release the GIL).  The single-thread rate comes from the objects'
    own durations inside the pool, so it includes the contention of the
    other threads."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    eligible = [j for j in order_idx if 0 < ks[j] <= max_k]
    sample, sk = [], 0
    for j in eligible[:: max(1, len(eligible) // count)]:
        if sk + ks[j] > budget_k:
            break
        sample.append(j)
        sk += ks[j]
    host = [pts[offs[j]:offs[j + 1]].cpu().numpy() for j in sample]
    # one GPU's share of the host: 16 threads at most, whatever the machine shows
    visible = len(os.sched_getaffinity(0))
    cores = min(visible, 16)

    def one(i):
        j = sample[i]
        t0 = time.perf_counter()
        oracle.greedy32_grid(host[i], ks[j], oracle.start_index(seeds[j], host[i].shape[0]))
        return time.perf_counter() - t0

    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        per = list(ex.map(one, range(len(sample))))
    wall = time.perf_counter() - t0
    par_rate = sk / wall
    one_rate = sk / sum(per)
    log("cpu oracle: %d objects, %d picks, %.1f s on %d threads" % (len(sample), sk, wall, cores))
    return {"kind": "oracle", "cores": cores, "host_cpus_visible": visible,
            "object_parallel_ordered_surfels_per_s": par_rate,
            "single_thread_ordered_surfels_per_s": one_rate,
            "estimated_seconds_object_parallel": sum_k_total / par_rate,
            "gpu_speedup_vs_object_parallel": (sum_k_total / par_rate) / gpu_seconds,
            "sample": "%d objects with n = %d..%d (k <= %d), %d picks, %.1f s wall on %d threads"
                      % (len(sample), host[0].shape[0], host[-1].shape[0], max_k, sk, wall, cores)}


def profile_leg(which, bs, torch, np):
    """The workload of the batch and serving profiles, alone on the device:
    one execute of the 1,000-part batch (default tuning), or the serving
    stream's 2,000 requests queued at once.  Prints one JSON line."""
    import synth
    dev = torch.device("cuda:0")
    if which == "batch":
        m = 1000
        sizes = synth.log_uniform_sizes(m, 2048, 2097152, seed=3)
        ks = [s // 4 for s in sizes]
        seeds = [3 * 1000003 + j for j in range(m)]
        pts, offs = synth.cad_parts_batch(sizes, seed=3, count=200, device=dev)
        plan = bs.BatchPlan(offs, ks, seeds)
        out_o = torch.empty(plan.total_k, dtype=torch.int32, device=dev)
        out_r = torch.empty(plan.total_k, dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        plan.execute(pts, out_o, out_r)
        torch.cuda.synchronize()
        rec = {"profile_leg": "batch", "objects": m, "candidates": int(pts.shape[0]), "sum_k": int(plan.total_k),
               "seconds": time.perf_counter() - t}
        plan.close()
    else:
        pool_m = 64
        sizes = synth.log_uniform_sizes(pool_m, 10000, 4000000, seed=4)
        pts, offs = synth.cad_parts_batch(sizes, seed=4, count=200, device=dev)
        rng = np.random.default_rng(4)
        nreq = 2000
        picks = rng.integers(0, pool_m, nreq)
        seeds = rng.integers(0, 2**62, nreq)
        ks = [sizes[p] // 8 for p in picks]
        out_o = torch.empty(int(sum(ks)), dtype=torch.int32, device=dev)
        out_r = torch.empty(int(sum(ks)), dtype=torch.float32, device=dev)
        views = [pts[offs[p]:offs[p + 1]] for p in range(pool_m)]
        torch.cuda.synchronize()
        srv = bs.Server(hbm_budget_bytes=80_000_000_000, max_jobs_per_batch=256, poll_us=20)
        off = 0
        for i in range(nreq):
            p = int(picks[i])
            srv.submit(views[p], ks[i], int(seeds[i]), out_o[off:off + ks[i]], out_r[off:off + ks[i]])
            off += ks[i]
        srv.drain()
        st = srv.stats()
        srv.close()
        rec = {"profile_leg": "serve", "requests": nreq, "sum_k": int(sum(ks)), "seconds": st["elapsed_s"],
               "batches": st["batches"], "worker_launches": st["worker_launches"],
               "stall_stops": st["stall_stops"]}
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-full-scan", action="store_true")
    ap.add_argument("--no-config1", action="store_true")
    ap.add_argument("--no-sampler", action="store_true")
    ap.add_argument("--no-capture", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-scene", action="store_true")
    ap.add_argument("--plan", choices=("auto", "grid"), default="auto",
                    help="main leg: the automatic plan, or the grid kernel (16 picks per round, leading scan)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the automatic kernel choice without timing candidates first")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run two plain device-to-device copies of BYTES bytes (scales the "
                         "FETCH_SIZE / WRITE_SIZE counters to bytes) and exit")
    ap.add_argument("--profile-leg", choices=("batch", "serve"), default=None,
                    help="only run the batched (one execute) or the saturated serving workload once, for "
                         "a profiler, and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: every object is ordered on a single MI355X and this build has "
              "no multi-GPU path; --gpus %d is not supported (DESIGN.md describes how it would shard)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1904_08225_amd as bs

    torch.cuda.set_device(0)
    if args.copy_calibration > 0:
        src = torch.empty(args.copy_calibration, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": args.copy_calibration, "copies": 2}), flush=True)
        return
    if args.profile_leg:
        profile_leg(args.profile_leg, bs, torch, np)
        return
    pts, surf, out_o, ms, ev_ms, kern_s, lat, kernel, tuned, lead = bench_main(args, bs, torch, np)
    n, k = N_MAIN, K_MAIN
    rec = {
        "metric": "ordered surfels/sec (exact greedy blue-noise ordering)",
        "value": k / (ms / 1000.0),
        "unit": "ordered surfels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded union-boundary samples of 200 random boxes/cylinders)",
        "config": {"workload": "cad_part n=4,194,304 k=262,144 (union of 200 boxes/cylinders)",
                   "n": n, "k": k, "seed": SEED_MAIN,
                   "kernel": ("cooperative scan over all CUs, candidates in VGPRs in Morton order, "
                              "several exact picks per step" if kernel == 2 and tuned.picks > 1 else
                              {1: "resident workgroup", 2: "cooperative full scan",
                               3: "grid-pruned, several exact picks per round"}.get(kernel, str(kernel))),
                   "event_ms_per_step": ev_ms,
                   "tuning": {"kernel": int(tuned.kernel), "block": int(tuned.block),
                              "per_thread": int(tuned.per_thread), "groups": int(tuned.groups),
                              "cell_points": float(tuned.cell_points), "picks": int(tuned.picks),
                              "lead_picks": lead,
                              "source": "grid kernel asked for (--plan grid)" if args.plan == "grid" else
                              "library defaults (no autotuning)" if args.no_autotune else
                              "library autotuner (bs_autotune), run before the timed steps"}},
        "latency": {"per_round_p50_us": lat["p50_us"], "per_round_p99_us": lat["p99_us"],
                    "per_round_mean_us": lat["mean_us"], "rounds": lat["rounds"],
                    "picks_per_round": lat["picks_per_round"], "mean_us_per_pick": lat["mean_us_per_pick"],
                    "lead_step_p50_us": lat.get("lead_step_p50_us"),
                    "lead_step_p99_us": lat.get("lead_step_p99_us"),
                    "source": "device wall clock at each pick's emission: steps of the ordering kernel "
                              "(a step emits several exact picks) and, for the grid plan, apart, the "
                              "steps of its leading full scan"},
    }
    host = pts.cpu().numpy()
    n_ball = None
    if not args.no_cpu_baseline:
        cb, eo, n_ball = cpu_baseline(host, k, bs.start_index(SEED_MAIN, n))
        rec["cpu_baseline"] = cb
        rec["config"]["matches_oracle"] = bool(np.array_equal(out_o.cpu().numpy(), eo))
        log("cpu baseline: " + cb["sample"])
    if n_ball is not None:
        several = kernel == bs.KERNEL_COOP and tuned.picks > 1
        if several:
            kname = "scan_mp_kernel<%d, %d, %d> x %d workgroups" % (
                tuned.block, tuned.per_thread, 256 if tuned.picks > 128 else 128, tuned.groups)
            which = "scan_mp"
        else:
            kname = {3: "grid_multi_kernel<%d,...>" % (tuned.block or 1024)}.get(kernel, "kernel %d" % kernel)
            which = "grid"
        # the ordering kernel makes the updates of picks lead-1 .. k-2 (a
        # leading scan of the grid plan those of picks 0 .. lead-2)
        abytes = 16 * int(n_ball[max(lead - 1, 0):].sum())
        achieved = abytes / kern_s / 1e9
        plain = 16 * sum(n - j - 1 for j in range(max(lead - 1, 0), k - 1))
        rec["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(which),
                           "kernel": kname, "algorithmic_bytes": abytes, "kernel_seconds": kern_s,
                           "plain_definition_bytes": plain,
                           "plain_definition_GBs": plain / kern_s / 1e9,
                           "traffic_source": "rocprofv3 FETCH_SIZE and WRITE_SIZE per launch, scaled by a "
                                             "plain copy of known size (%s)"
                                             % os.path.relpath(TRAFFIC_FILES[which], ROOT),
                           "kernel_time_source": "HIP events recorded on the launch stream around the "
                                                 "ordering kernel, mean over the timed steps",
                           "note": "16 B per live candidate inside the covering-radius ball per step "
                                   "(pruned accounting); the step chain is latency-bound (one exchange "
                                   "across all CUs per step).  plain_definition: 16 B per live candidate "
                                   "per step, the work of the method as defined, which register residency "
                                   "and ball pruning let the kernel exceed the HBM peak on"}
        if lead:
            live = sum(n - j - 1 for j in range(lead - 1))
            ls = lat["lead_seconds"]
            rec["lead_scan"] = {"kernel": "scan_kernel<1024,%d,true> x %d workgroups" % (tuned.per_thread,
                                                                                       tuned.groups),
                                "picks": lead, "seconds": ls, "algorithmic_bytes": 16 * live,
                                "achieved_GBs": 16 * live / ls / 1e9,
                                "frac_of_hbm_peak": 16 * live / ls / 1e9 / HBM_PEAK_GBS,
                                "time_source": "device wall clock from pick 0 to the scan's last pick"}
    if not args.no_config1:
        rec["config1"] = bench_config1(bs, torch, np, cpu=not args.no_cpu_baseline)
        log("config1: %.2f ms per ordering of sphere_and_box 16,384 (k = n), step p50 %.2f us p99 %.2f us"
            % (rec["config1"]["ms_per_ordering"], rec["config1"]["per_step_p50_us"],
               rec["config1"]["per_step_p99_us"]))
    rec["emit"] = bench_emit(bs, torch, surf, pts, out_o)
    log("emit: %.1f us for %d records (%.0f GB/s algorithmic); r_m in %.1f us"
        % (rec["emit"]["seconds"] * 1e6, k, rec["emit"]["achieved_GBs"], rec["emit"]["median_nn_seconds"] * 1e6))
    if not args.no_capture:
        rec["capture"] = bench_capture(bs, torch, np, cpu=not args.no_cpu_baseline)
        log("capture: %d candidates in %.2f ms, ordered to %d in %.1f ms" % (
            rec["capture"]["candidates"], rec["capture"]["capture_seconds"] * 1e3, rec["capture"]["order_k"],
            rec["capture"]["order_seconds"] * 1e3))
    if not args.no_sampler:
        rec["sampler"] = bench_sampler(bs, torch, np, pts, out_o, cpu=not args.no_cpu_baseline)
        rec["sampler"]["exact_ordering_seconds"] = ms / 1e3
        log("sampler: %.3f s for %d picks (exact ordering %.1f ms)" % (rec["sampler"]["seconds"], k, ms))
    if not args.no_full_scan:
        fs, fo = bench_full_scan(bs, torch, pts, k)
        fs["matches_ordering_kernel"] = bool(torch.equal(fo, out_o))
        rec["full_scan"] = fs
        log("full scan: %.2f s, %.0f GB/s algorithmic" % (fs["seconds"], fs["achieved_GBs"]))
    del surf, pts
    torch.cuda.empty_cache()
    if not args.no_batch:
        rec["batched"] = bench_batched(bs, torch, np, cpu=not args.no_cpu_baseline)
        torch.cuda.empty_cache()
    if not args.no_scene:
        rec["scene_batched"] = bench_scene(bs, torch, np, cpu=not args.no_cpu_baseline)
        torch.cuda.empty_cache()
    if not args.no_serve:
        rec["served"] = bench_served(bs, torch, np)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
