"""Parity at the benchmark's full sizes, in the configuration bench.py times,
on sampled outputs the oracle can compute one by one: the 1,000-part batch
(2.95e8 candidates) and the heterogeneous scene (10,000 objects, 1.5e9
candidates) with their autotuned cell occupancy, and a served Poisson stream.
The largest object of each batch is checked by invariants that hold at any
size (radii non-increasing, the prefix an r-net for a sample of points)."""
import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_scan import assert_parity

pytestmark = pytest.mark.gpu


def _check_sampled(hip, pts, offs, ks, seeds, plan, o, r, label):
    m = len(ks)
    sizes = [offs[j + 1] - offs[j] for j in range(m)]
    by_size = sorted(range(m), key=lambda j: sizes[j])
    oo = o.cpu().numpy()
    rr = r.cpu().numpy()
    # four objects across the size range, exactly against the oracle
    for q in (0.0, 0.25, 0.5, 0.7):
        j = by_size[int(q * (m - 1))]
        P = pts[offs[j]:offs[j + 1]].cpu().numpy()
        a, b = plan.out_offsets[j], plan.out_offsets[j + 1]
        eo, er = oracle.greedy32_grid(P, ks[j], oracle.start_index(seeds[j], P.shape[0]))
        assert_parity(oo[a:b], rr[a:b], eo, er, "%s object %d (n=%d k=%d)" % (label, j, P.shape[0], ks[j]))
    # the largest: invariants at any size
    j = by_size[-1]
    a, b = plan.out_offsets[j], plan.out_offsets[j + 1]
    oj, rj = oo[a:b], rr[a:b]
    assert len(np.unique(oj)) == ks[j] and oj.min() >= 0 and oj.max() < sizes[j]
    assert np.all(rj[2:] <= rj[1:-1]), "radii must not increase"
    P = pts[offs[j]:offs[j + 1]].cpu().numpy().astype(np.float64)
    t = ks[j] // 2
    pref = P[oj[:t]]
    rng = np.random.default_rng(5)
    probe = P[rng.choice(sizes[j], 64, replace=False)]
    d = np.array([np.sqrt(((pref - q) ** 2).sum(-1)).min() for q in probe])
    # covering: every candidate lies within (about) the covering radius of the t-prefix
    assert np.all(d <= float(rj[t]) * (1 + 1e-5) + 1e-30), "prefix is not a covering at its radius"


def test_full_batch_1000_parts(hip):
    import torch
    m = 1000
    sizes = synth.log_uniform_sizes(m, 2048, 2097152, seed=3)
    ks = [s // 4 for s in sizes]
    seeds = [3 * 1000003 + j for j in range(m)]
    pts, offs = synth.cad_parts_batch(sizes, seed=3, count=200, device="cuda")
    tune = hip.batch_autotune(pts, offs, ks, seeds)
    plan = hip.BatchPlan(offs, ks, seeds, tune=tune)
    o, r = plan.execute(pts)
    torch.cuda.synchronize()
    _check_sampled(hip, pts, offs, ks, seeds, plan, o, r, "parts")
    plan.close()


def test_full_scene_10000_objects(hip):
    import torch
    m = 10000
    sizes = synth.scene_sizes(m, 1_500_000_000, seed=5)
    ks = [int(0.12 * s) for s in sizes]
    seeds = [5 * 1000003 + j for j in range(m)]
    pts, offs = synth.scene_batch(sizes, seed=5, device="cuda")
    tune = hip.batch_autotune(pts, offs, ks, seeds)
    plan = hip.BatchPlan(offs, ks, seeds, tune=tune)
    o, r = plan.execute(pts)
    torch.cuda.synchronize()
    _check_sampled(hip, pts, offs, ks, seeds, plan, o, r, "scene")
    plan.close()
    del pts, o, r
    torch.cuda.empty_cache()


def test_served_poisson_stream(hip):
    """A Poisson stream (200/s) of jobs n log-uniform 1e4..4e6, k = n/8, under
    an 80 GB budget: every sampled job equals ordering it alone, a few equal
    the oracle."""
    import time
    import torch
    pool_m = 16
    sizes = synth.log_uniform_sizes(pool_m, 10000, 4000000, seed=4)
    pts, offs = synth.cad_parts_batch(sizes, seed=4, count=200, device="cuda")
    views = [pts[offs[p]:offs[p + 1]] for p in range(pool_m)]
    rng = np.random.default_rng(4)
    nreq = 300
    arrivals = synth.poisson_arrivals(nreq, 200.0, seed=4)
    picks = rng.integers(0, pool_m, nreq)
    seeds = rng.integers(0, 2**62, nreq)
    srv = hip.Server(hbm_budget_bytes=80_000_000_000, max_jobs_per_batch=256, poll_us=20)
    jobs = []
    t0 = time.perf_counter()
    for i in range(nreq):
        now = time.perf_counter() - t0
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        p = int(picks[i])
        k = sizes[p] // 8
        oo = torch.empty(k, dtype=torch.int32, device="cuda")
        rr = torch.empty(k, dtype=torch.float32, device="cuda")
        jobs.append((srv.submit(views[p], k, int(seeds[i]), oo, rr), p, k, int(seeds[i]), oo, rr))
    srv.drain(300_000_000)
    st = srv.stats()
    srv.close()
    assert st["completed"] == nreq and st["p99_us"] >= st["p50_us"] > 0
    for idx in range(0, nreq, 15):
        t, p, k, seed, oo, rr = jobs[idx]
        ao, ar = hip.order(views[p], k, seed=seed)
        assert torch.equal(oo, ao) and torch.equal(rr.view(torch.int32), ar.view(torch.int32)), "job %d" % idx
    small = sorted(range(nreq), key=lambda i: sizes[jobs[i][1]])[:3]
    for idx in small:
        t, p, k, seed, oo, rr = jobs[idx]
        P = views[p].cpu().numpy()
        eo, er = oracle.greedy32_grid(P, k, oracle.start_index(seed, P.shape[0]))
        assert_parity(oo.cpu().numpy(), rr.cpu().numpy(), eo, er, "served job %d" % idx)
