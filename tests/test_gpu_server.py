"""Serving loop: each job's result equals ordering it alone (and the oracle),
whatever it was batched and overlapped with; admission respects the budget."""
import time

import numpy as np
import pytest

import oracle
import synth
from tests import cases
from tests.test_gpu_scan import assert_parity

pytestmark = pytest.mark.gpu


def _jobs(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        n = int(rng.integers(1, 20000)) if j % 4 else int(rng.integers(20000, 120000))
        if j % 9 == 8:
            n = int(rng.integers(1, 5))
        P = synth.cad_part(n, seed=700 + j, count=12).points.numpy() if j % 3 == 0 else \
            cases.ADVERSARIAL[sorted(cases.ADVERSARIAL)[j % 7]](n, 800 + j)
        k = n if j % 5 == 0 else int(rng.integers(0, n + 1))
        out.append((np.asarray(P, dtype=np.float32), k, int(rng.integers(0, 2**63))))
    return out


def test_server_results_equal_alone(hip):
    import torch
    jobs = _jobs(3, 40)
    srv = hip.Server(hbm_budget_bytes=8 << 30, max_inflight=4, max_jobs_per_batch=8)
    pending = []
    for j, (P, k, seed) in enumerate(jobs):
        pts = torch.from_numpy(P).cuda()
        oo = torch.full((max(k, 1),), -7, dtype=torch.int32, device="cuda")
        rr = torch.zeros((max(k, 1),), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t = srv.submit(pts, k, seed, oo, rr)
        pending.append((t, pts, oo, rr, P, k, seed))
        if j % 6 == 5:
            time.sleep(0.002)  # arrivals while earlier jobs run
    for t, pts, oo, rr, P, k, seed in pending:
        srv.wait(t, timeout_us=60_000_000)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(jobs) and st["queued"] == 0
    assert st["batches"] >= 2
    for t, pts, oo, rr, P, k, seed in pending:
        if k == 0:
            continue
        o = oo.cpu().numpy()[:k]
        r = rr.cpu().numpy()[:k]
        st0 = oracle.start_index(seed, P.shape[0])
        eo, er = oracle.greedy32_grid(P, k, st0)
        assert_parity(o, r, eo, er, "served job n=%d k=%d" % (P.shape[0], k))
        ao, ar = hip.order(pts, k, seed=seed)
        assert_parity(o, r, ao.cpu().numpy(), ar.cpu().numpy(), "served vs alone")


def test_server_budget_admission_and_rejection(hip):
    import torch
    # room for about one 50k-candidate job at a time
    srv = hip.Server(hbm_budget_bytes=12 << 20, max_inflight=3, max_jobs_per_batch=4)
    P = synth.cad_part(50000, seed=5, count=20).points.numpy()
    pts = torch.from_numpy(P).cuda()
    outs = []
    for s in range(6):
        oo = torch.empty(2000, dtype=torch.int32, device="cuda")
        outs.append((srv.submit(pts, 2000, s, oo), oo, s))
    big = torch.zeros((300000, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(hip.BSError) as ei:
        srv.submit(big, 10, 0, torch.empty(10, dtype=torch.int32, device="cuda"))
    assert ei.value.code == hip.BS_ERR_OVER_BUDGET
    srv.drain(60_000_000)
    st = srv.stats()
    assert st["completed"] == 6 and st["rejected"] == 1
    assert st["hbm_peak"] <= 12 << 20
    for t, oo, s in outs:
        eo, _ = oracle.greedy32_grid(P, 2000, oracle.start_index(s, 50000))
        assert np.array_equal(oo.cpu().numpy(), eo)
    srv.close()


def test_server_later_job_overlaps_earlier(hip):
    """A job admitted while a long one is on the device finishes first (it
    only waits for a free worker), and both equal the oracle."""
    import torch
    srv = hip.Server(hbm_budget_bytes=8 << 30, max_jobs_per_batch=8)
    big = synth.cad_part(1_000_000, seed=12, count=60, device="cuda").points.contiguous()
    kb = 200_000
    ob = torch.empty(kb, dtype=torch.int32, device="cuda")
    tb = srv.submit(big, kb, 5, ob)
    time.sleep(0.02)  # the long job is claimed
    small = synth.cad_part(3000, seed=13, count=10).points.cuda()
    os_ = torch.empty(500, dtype=torch.int32, device="cuda")
    ts = srv.submit(small, 500, 6, os_)
    srv.wait(ts, timeout_us=60_000_000)
    assert not srv.poll(tb), "the small job waited for the long one"
    srv.wait(tb, timeout_us=120_000_000)
    srv.close()
    P = small.cpu().numpy()
    eo, _ = oracle.greedy32(P, 500, oracle.start_index(6, 3000))
    assert np.array_equal(os_.cpu().numpy(), eo)
    B = big.cpu().numpy()
    eo, _ = oracle.greedy32_grid(B, kb, oracle.start_index(5, B.shape[0]))
    assert np.array_equal(ob.cpu().numpy(), eo)


def test_server_producer_event_orders_the_copy(hip):
    """Points written by a kernel on the caller's stream just before submit:
    the server reads them after that work (the job's ready event)."""
    import torch
    srv = hip.Server(hbm_budget_bytes=1 << 30)
    P = synth.cad_part(40000, seed=14, count=20).points
    src = P.cuda()
    dst = torch.zeros_like(src)
    torch.cuda.synchronize()
    dst.copy_(src * 1.0)  # queued on the current stream, not waited for
    oo = torch.empty(3000, dtype=torch.int32, device="cuda")
    t = srv.submit(dst, 3000, 9, oo)
    srv.wait(t, timeout_us=60_000_000)
    srv.close()
    eo, _ = oracle.greedy32_grid(P.numpy(), 3000, oracle.start_index(9, 40000))
    assert np.array_equal(oo.cpu().numpy(), eo)
