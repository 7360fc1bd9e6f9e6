"""Autotuner: the chosen configuration is recorded for its size, used by
calls without a tuning, and (like every configuration) orders exactly as the
oracle; the batch tuner's cell occupancy gives the same batch results."""
import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_batch import make_batch
from tests.test_gpu_scan import assert_parity

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,k", [(16384, 16384), (60000, 6000)])
def test_autotune_records_and_orders_exactly(hip, n, k):
    import torch
    hip.autotune_clear()
    P = synth.cad_part(n, seed=71).points.numpy()
    pts = torch.from_numpy(P).cuda()
    t = hip.autotune(pts, k, seed=4)
    assert t.kernel in (hip.KERNEL_WG, hip.KERNEL_COOP, hip.KERNEL_GRID)
    got = hip.autotune_lookup(n, k)
    assert got is not None and bytes(got) == bytes(t)
    assert hip.auto_kernel(n, k) == t.kernel
    # calls without a tuning now use the recorded one
    o, r = hip.order(pts, k, seed=4)
    torch.cuda.synchronize()
    eo, er = oracle.greedy32_grid(P, k, oracle.start_index(4, n))
    assert_parity(o.cpu().numpy(), r.cpu().numpy(), eo, er, "tuned n=%d" % n)
    hip.autotune_clear()
    assert hip.autotune_lookup(n, k) is None


def test_batch_autotune(hip):
    import torch
    objs, ks, seeds, offs = make_batch(17)
    pts = torch.from_numpy(np.concatenate(objs).astype(np.float32)).cuda()
    t = hip.batch_autotune(pts, offs, ks, seeds)
    assert t.kernel == hip.KERNEL_GRID and t.cell_points in (4.0, 8.0, 16.0, 32.0)
    plan = hip.BatchPlan(offs, ks, seeds, tune=t)
    o, r = plan.execute(pts)
    torch.cuda.synchronize()
    oo = o.cpu().numpy()
    rr = r.cpu().numpy()
    for j in range(len(objs)):
        if ks[j] == 0:
            continue
        a, b = plan.out_offsets[j], plan.out_offsets[j + 1]
        eo, er = oracle.greedy32(objs[j], ks[j], oracle.start_index(seeds[j], objs[j].shape[0]))
        assert_parity(oo[a:b], rr[a:b], eo, er, "tuned batch object %d" % j)
    plan.close()


def test_batch_autotune_wide_share(hip):
    """A batch with objects for the 1024-thread workgroups: the tuner also
    times the whole batch per share of the CUs given to them and returns one
    of its candidates in `groups`; every object of the tuned plan orders as
    the oracle (the two long chains by the grid oracle)."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    sizes = [270000, 262000] + [3000 + 1700 * i for i in range(10)]
    ks = [66000, 65600] + [s // 4 for s in sizes[2:]]
    objs = [synth.cad_part(s, seed=90 + i, count=30).points.numpy() for i, s in enumerate(sizes)]
    seeds = [7 * i + 3 for i in range(len(sizes))]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pts = torch.from_numpy(np.concatenate(objs).astype(np.float32)).cuda()
    t = hip.batch_autotune(pts, offs, ks, seeds)
    assert t.kernel == hip.KERNEL_GRID and t.cell_points in (4.0, 8.0, 16.0, 32.0)
    assert t.groups in [cus * e // 8 for e in range(4, 8)], t.groups
    plan = hip.BatchPlan(offs, ks, seeds, tune=t)
    o, r = plan.execute(pts)
    torch.cuda.synchronize()
    oo, rr = o.cpu().numpy(), r.cpu().numpy()
    for j in range(len(objs)):
        a, b = plan.out_offsets[j], plan.out_offsets[j + 1]
        st = oracle.start_index(seeds[j], objs[j].shape[0])
        if ks[j] > 20000:
            eo, er = oracle.greedy32_grid(objs[j], ks[j], st)
        else:
            eo, er = oracle.greedy32(objs[j], ks[j], st)
        assert_parity(oo[a:b], rr[a:b], eo, er, "tuned wide batch object %d" % j)
    plan.close()


def test_tune_cache_file(hip, tmp_path, monkeypatch):
    """BS_TUNE_CACHE: the autotuner records its winner in the file, and after
    the in-memory table is cleared the automatic choice reads it back (what a
    later process does); the recorded configuration orders exactly."""
    import torch
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("BS_TUNE_CACHE", str(path))
    hip.autotune_clear()
    n, k = 30000, 3000
    P = synth.cad_part(n, seed=72).points.numpy()
    pts = torch.from_numpy(P).cuda()
    t = hip.autotune(pts, k, seed=5)
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("bluesurfels-tune-v1 gfx")
    f = lines[0].split()
    assert (int(f[2]), int(f[3]), int(f[4])) == (14, 11, t.kernel)  # floor(log2 n), floor(log2 k)
    hip.autotune_clear()
    got = hip.autotune_lookup(n, k)
    assert got is not None and bytes(got) == bytes(t)
    # a malformed line and another size class leave the entry usable
    path.write_text("garbage line\n" + lines[0] + "\n" + lines[0].replace(" 14 11 ", " 20 11 ", 1) + "\n")
    hip.autotune_clear()
    got = hip.autotune_lookup(n, k)
    assert got is not None and bytes(got) == bytes(t)
    o, r = hip.order(pts, k, seed=5)
    torch.cuda.synchronize()
    eo, er = oracle.greedy32_grid(P, k, oracle.start_index(5, n))
    assert_parity(o.cpu().numpy(), r.cpu().numpy(), eo, er, "cached tuning")
    monkeypatch.delenv("BS_TUNE_CACHE")
    hip.autotune_clear()
    assert hip.autotune_lookup(n, k) is None
