"""Batched ordering: every object bit-identical to the oracle and to ordering
it alone (the same result in the batch as alone)."""
import numpy as np
import pytest

import oracle
import synth
from tests import cases, pins
from tests.test_gpu_scan import assert_parity

pytestmark = pytest.mark.gpu


def make_batch(seed, count=40):
    rng = np.random.default_rng(seed)
    objs, ks, seeds = [], [], []
    kinds = sorted(cases.ADVERSARIAL)
    for j in range(count):
        r = j % 5
        if r == 0:
            n = int(rng.integers(1, 5))
            P = cases.random_cloud(n, 1000 + j)
        elif r == 1:
            n = int(rng.integers(100, 3000))
            P = cases.ADVERSARIAL[kinds[j % len(kinds)]](n, 2000 + j)
        elif r == 2:
            n = int(rng.integers(2000, 30000))
            P = synth.cad_part(n, seed=3000 + j, count=20).points.numpy()
        elif r == 3:
            n = int(rng.integers(500, 9000))
            P = synth.scene_object(j % 3, n, seed=4000 + j).points.numpy()
        else:
            n = 0 if j % 10 == 4 else int(rng.integers(1, 400))
            P = cases.random_cloud(max(n, 0), 5000 + j)[:n]
        k = 0 if n == 0 else int(rng.integers(0, n + 1)) if j % 7 else n
        objs.append(np.asarray(P, dtype=np.float32).reshape(-1, 3))
        ks.append(k)
        seeds.append(int(rng.integers(0, 2**63)))
    offs = np.concatenate([[0], np.cumsum([o.shape[0] for o in objs])]).astype(np.int64)
    return objs, ks, seeds, offs


def test_batch_matches_oracle_and_alone(hip):
    import torch
    objs, ks, seeds, offs = make_batch(7)
    plan = hip.BatchPlan(offs, ks, seeds)
    allp = torch.from_numpy(np.concatenate(objs)).cuda()
    o, r = plan.execute(allp)
    torch.cuda.synchronize()
    o = o.cpu().numpy()
    r = r.cpu().numpy()
    for j, P in enumerate(objs):
        a, b = plan.out_offsets[j], plan.out_offsets[j + 1]
        assert b - a == ks[j]
        if ks[j] == 0:
            continue
        st = oracle.start_index(seeds[j], P.shape[0])
        eo, er = oracle.greedy32_grid(P, ks[j], st)
        assert_parity(o[a:b], r[a:b], eo, er, "batch object %d (n=%d k=%d)" % (j, P.shape[0], ks[j]))
        # alone through the single-object entry point
        so, sr = hip.order(torch.from_numpy(P).cuda(), ks[j], seed=seeds[j])
        assert_parity(o[a:b], r[a:b], so.cpu().numpy(), sr.cpu().numpy(), "alone vs batch %d" % j)
    plan.close()


def test_batch_replay_and_nonfinite(hip):
    import torch
    objs, ks, seeds, offs = make_batch(11, count=25)
    objs[3] = objs[3].copy()
    if objs[3].shape[0] > 0:
        objs[3][0, 1] = np.nan
    plan = hip.BatchPlan(offs, ks, seeds)
    allp = torch.from_numpy(np.concatenate(objs)).cuda()
    # fixed outputs and workspace: the first execute captures the graph of
    # the whole execute, the others replay it (with the program's own work
    # and synchronisations between them)
    oo = torch.empty(plan.total_k, dtype=torch.int32, device="cuda")
    rr = torch.empty(plan.total_k, dtype=torch.float32, device="cuda")
    first = [x.cpu().numpy().copy() for x in plan.execute(allp, oo, rr)]
    junk = torch.zeros(1 << 20, device="cuda")
    for rep in range(3):
        oo.fill_(-7)
        junk.add_(1.0)
        torch.cuda.synchronize()
        o, r = plan.execute(allp, oo, rr)
        torch.cuda.synchronize()
        assert np.array_equal(o.cpu().numpy(), first[0]), "replay %d order" % rep
        assert pins.same_f32(r.cpu().numpy(), first[1]), "replay %d radius" % rep
    # a replay reads the points' current contents: swapping two objects'
    # coordinates within the buffer changes only those objects' outputs
    saved = allp.clone()
    a0, a1 = int(offs[0]), int(offs[1])
    allp[a0:a1] = allp[a0:a1].flip(0)
    o2, _ = plan.execute(allp, oo, rr)
    torch.cuda.synchronize()
    P0 = allp[a0:a1].cpu().numpy()
    if ks[0] > 0:
        eo0, _ = oracle.greedy32_grid(P0, ks[0], oracle.start_index(seeds[0], P0.shape[0]))
        assert np.array_equal(o2.cpu().numpy()[plan.out_offsets[0]:plan.out_offsets[1]], eo0)
    allp.copy_(saved)
    for j, P in enumerate(objs):
        a, b = plan.out_offsets[j], plan.out_offsets[j + 1]
        if ks[j] == 0:
            continue
        if j == 3 and P.shape[0] > 0:
            assert (first[0][a:b] == -1).all() and np.isnan(first[1][a:b]).all()
        else:
            st = oracle.start_index(seeds[j], P.shape[0])
            eo, er = oracle.greedy32_grid(P, ks[j], st)
            assert_parity(first[0][a:b], first[1][a:b], eo, er, "object %d" % j)
    plan.close()


def test_batch_many_small_objects(hip):
    import torch
    sizes = synth.log_uniform_sizes(600, 64, 4096, seed=5)
    objs = [synth.cad_part(n, seed=9000 + j, count=8).points.numpy() if j % 50 == 0
            else cases.random_cloud(n, 9000 + j) for j, n in enumerate(sizes)]
    ks = [n // 4 for n in sizes]
    seeds = list(range(len(sizes)))
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    plan = hip.BatchPlan(offs, ks, seeds)
    o, r = plan.execute(torch.from_numpy(np.concatenate(objs)).cuda())
    torch.cuda.synchronize()
    o = o.cpu().numpy()
    r = r.cpu().numpy()
    for j in range(0, len(sizes), 7):
        a, b = plan.out_offsets[j], plan.out_offsets[j + 1]
        eo, er = oracle.greedy32(objs[j], ks[j], oracle.start_index(seeds[j], sizes[j]))
        assert_parity(o[a:b], r[a:b], eo, er, "small object %d" % j)
    plan.close()


def test_batch_scene_objects(hip):
    """Objects of the heterogeneous scene (sheets, tori, box clusters) in one
    batch equal the oracle, at the scene's k = 12% of n."""
    import torch
    sizes = synth.scene_sizes(24, total=60000, lo=200, hi=12000, seed=9)
    pts, offs = synth.scene_batch(sizes, seed=9)
    ks = [int(0.12 * s) for s in sizes]
    seeds = [90 + j for j in range(len(sizes))]
    plan = hip.BatchPlan(offs, ks, seeds)
    o, r = plan.execute(pts.cuda())
    torch.cuda.synchronize()
    oo, rr = o.cpu().numpy(), r.cpu().numpy()
    P = pts.numpy()
    for j in range(len(sizes)):
        a, b = plan.out_offsets[j], plan.out_offsets[j + 1]
        Pj = P[offs[j]:offs[j + 1]]
        eo, er = oracle.greedy32(Pj, ks[j], oracle.start_index(seeds[j], Pj.shape[0]))
        assert_parity(oo[a:b], rr[a:b], eo, er, "scene object %d (kind %d)" % (j, j % 3))
    plan.close()


@pytest.mark.parametrize("wide", [2, 5])
def test_batch_wide_workgroups(hip, wide):
    """The objects with the largest k on 1024-thread workgroups beside the
    256-thread ones (a non-finite object and a k = 0 object among the large
    ones): every object equals the oracle, or -1 / NaN when non-finite."""
    import torch
    rng = np.random.default_rng(70 + wide)
    objs, ks, seeds = [], [], []
    for j in range(12):
        n = int(rng.integers(40000, 160000)) if j < 6 else int(rng.integers(200, 5000))
        P = np.ascontiguousarray(synth.cad_part(n, seed=900 + j, count=30).points.numpy())
        if j == 2:
            P[17, 1] = np.nan
        objs.append(P)
        ks.append(0 if j == 4 else n // 4)
        seeds.append(int(rng.integers(0, 2**63)))
    offs = np.concatenate([[0], np.cumsum([o.shape[0] for o in objs])]).astype(np.int64)
    plan = hip.BatchPlan(offs, ks, seeds, tune=hip.tuning(batch_wide=wide))
    allp = torch.from_numpy(np.concatenate(objs)).cuda()
    oo = torch.empty(plan.total_k, dtype=torch.int32, device="cuda")
    rr = torch.empty(plan.total_k, dtype=torch.float32, device="cuda")
    for rep in range(2):  # capture, then a replay of the forked graph
        oo.fill_(-7)
        o, r = plan.execute(allp, oo, rr)
        torch.cuda.synchronize()
        o = o.cpu().numpy()
        r = r.cpu().numpy()
        for j, P in enumerate(objs):
            a, b = plan.out_offsets[j], plan.out_offsets[j + 1]
            if ks[j] == 0:
                continue
            if j == 2:
                assert (o[a:b] == -1).all() and np.isnan(r[a:b]).all()
                continue
            eo, er = oracle.greedy32_grid(P, ks[j], oracle.start_index(seeds[j], P.shape[0]))
            assert_parity(o[a:b], r[a:b], eo, er, "wide=%d object %d (n=%d k=%d) rep %d"
                          % (wide, j, P.shape[0], ks[j], rep))
    plan.close()


@pytest.mark.parametrize("picks", [1, 2, 16, 32])
def test_batch_picks_per_round(hip, picks):
    """Every cap on the picks per round (by default 24, 16 for large cells) orders each
    object exactly as the oracle does, wide objects included."""
    import torch
    objs, ks, seeds, offs = make_batch(11 + picks, count=20)
    big = [np.ascontiguousarray(synth.cad_part(n, seed=950 + n % 97, count=30).points.numpy())
           for n in (70000, 140000)]
    objs += big
    ks += [b.shape[0] // 3 for b in big]
    seeds += [picks * 1000 + 1, picks * 1000 + 2]
    offs = np.concatenate([[0], np.cumsum([o.shape[0] for o in objs])]).astype(np.int64)
    plan = hip.BatchPlan(offs, ks, seeds, tune=hip.tuning(picks=picks, batch_wide=2))
    o, r = plan.execute(torch.from_numpy(np.concatenate(objs)).cuda())
    torch.cuda.synchronize()
    o = o.cpu().numpy()
    r = r.cpu().numpy()
    for j, P in enumerate(objs):
        a, b = plan.out_offsets[j], plan.out_offsets[j + 1]
        if ks[j] == 0:
            continue
        eo, er = oracle.greedy32_grid(P, ks[j], oracle.start_index(seeds[j], P.shape[0]))
        assert_parity(o[a:b], r[a:b], eo, er, "picks=%d object %d (n=%d k=%d)" % (picks, j, P.shape[0], ks[j]))
    plan.close()


def test_batch_wide_object_with_more_blocks(hip):
    """An object of more than 4,194,304 candidates on a 1024-thread
    workgroup gets up to 2048 blocks of cells: equal to the oracle, and the
    small objects beside it too."""
    import torch
    big = np.ascontiguousarray(synth.cad_part(4_400_000, seed=977, count=60).points.numpy())
    objs = [big] + [np.ascontiguousarray(synth.cad_part(n, seed=978 + n % 7, count=20).points.numpy())
                    for n in (3000, 25000)]
    ks = [30000, 3000, 6000]
    seeds = [11, 12, 13]
    offs = np.concatenate([[0], np.cumsum([o.shape[0] for o in objs])]).astype(np.int64)
    plan = hip.BatchPlan(offs, ks, seeds, tune=hip.tuning(batch_wide=1))
    o, r = plan.execute(torch.from_numpy(np.concatenate(objs)).cuda())
    torch.cuda.synchronize()
    o = o.cpu().numpy()
    r = r.cpu().numpy()
    for j, P in enumerate(objs):
        a, b = plan.out_offsets[j], plan.out_offsets[j + 1]
        eo, er = oracle.greedy32_grid(P, ks[j], oracle.start_index(seeds[j], P.shape[0]))
        assert_parity(o[a:b], r[a:b], eo, er, "object %d (n=%d k=%d)" % (j, P.shape[0], ks[j]))
    plan.close()
