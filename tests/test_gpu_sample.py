"""GPU parity of the paper's randomized progressive sampler (Sec. 3.2)
against the CPU oracle's implementation of the same rules: orders, radii
and counts bit for bit, alone and batched; the whole-set sample equals the
exact greedy permutation; the prefix nearest-neighbour measure (Sec. 3.3)."""
import numpy as np
import pytest

import oracle
import synth
from tests import cases, pins

pytestmark = pytest.mark.gpu


def _gpu(hip, P, k, seed, start, **kw):
    import torch
    pts = torch.from_numpy(np.ascontiguousarray(P, dtype=np.float32)).cuda()
    o, r, c = hip.sample(pts, k, seed=seed, start=start, **kw)
    torch.cuda.synchronize()
    return o.cpu().numpy(), r.cpu().numpy(), c


def _same(o, r, c, eo, er, ec, label):
    assert c == ec, "%s: count %d, oracle %d" % (label, c, ec)
    if not np.array_equal(o, eo):
        i = int(np.argmax(o != eo))
        raise AssertionError("%s: order differs first at %d: gpu %d oracle %d" % (label, i, o[i], eo[i]))
    assert pins.same_f32(r, er), label + ": radius bits differ"


@pytest.mark.parametrize("S,K,v", [(200, 500, 0.0), (200, 20, 0.0), (17, 3, 0.0), (1, -1, 0.0), (256, 1, 0.0),
                                   (64, 50, 0.5), (8, 2, 1.5)])
def test_sampler_matches_oracle(hip, S, K, v):
    s = synth.cad_part(30000, seed=21)
    P = s.points.numpy()
    for k, seed in ((7500, 5), (30000, 2**63 + 11)):
        st = oracle.start_index(seed, P.shape[0])
        eo, er, ec = oracle.sample32(P, k, seed, st, S, K, v)
        o, r, c = _gpu(hip, P, k, seed, None, sample_size=S, growth_rounds=K, vicinity=v)
        _same(o, r, c, eo, er, ec, "cad_part S=%d K=%d v=%g k=%d" % (S, K, v, k))


def test_sampler_sphere_box_paper_defaults(hip):
    P = synth.sphere_and_box(n=16384, seed=1).points.numpy()
    eo, er, ec = oracle.sample32(P, 16384, 1, oracle.start_index(1, 16384))
    o, r, c = _gpu(hip, P, 16384, 1, None)
    _same(o, r, c, eo, er, ec, "sphere_and_box defaults")


@pytest.mark.parametrize("name", sorted(cases.ADVERSARIAL))
def test_sampler_adversarial(hip, name):
    for n in (1, 2, 3, 64, 1000, 5000):
        P = cases.ADVERSARIAL[name](n, 41 + n)
        for S, K, v in ((200, 500, 0.0), (5, 2, 0.0), (33, 7, 0.8)):
            k = n if S != 5 else max(1, n // 2)
            st = (5 * n) // 7
            eo, er, ec = oracle.sample32(P, k, 1234 + n, st, S, K, v)
            o, r, c = _gpu(hip, P, k, 1234 + n, st, sample_size=S, growth_rounds=K, vicinity=v)
            _same(o, r, c, eo, er, ec, "%s n=%d S=%d" % (name, n, S))


def test_sampler_whole_set_is_exact_greedy(hip):
    P = synth.cad_part(20000, seed=8).points.numpy()
    k = 6000
    eo, er = oracle.greedy32_grid(P, k, 77)
    for K in (1, 3, 500, -1):
        o, r, c = _gpu(hip, P, k, 9, 77, sample_size=0, growth_rounds=K)
        _same(o, r, c, eo, er, k, "whole set K=%d" % K)


def test_sampler_nonfinite_and_edges(hip):
    import torch
    P = cases.random_cloud(500, 3)
    P[17, 1] = np.nan
    o, r, c = _gpu(hip, P, 40, 1, 0, check=False)
    assert (o == -1).all() and np.isnan(r).all() and c == 0
    with pytest.raises(ValueError):
        _gpu(hip, P, 40, 1, 0)
    Q = cases.random_cloud(10, 4)
    o, r, c = _gpu(hip, Q, 0, 1, 0)
    assert o.size == 0
    with pytest.raises(hip.BSError):
        _gpu(hip, Q, 5, 1, 0, sample_size=300)
    with pytest.raises(hip.BSError):
        _gpu(hip, Q, 5, 1, 0, sample_size=0, vicinity=1.0)
    with pytest.raises(hip.BSError):
        _gpu(hip, Q, 11, 1, 0)
    del torch


def test_sampler_batched_equals_alone(hip):
    import torch
    sizes = [1, 2, 70, 3000, 9000, 20000, 257, 5000] * 3
    ks = [min(s, max(1, s // 4)) for s in sizes]
    ks[5] = 0
    seeds = [(977 * j + 5) * 0x9E3779B97F4A7C15 % 2**64 for j in range(len(sizes))]
    pts, offs = synth.cad_parts_batch(sizes, seed=31, count=40, device="cuda")
    P = pts.cpu().numpy()
    plan = hip.BatchPlan(offs, ks, seeds)
    for S, K, v in ((200, 500, 0.0), (12, 4, 0.7)):
        o, r, c = plan.execute_sample(pts, sample_size=S, growth_rounds=K, vicinity=v)
        torch.cuda.synchronize()
        o, r, c = o.cpu().numpy(), r.cpu().numpy(), c.cpu().numpy()
        for j in range(len(sizes)):
            a, b = plan.out_offsets[j], plan.out_offsets[j + 1]
            Pj = P[offs[j]:offs[j + 1]]
            if ks[j] == 0:
                assert c[j] == 0
                continue
            eo, er, ec = oracle.sample32(Pj, ks[j], seeds[j], oracle.start_index(seeds[j], Pj.shape[0]), S, K, v)
            _same(o[a:b], r[a:b], int(c[j]), eo, er, ec, "object %d S=%d" % (j, S))
    plan.close()


def test_sampler_batch_full_size_sampled(hip):
    """The 1,000-part batch (n log-uniform 2,048..2,097,152, k = n/4) through
    the batched sampler; checked against the oracle on the 12 smallest objects
    in full and on the first 600 picks of 6 larger ones (the sampler's rounds
    do not depend on k, so a prefix is an ordering of its own)."""
    import torch
    m = 1000
    sizes = synth.log_uniform_sizes(m, 2048, 2097152, seed=3)
    ks = [s // 4 for s in sizes]
    seeds = [3 * 1000003 + j for j in range(m)]
    pts, offs = synth.cad_parts_batch(sizes, seed=3, count=200, device="cuda")
    plan = hip.BatchPlan(offs, ks, seeds)
    o, r, c = plan.execute_sample(pts)
    torch.cuda.synchronize()
    o, r, c = o.cpu().numpy(), r.cpu().numpy(), c.cpu().numpy()
    assert np.array_equal(c, np.asarray(ks, dtype=np.int32))
    by_size = sorted(range(m), key=lambda j: sizes[j])
    for j in by_size[:12] + by_size[200:1000:160]:
        Pj = pts[offs[j]:offs[j + 1]].cpu().numpy()
        kk = ks[j] if j in by_size[:12] else 600
        eo, er, ec = oracle.sample32(Pj, kk, seeds[j], oracle.start_index(seeds[j], Pj.shape[0]))
        a = plan.out_offsets[j]
        _same(o[a:a + kk], r[a:a + kk], kk, eo, er, ec, "object %d (n=%d)" % (j, sizes[j]))
    plan.close()


def test_prefix_nn_matches_oracle(hip):
    import torch
    P = synth.cad_part(20000, seed=2).points.numpy()
    o, _ = oracle.greedy32_grid(P, 5000, 3)
    pts = torch.from_numpy(P).cuda()
    od = torch.from_numpy(o).cuda()
    for p in (1, 2, 255, 256, 257, 1000, 5000):
        g = hip.prefix_nn(pts, od, p).cpu().numpy()
        e = oracle.prefix_nn(P, o, p)
        assert pins.same_f32(g, e), p
    bad = od.clone()
    bad[3] = -1
    assert np.isnan(hip.prefix_nn(pts, bad, 100).cpu().numpy()).all()


def test_sampler_batch_wide_workgroups(hip):
    """The batch's largest objects sampled by 1024-thread workgroups beside
    the 256-thread ones (forced for two objects): every object equals the
    sampler oracle."""
    import torch
    sizes = [40000, 60000, 3000, 500, 9000]
    ks = [10000, 15000, 3000, 100, 2000]
    seeds = [41, 42, 43, 44, 45]
    pts, offs = synth.cad_parts_batch(sizes, seed=37, count=40, device="cuda")
    P = pts.cpu().numpy()
    expect = [oracle.sample32(P[offs[j]:offs[j + 1]], ks[j], seeds[j], oracle.start_index(seeds[j], sizes[j]))
              for j in range(len(sizes))]
    plan = hip.BatchPlan(offs, ks, seeds, tune=hip.tuning(batch_wide=2))
    for rep in range(2):
        o, r, c = plan.execute_sample(pts)
        torch.cuda.synchronize()
        o, r, c = o.cpu().numpy(), r.cpu().numpy(), c.cpu().numpy()
        for j in range(len(sizes)):
            a, b = plan.out_offsets[j], plan.out_offsets[j + 1]
            eo, er, ec = expect[j]
            _same(o[a:b], r[a:b], int(c[j]), eo, er, ec, "object %d rep %d" % (j, rep))
    plan.close()
