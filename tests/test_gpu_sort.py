"""The grid builds' Morton sort (hand-written radix sort, three passes of 10
bits, per object in a batch) against a numpy reference: the codes are
recomputed here from their definition in include/bluesurfels.h and the
expected permutation is numpy's stable argsort of them."""
import numpy as np
import pytest

import synth
from tests import cases

pytestmark = pytest.mark.gpu


def morton_codes(P):
    """30-bit codes of float32 points [n, 3] (binary32 quantization of the
    bounding box's longest side, 10 bits per axis, x lowest in each triple)."""
    P = np.asarray(P, dtype=np.float32)
    lo = P.min(axis=0)
    hi = P.max(axis=0)
    ext = np.float32(max(hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]))
    scale = np.float32(1024.0) / ext if (ext > 0 and np.isfinite(ext)) else np.float32(0.0)
    with np.errstate(invalid="ignore", over="ignore"):
        f = (P - lo) * scale
    q = np.where(np.isfinite(f), f, 0).astype(np.float64)
    q = np.clip(np.trunc(q), 0, 1023).astype(np.uint32)
    code = np.zeros(P.shape[0], dtype=np.uint32)
    for bit in range(10):
        for a in range(3):
            code |= ((q[:, a] >> bit) & 1) << (3 * bit + a)
    return code


def expected_order(P):
    return np.argsort(morton_codes(P), kind="stable").astype(np.int32)


@pytest.mark.parametrize("n", [1, 2, 63, 4095, 4096, 4097, 12289, 100003])
def test_morton_order_matches_stable_argsort(hip, n):
    import torch
    P = synth.cad_part(max(n, 8), seed=n, count=20).points.numpy()[:n]
    got = hip.morton_order(torch.from_numpy(P).cuda()).cpu().numpy()
    assert np.array_equal(got, expected_order(P))


def test_morton_order_ties_keep_index_order(hip):
    """Many equal codes (a lattice coarser than the quantization, and exact
    duplicates): the sort must be stable."""
    import torch
    g = np.stack(np.meshgrid(np.arange(7), np.arange(5), np.arange(3), indexing="ij"), -1).reshape(-1, 3)
    P = np.repeat(g.astype(np.float32), 97, axis=0)
    rng = np.random.default_rng(3)
    P = P[rng.permutation(P.shape[0])]
    got = hip.morton_order(torch.from_numpy(P).cuda()).cpu().numpy()
    assert np.array_equal(got, expected_order(P))


def test_batch_morton_order_per_object(hip):
    """Objects of many sizes (empty, below, at and above a 4,096-key tile)
    each sorted within its own rows."""
    import torch
    sizes = [0, 1, 4095, 4096, 0, 4097, 9000, 3, 20000, 8192]
    objs = [synth.cad_part(max(s, 8), seed=30 + i, count=15).points.numpy()[:s] for i, s in enumerate(sizes)]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    ks = [min(s, 1) for s in sizes]
    pts = torch.from_numpy(np.concatenate([o for o in objs if o.shape[0]]).astype(np.float32)).cuda()
    plan = hip.BatchPlan(offs, ks, None)
    got = plan.morton_order(pts).cpu().numpy()
    plan.close()
    for j, P in enumerate(objs):
        if P.shape[0]:
            assert np.array_equal(got[offs[j]:offs[j + 1]], expected_order(P)), "object %d" % j


def test_morton_order_adversarial_sets(hip):
    import torch
    for name in ("collinear", "duplicates", "lattice", "mixed_scale", "subnormal", "huge"):
        P = np.ascontiguousarray(cases.ADVERSARIAL[name](3000, 5), dtype=np.float32)
        got = hip.morton_order(torch.from_numpy(P).cuda()).cpu().numpy()
        assert np.array_equal(got, expected_order(P)), name
