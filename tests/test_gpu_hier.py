"""GPU parity of the bottom-up hierarchical generation (Sec. 3.4): every
node's picks, radii and source rows equal the oracle composed node by node
(a parent orders the surfels its children chose)."""
import numpy as np
import pytest

import synth
from tests import pins

pytestmark = pytest.mark.gpu


def _hierarchy():
    # 3 groups of 4 leaves under 3 inner nodes, one leaf straight under the
    # root, one leaf with k = 0; post-order numbering
    sizes, parents, ks = [], [], []
    leaf_sizes = [700, 5000, 1200, 20000, 333, 9000, 4100, 64, 2500, 15000, 800, 3000, 6000, 50]
    nodes = []
    li = 0
    for g in range(3):
        first = len(nodes)
        for _ in range(4):
            nodes.append(("leaf", leaf_sizes[li]))
            li += 1
        nodes.append(("inner", list(range(first, first + 4))))
    nodes.append(("leaf", leaf_sizes[li]))     # under the root directly
    li += 1
    nodes.append(("leaf", leaf_sizes[li]))     # k = 0
    nodes.append(("inner", [4, 9, 14, 15, 16]))  # root
    m = len(nodes)
    parents = [-1] * m
    for j, (kind, arg) in enumerate(nodes):
        if kind == "inner":
            for c in arg:
                parents[c] = j
    leaf_n = [arg if kind == "leaf" else 0 for kind, arg in nodes]
    offs = np.concatenate([[0], np.cumsum(leaf_n)]).astype(np.int64)
    ks = [0] * m
    for j, (kind, arg) in enumerate(nodes):
        if kind == "leaf":
            ks[j] = 0 if j == 16 else max(1, arg // 4)
        else:
            ks[j] = max(1, sum(ks[c] for c in arg) // 3)
    seeds = [(j * 0x9E3779B97F4A7C15 + 77) % 2**64 for j in range(m)]
    return parents, offs, ks, seeds, leaf_n


@pytest.mark.parametrize("method", ["exact", "sampler"])
def test_hierarchy_matches_composed_oracle(hip, method):
    import torch
    parents, offs, ks, seeds, leaf_n = _hierarchy()
    sizes = [n for n in leaf_n if n > 0]
    pts, _ = synth.cad_parts_batch(sizes, seed=41, count=30, device="cuda")
    P = pts.cpu().numpy()
    plan = hip.HierPlan(parents, offs, ks, seeds)
    sp = hip.sampler(200, 7, 0.0) if method == "sampler" else None
    o, r, s = plan.execute(pts, sp)
    torch.cuda.synchronize()
    o, r, s = o.cpu().numpy(), r.cpu().numpy(), s.cpu().numpy()
    ref = pins.hier_reference(P, parents, offs, ks, seeds, None if sp is None else (200, 7, 0.0))
    for j in range(len(parents)):
        a, b = plan.out_offsets[j], plan.out_offsets[j + 1]
        eo, er, es = ref[j]
        assert np.array_equal(o[a:b], eo), ("node", j, method)
        assert pins.same_f32(r[a:b], er), ("radius", j)
        assert np.array_equal(s[a:b].astype(np.int64), es), ("source", j)
    plan.close()


def test_hierarchy_nonfinite_propagates(hip):
    import torch
    parents = [2, 2, 4, -1, -1]      # leaves 0, 1 under 2; 2 under 4; leaf 3 alone
    leaf_n = [300, 400, 0, 500, 0]
    offs = np.concatenate([[0], np.cumsum(leaf_n)]).astype(np.int64)
    ks = [60, 80, 50, 100, 20]
    pts, _ = synth.cad_parts_batch([300, 400, 500], seed=9, count=10, device="cuda")
    pts[350, 2] = float("inf")       # a candidate of leaf 1
    plan = hip.HierPlan(parents, offs, ks, [1, 2, 3, 4, 5])
    o, r, s = plan.execute(pts)
    torch.cuda.synchronize()
    o, s = o.cpu().numpy(), s.cpu().numpy()
    oo = plan.out_offsets
    for j in (1, 2, 4):
        assert (o[oo[j]:oo[j + 1]] == -1).all() and (s[oo[j]:oo[j + 1]] == -1).all(), j
    for j in (0, 3):
        assert (o[oo[j]:oo[j + 1]] >= 0).all(), j
    plan.close()
