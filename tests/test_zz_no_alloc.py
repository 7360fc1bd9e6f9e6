"""The no-allocation entry point (bs_order_noalloc) against bs_order_ex.

Two calls in a row on the library's per-GPU scratch array, the second with a
smaller input (the array keeps the first call's contents), then a third on
the single-workgroup plan; each must equal bs_order_ex on a torch-allocated
workspace bit for bit (and the oracle on the small one).  Sizes beyond the
array are rejected before anything is enqueued.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import pins

pytestmark = pytest.mark.gpu


def _pair(hip, P, k, start, tune=None):
    import torch
    pts = torch.from_numpy(np.ascontiguousarray(P, dtype=np.float32)).cuda()
    o1, r1 = hip.order_noalloc(pts, k, start=start, tune=tune)
    n = P.shape[0]
    ws = torch.empty(hip.workspace_size(n, k, tune), dtype=torch.uint8, device="cuda")
    o2, r2 = hip.order(pts, k, start=start, tune=tune, workspace=ws)
    torch.cuda.synchronize()
    return o1.cpu().numpy(), r1.cpu().numpy(), o2.cpu().numpy(), r2.cpu().numpy()


def test_noalloc_equals_workspace_entry(hip):
    big = synth.cad_part(400000, seed=12).points.numpy()
    small = synth.sphere_and_box(n=9000, seed=3).points.numpy()
    tiny = synth.cad_part(3000, seed=13).points.numpy()
    for label, P, k, start in (("400,000 -> 40,000", big, 40000, 17), ("9,000 -> 9,000", small, 9000, 5),
                               ("3,000 -> 1,000", tiny, 1000, 0)):
        print("noalloc case:", label, flush=True)
        o1, r1, o2, r2 = _pair(hip, P, k, start)
        assert np.array_equal(o1, o2), label
        assert pins.same_f32(r1, r2), label
        if P.shape[0] <= 9000:
            eo, er = oracle.greedy32(P, k, start)
            assert np.array_equal(o1, eo) and pins.same_f32(r1, er), label
    # a forced tuning through the same array: the grid kernel
    tune = hip.tuning(kernel=hip.KERNEL_GRID, picks=16)
    o1, r1, o2, r2 = _pair(hip, small, 4000, 9, tune)
    assert np.array_equal(o1, o2) and pins.same_f32(r1, r2)


def test_noalloc_rejects_beyond_the_array(hip):
    import torch
    n = 700000  # beyond the documented 524,288 and beyond the array's bytes
    assert hip.workspace_size(n, 1000) > hip.noalloc_max_bytes()
    pts = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(hip.BSError) as e:
        hip.order_noalloc(pts, 1000)
    assert e.value.code == hip.BS_ERR_UNSUPPORTED
