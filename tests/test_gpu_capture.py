"""GPU parity of the visible-surface capture (Sec. 3.1) against the oracle's
ray cast: the same candidates in the same order, positions and normals bit
for bit, colours equal; then the capture feeds the ordering on the device."""
import numpy as np
import pytest

import oracle
import synth
from tests import pins

pytestmark = pytest.mark.gpu


def _scene(name):
    if name == "sphere_and_box":
        return pins.pins_sphere_box()
    seed, cnt = {"cad12": (7, 12), "cad200": (2, 200)}[name]
    return pins.prims_arrays(synth.cad_primitives(seed, count=cnt))


def _gpu_capture(hip, arrays, R):
    import torch
    kind, center, rot, prm, rgb, lo, hi = arrays
    rec = hip.primitive_records(kind, center, rot, prm, rgb)
    p, n, c = hip.capture(rec, lo, hi, R)
    torch.cuda.synchronize()
    return p, n, c


@pytest.mark.parametrize("name,R", [("sphere_and_box", 64), ("cad12", 100), ("cad200", 256)])
def test_capture_matches_oracle(hip, name, R):
    arrays = _scene(name)
    ep, en, ec = oracle.capture32(*arrays, R)
    p, n, c = _gpu_capture(hip, arrays, R)
    p, n, c = p.cpu().numpy(), n.cpu().numpy(), c.cpu().numpy()
    assert p.shape == ep.shape, (p.shape, ep.shape)
    assert pins.same_f32(p, ep), "positions differ"
    assert pins.same_f32(n, en), "normals differ"
    assert np.array_equal(c, ec), "colours differ"


def test_capture_degenerate_and_errors(hip):
    import torch
    # one flat box: a box of zero height still has eight views that see it
    kind = np.array([1], np.int32)
    center = np.zeros((1, 3), np.float32)
    rot = np.eye(3, dtype=np.float32)[None]
    prm = np.array([[0.5, 0.25, 0.0]], np.float32)
    rgb = np.array([[9, 8, 7]], np.uint8)
    lo, hi = np.array([-0.5, -0.25, 0], np.float32), np.array([0.5, 0.25, 0], np.float32)
    ep, en, ec = oracle.capture32(kind, center, rot, prm, rgb, lo, hi, 32)
    p, n, c = _gpu_capture(hip, (kind, center, rot, prm, rgb, lo, hi), 32)
    assert pins.same_f32(p.cpu().numpy(), ep) and np.array_equal(c.cpu().numpy(), ec)
    # a point box: every view degenerate, nothing captured
    z = np.zeros(3, np.float32)
    p, n, c = _gpu_capture(hip, (kind, center, rot, prm, rgb, z, z), 16)
    assert p.shape[0] == 0
    # no primitives: nothing captured
    p, n, c = _gpu_capture(hip, (kind[:0], center[:0], rot[:0], prm[:0], rgb[:0], lo, hi), 16)
    assert p.shape[0] == 0
    with pytest.raises(hip.BSError):
        _gpu_capture(hip, (kind, center, rot, prm, rgb, hi, lo - 1), 16)
    del torch


def test_capture_then_order_on_device(hip):
    """The captured candidates ordered on the device equal the oracle's capture
    ordered by the oracle (the whole preprocessing of one node)."""
    import torch
    arrays = _scene("cad200")
    R = 128
    p, n, c = _gpu_capture(hip, arrays, R)
    k = min(5000, p.shape[0])
    o, r = hip.order(p.contiguous(), k, seed=3)
    ep, _, _ = oracle.capture32(*arrays, R)
    eo, er = oracle.greedy32_grid(ep, k, oracle.start_index(3, ep.shape[0]))
    assert np.array_equal(o.cpu().numpy(), eo) and pins.same_f32(r.cpu().numpy(), er)
    del torch
