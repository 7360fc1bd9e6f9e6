"""GPU parity of the ordered surfel records and of r_m against the oracle:
byte-identical records (octahedral normal codes included), bit-identical
r_m (paper Sec. 3 vertex buffer, Sec. 4.1 prefix-length estimate)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _normals(n, seed):
    rng = np.random.default_rng(seed)
    N = rng.normal(size=(n, 3)).astype(np.float32)
    N[:: 97] = 0.0                                   # zero normals
    N[5:: 101] = [0.0, 0.0, -1.0]                    # exact -z (folded corner)
    N[7:: 103] = [0.70710677, 0.70710677, 0.0]       # exact halves
    N[9:: 107] *= 1e-30                              # tiny, still finite
    N[11:: 109] = [np.inf, 0.0, 1.0]                 # non-finite
    return N


def test_emit_matches_oracle(hip):
    import torch
    n = 50000
    s = synth.cad_part(n, seed=41, count=30)
    P = s.points.numpy()
    N = _normals(n, 3)
    C = np.random.default_rng(4).integers(0, 256, size=(n, 3), dtype=np.uint8)
    pts = torch.from_numpy(P).cuda()
    o, _ = hip.order(pts, 20000, seed=9)
    torch.cuda.synchronize()
    oh = o.cpu().numpy()
    Nt, Ct = torch.from_numpy(N).cuda(), torch.from_numpy(C).cuda()
    for k in (1, 255, 256, 257, 1000, 20000):
        rec = hip.emit_surfels(pts, o[:k], Nt, Ct).cpu().numpy()
        exp = oracle.emit_surfels(P, oh[:k], N, C)
        assert np.array_equal(rec, exp), "k=%d: records differ first at %d" % (k, int(np.argmax((rec != exp).any(1))))
    bare = hip.emit_surfels(pts, o).cpu().numpy()
    assert np.array_equal(bare, oracle.emit_surfels(P, oh))
    # order entries outside [0, n): NaN position, zero codes and colour
    bad = torch.tensor([3, -1, n, n + 5, 0], dtype=torch.int32, device="cuda")
    rec = hip.emit_surfels(pts, bad, Nt, Ct).cpu().numpy()
    assert np.array_equal(rec.view(np.uint32), oracle.emit_surfels(P, bad.cpu().numpy(), N, C).view(np.uint32))


def test_emit_headline_size(hip):
    """4,194,304 candidates ordered to 262,144: every record equals the oracle's."""
    import torch
    n, k = 4194304, 262144
    s = synth.cad_part(n, seed=2)
    P = s.points.numpy()
    pts = torch.from_numpy(P).cuda()
    o, _ = hip.order(pts, k, seed=2)
    N = s.normals.numpy().astype(np.float32)
    C = s.colors.numpy().astype(np.uint8)
    rec = hip.emit_surfels(pts, o, torch.from_numpy(N).cuda(), torch.from_numpy(C).cuda()).cpu().numpy()
    assert np.array_equal(rec, oracle.emit_surfels(P, o.cpu().numpy(), N, C))


def test_median_nn_matches_oracle(hip):
    import torch
    n = 60000
    P = synth.cad_part(n, seed=43, count=40).points.numpy()
    pts = torch.from_numpy(P).cuda()
    o, _ = hip.order(pts, 5000, seed=1)
    oh = o.cpu().numpy()
    for pm in (2, 3, 999, 1000, 1001, 2048, 4096):
        got = hip.prefix_median_nn(pts, o, pm)
        exp = oracle.median_nn(P, oh, pm)
        assert np.float32(got).view(np.uint32) == np.float32(exp).view(np.uint32), "pm=%d: %r vs %r" % (pm, got, exp)
    # an order from a non-finite input: no estimate
    bad = o.clone()
    bad[17] = -1
    assert np.isnan(hip.prefix_median_nn(pts, bad, 100))
    # the estimate and the exact prefix for the same radius stay in a sane ratio
    r_m = hip.prefix_median_nn(pts, o, 1000)
    p_est = hip.prefix_length(r_m / 2, r_m, 1000, 5000)
    assert p_est == 4000
