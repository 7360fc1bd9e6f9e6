"""The profiling entry point orders exactly like the plain one.

bs_order_profile runs the same kernels with optional per-step device
timestamps and HIP events around the ordering kernel; neither instrument
may change a bit of the result.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_scan import assert_parity

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kernel", ["wg", "coop", "grid"])
def test_profile_matches_oracle(hip, kernel):
    import torch
    n, k = 20000, 5000
    P = synth.cad_part(n, seed=31).points.numpy()
    tune = {"wg": hip.tuning(kernel=hip.KERNEL_WG, block=1024, per_thread=16),
            "coop": hip.tuning(kernel=hip.KERNEL_COOP, block=1024, per_thread=1),
            "grid": hip.tuning(kernel=hip.KERNEL_GRID)}[kernel]
    if kernel == "wg":
        n = 16384
        P = P[:n]
    eo, er = oracle.greedy32(P, k, 9)
    Pt = torch.from_numpy(np.ascontiguousarray(P)).cuda()
    stream = torch.cuda.current_stream()
    b, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.record(stream)
    e.record(stream)
    o, r, t = hip.order_profile(Pt, k, start=9, tune=tune, stream=stream, events=(b, e))
    torch.cuda.synchronize()
    assert_parity(o.cpu().numpy(), r.cpu().numpy(), eo, er, "profile " + kernel)
    ticks = t.cpu().numpy()
    assert np.all(np.diff(ticks) >= 0) and ticks[0] > 0
    ms = b.elapsed_time(e)
    # the events bracket the ordering kernel: its duration covers the picks
    span_ms = (ticks[-1] - ticks[0]) / hip.wall_clock_hz() * 1e3
    assert ms > 0 and ms >= 0.9 * span_ms
    # without instruments
    o2, r2, t2 = hip.order_profile(Pt, k, start=9, tune=tune, ticks=False)
    torch.cuda.synchronize()
    assert t2 is None
    assert_parity(o2.cpu().numpy(), r2.cpu().numpy(), eo, er, "profile bare " + kernel)
