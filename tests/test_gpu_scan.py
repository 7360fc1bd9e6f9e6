"""GPU parity of the resident full-scan kernels against the CPU oracle.

Orders and radii must match bit for bit (the radii are the binary32
square roots of the selected squared distances on both sides).
"""
import numpy as np
import pytest

import oracle
import synth
from tests import cases, pins

pytestmark = pytest.mark.gpu


def run(hip, P_np, k, start=None, tune=None, seed=0):
    import torch
    P = torch.from_numpy(np.ascontiguousarray(P_np, dtype=np.float32)).cuda()
    o, r = hip.order(P, k, seed=seed, start=start, tune=tune)
    torch.cuda.synchronize()
    return o.cpu().numpy(), r.cpu().numpy()


def assert_parity(o, r, eo, er, label=""):
    if not np.array_equal(o, eo):
        i = int(np.argmax(o != eo))
        raise AssertionError("%s: order differs first at %d: gpu %d oracle %d" % (label, i, o[i], eo[i]))
    assert pins.same_f32(r, er), label + ": radius bits differ"


def test_sphere_box_full_order(hip):
    s = synth.sphere_and_box(n=16384, seed=1)
    P = s.points.numpy()
    st = oracle.start_index(1, P.shape[0])
    eo, er = oracle.greedy32(P, 16384, st)
    o, r = run(hip, P, 16384, start=st)
    assert_parity(o, r, eo, er, "sphere_and_box")
    o, r = run(hip, P, 16384, start=st, tune=hip.tuning(kernel=hip.KERNEL_WG))
    assert_parity(o, r, eo, er, "sphere_and_box one workgroup")
    # radius within 1e-6 relative of the binary64 recomputation along the order
    r64 = oracle.along_order64(P, o)
    assert np.all(np.abs(r[1:].astype(np.float64) - r64[1:]) <= 1e-6 * r64[1:])


@pytest.mark.parametrize("name", sorted(cases.ADVERSARIAL))
def test_adversarial_single_workgroup(hip, name):
    for n in (1, 2, 3, 64, 65, 1000, 1025, 4097):
        P = cases.ADVERSARIAL[name](n, 31 + n)
        st = (7 * n) // 11
        eo, er = oracle.greedy32(P, n, st)
        o, r = run(hip, P, n, start=st, tune=hip.tuning(kernel=hip.KERNEL_WG))
        assert_parity(o, r, eo, er, "%s n=%d" % (name, n))


@pytest.mark.parametrize("pt", [1, 2, 4, 8, 12, 16])
def test_single_workgroup_tilings(hip, pt):
    n = min(1024 * pt, 9000)
    P = synth.cad_part(n, seed=5).points.numpy()
    eo, er = oracle.greedy32(P, n, 3)
    o, r = run(hip, P, n, start=3, tune=hip.tuning(kernel=hip.KERNEL_WG, block=1024, per_thread=pt))
    assert_parity(o, r, eo, er, "pt=%d" % pt)


@pytest.mark.parametrize("pt", [1, 4, 8, 16])
def test_cooperative_tilings(hip, pt):
    n = 40000
    P = synth.cad_part(n, seed=6).points.numpy()
    k = 6000
    eo, er = oracle.greedy32_grid(P, k, 11)
    o, r = run(hip, P, k, start=11, tune=hip.tuning(kernel=hip.KERNEL_COOP, block=1024, per_thread=pt))
    assert_parity(o, r, eo, er, "coop pt=%d" % pt)


def test_cooperative_512_threads(hip):
    n = 70000
    P = synth.cad_part(n, seed=7).points.numpy()
    eo, er = oracle.greedy32_grid(P, 3000, 0)
    for pt in (24, 32):
        o, r = run(hip, P, 3000, start=0, tune=hip.tuning(kernel=hip.KERNEL_COOP, block=512, per_thread=pt))
        assert_parity(o, r, eo, er, "coop512 pt=%d" % pt)


@pytest.mark.parametrize("name", ["duplicates", "lattice", "subnormal", "huge", "mixed_scale"])
def test_cooperative_adversarial(hip, name):
    n = 20000
    P = cases.ADVERSARIAL[name](n, 77)
    k = n // 2
    eo, er = oracle.greedy32_grid(P, k, 123)
    o, r = run(hip, P, k, start=123, tune=hip.tuning(kernel=hip.KERNEL_COOP, block=1024, per_thread=4))
    assert_parity(o, r, eo, er, name)


def test_all_kernels_agree_and_repeat(hip):
    n = 12000
    P = synth.sphere_and_box(n=n, seed=9).points.numpy()
    base = run(hip, P, n, start=5, tune=hip.tuning(kernel=hip.KERNEL_WG))
    for tune in (hip.tuning(kernel=hip.KERNEL_COOP, per_thread=1),
                 hip.tuning(kernel=hip.KERNEL_COOP, per_thread=4),
                 hip.tuning(kernel=hip.KERNEL_WG, per_thread=16),
                 None):
        for _ in range(2):
            o, r = run(hip, P, n, start=5, tune=tune)
            assert_parity(o, r, base[0], base[1], "tiling")


def test_seeded_start_and_prefix_stability(hip):
    import torch
    n = 5000
    P = cases.random_cloud(n, 3)
    Pt = torch.from_numpy(P).cuda()
    for seed in (0, 1, 2, 2**63 + 5):
        o, r = hip.order(Pt, 300, seed=seed)
        o = o.cpu().numpy()
        assert o[0] == oracle.start_index(seed, n)
        eo, er = oracle.greedy32(P, 300, int(o[0]))
        assert_parity(o, r.cpu().numpy(), eo, er, "seed")
        o2, _ = hip.order(Pt, 40, seed=seed)
        assert np.array_equal(o2.cpu().numpy(), o[:40])


def test_k_edges(hip):
    import torch
    P = cases.random_cloud(100, 1)
    Pt = torch.from_numpy(P).cuda()
    o, r = hip.order(Pt, 0)
    assert o.numel() == 0
    o, r = run(hip, P, 1, start=42)
    assert o.tolist() == [42] and np.isinf(r[0])
    eo, er = oracle.greedy32(P, 100, 42)
    o, r = run(hip, P, 100, start=42)
    assert_parity(o, r, eo, er, "k=n")
    with pytest.raises(hip.BSError):
        hip.order(Pt, 101)


def test_nonfinite_input(hip):
    import torch
    for tune in (hip.tuning(kernel=hip.KERNEL_WG), hip.tuning(kernel=hip.KERNEL_COOP, per_thread=1)):
        P = cases.random_cloud(3000, 2)
        P[1234, 2] = np.nan
        Pt = torch.from_numpy(P).cuda()
        with pytest.raises(ValueError):
            hip.order(Pt, 50, start=0, tune=tune)
        o, r = hip.order(Pt, 50, start=0, tune=tune, check=False)
        torch.cuda.synchronize()
        assert (o.cpu().numpy() == -1).all() and np.isnan(r.cpu().numpy()).all()


def test_cooperative_cad_part_full_size(hip):
    """4,194,304 candidates ordered to k = 262,144 by the cooperative resident scan."""
    n, k = 4194304, 262144
    P = synth.cad_part(n, seed=2).points.numpy()
    st = oracle.start_index(2, n)
    o, r = run(hip, P, k, start=st, tune=hip.tuning(kernel=hip.KERNEL_COOP, block=1024, per_thread=16))
    eo, er = oracle.greedy32_grid(P, k, st)
    assert_parity(o, r, eo, er, "cad_part full")


@pytest.mark.parametrize("picks", [2, 8, 32, 64, 128, 256])
def test_cooperative_several_picks(hip, picks):
    """Several exact picks per step of the cooperative full scan (every
    workgroup a bucket with three entries and a bound on the rest): the
    same order and radii, across shapes and point sets with ties and
    duplicates."""
    n = 100000
    P = synth.cad_part(n, seed=71).points.numpy()
    eo, er = oracle.greedy32_grid(P, 20000, 23)
    for blk, pt in ((1024, 1), (1024, 2), (1024, 4), (1024, 8), (1024, 16), (512, 24), (512, 32)):
        o, r = run(hip, P, 20000, start=23,
                   tune=hip.tuning(kernel=hip.KERNEL_COOP, block=blk, per_thread=pt, picks=picks))
        assert_parity(o, r, eo, er, "cad n=%d block=%d per_thread=%d picks=%d" % (n, blk, pt, picks))
    for name in ("duplicates", "lattice", "huge", "mixed_scale", "collinear"):
        Q = cases.ADVERSARIAL[name](40000, 77)
        eo, er = oracle.greedy32_grid(Q, 40000 // 3, 5)
        for pt in (1, 4):
            o, r = run(hip, Q, 40000 // 3, start=5,
                       tune=hip.tuning(kernel=hip.KERNEL_COOP, block=1024, per_thread=pt, picks=picks))
            assert_parity(o, r, eo, er, "%s per_thread=%d picks=%d" % (name, pt, picks))


def test_cooperative_several_picks_full_size(hip):
    """4,194,304 candidates to k = 262,144, at most 32, 128 and 256 picks per step."""
    n, k = 4194304, 262144
    P = synth.cad_part(n, seed=2).points.numpy()
    st = oracle.start_index(2, n)
    eo, er = oracle.greedy32_grid(P, k, st)
    for picks in (32, 128, 256):
        o, r = run(hip, P, k, seed=2,
                   tune=hip.tuning(kernel=hip.KERNEL_COOP, block=1024, per_thread=16, picks=picks))
        assert_parity(o, r, eo, er, "cooperative several picks, full size, picks=%d" % picks)


@pytest.mark.parametrize("n,k", [(20000, 1), (20000, 2), (20000, 3), (20000, 20000), (262144, 32768),
                                 (1000003, 40000)])
def test_several_picks_automatic_plan(hip, n, k):
    """The automatic plan (several-picks cooperative scan on the most
    workgroups that fit) against the oracle: the first picks, a full order
    (every candidate chosen, the last steps with fewer live candidates than
    picks), and ragged sizes spanning many workgroups."""
    plan = hip.plan_describe(n, k)
    assert plan.kernel == hip.KERNEL_COOP and plan.groups >= 2
    assert plan.picks == (256 if plan.groups >= 64 else 128)
    P = synth.cad_part(n, seed=13).points.numpy()
    st = oracle.start_index(4, n)
    eo, er = oracle.greedy32_grid(P, k, st)
    o, r = run(hip, P, k, seed=4)
    assert_parity(o, r, eo, er, "automatic n=%d k=%d (%d x %d)" % (n, k, plan.groups, plan.per_thread))


def test_several_picks_nonfinite_input(hip):
    """A non-finite coordinate: every output entry is -1 with a NaN radius,
    as for the other kernels."""
    import torch
    P = synth.cad_part(50000, seed=3).points.numpy().copy()
    P[31337, 1] = np.inf
    Pt = torch.from_numpy(P).cuda()
    o, r = hip.order(Pt, 5000, start=0, tune=hip.tuning(kernel=hip.KERNEL_COOP, per_thread=4, picks=64),
                     check=False)
    torch.cuda.synchronize()
    assert (o.cpu().numpy() == -1).all() and np.isnan(r.cpu().numpy()).all()
    with pytest.raises(ValueError):
        hip.order(Pt, 5000, start=0, tune=hip.tuning(kernel=hip.KERNEL_COOP, per_thread=4, picks=64))


@pytest.mark.parametrize("name", sorted(cases.ADVERSARIAL))
def test_several_picks_adversarial_many_groups(hip, name):
    """The automatic plan on the adversarial point sets (duplicates, lattice
    ties, overflowing distances, mixed scales, collinear points) at a size
    spanning dozens of workgroups, and with 16 candidates per thread."""
    n, k = 120000, 15000
    Q = cases.ADVERSARIAL[name](n, 901)
    eo, er = oracle.greedy32_grid(Q, k, 11)
    o, r = run(hip, Q, k, start=11)
    assert_parity(o, r, eo, er, "%s automatic" % name)
    o, r = run(hip, Q, k, start=11, tune=hip.tuning(kernel=hip.KERNEL_COOP, block=1024, per_thread=16, picks=128))
    assert_parity(o, r, eo, er, "%s per_thread=16" % name)


def test_several_picks_one_wavefront_holds_every_entry(hip):
    """Far clumps of four points: each clump's workgroup offers three keys
    from one wavefront, so its bound R comes from that wavefront's third
    key (an entry itself) rather than from a key kept back."""
    n, k = 120000, 15000
    Q = cases.clumped_outliers(n, 23, clumps=24)
    eo, er = oracle.greedy32_grid(Q, k, 5)
    o, r = run(hip, Q, k, start=5)
    assert_parity(o, r, eo, er, "clumped automatic")
    for pt in (4, 16):
        o, r = run(hip, Q, k, start=5, tune=hip.tuning(kernel=hip.KERNEL_COOP, block=1024, per_thread=pt, picks=128))
        assert_parity(o, r, eo, er, "clumped per_thread=%d" % pt)


def test_bounded_wait_give_up_is_reported(hip):
    """A poll limit of one makes the cooperative kernels' bounded wait give
    up (forced from the host; every workgroup still leaves normally): the
    outputs become -2 / NaN, bs_order_status reports BS_ERR_TIMEOUT and the
    checked binding raises.  Without the limit the same call orders
    normally and the status is BS_OK."""
    import torch
    n, k = 262144, 6000
    P = synth.cad_part(n, seed=9).points.numpy()
    pts = torch.from_numpy(P).cuda()
    tunes = {"several picks": dict(kernel=hip.KERNEL_COOP, picks=128),
             "full scan": dict(kernel=hip.KERNEL_COOP, block=1024, per_thread=16),
             "grid with a leading scan": dict(kernel=hip.KERNEL_GRID, picks=16, lead_picks=1000)}
    eo, er = oracle.greedy32_grid(P, k, 11)
    for label, kw in tunes.items():
        print("give-up case:", label, flush=True)
        forced = hip.tuning(spin_limit=1, **kw)
        ws = torch.empty(hip.workspace_size(n, k, forced), dtype=torch.uint8, device="cuda")
        o, r = hip.order(pts, k, start=11, tune=forced, workspace=ws, check=False)
        assert hip.order_status(ws) == hip.BS_ERR_TIMEOUT, label
        o, r = o.cpu().numpy(), r.cpu().numpy()
        assert (o == -2).all() and np.isnan(r).all(), label
        with pytest.raises(hip.BSError) as err:
            hip.order(pts, k, start=11, tune=forced, workspace=ws)
        assert err.value.code == hip.BS_ERR_TIMEOUT
        # the workspace header is reset by the next call: a normal ordering
        o, r = hip.order(pts, k, start=11, tune=hip.tuning(**kw), workspace=ws)
        assert hip.order_status(ws) == hip.BS_OK
        assert_parity(o.cpu().numpy(), r.cpu().numpy(), eo, er, label + " after a give-up")


def test_order_status_nonfinite(hip):
    import torch
    P = synth.cad_part(30000, seed=4).points.numpy().copy()
    P[123, 2] = np.inf
    pts = torch.from_numpy(P).cuda()
    ws = torch.empty(hip.workspace_size(30000, 500), dtype=torch.uint8, device="cuda")
    o, r = hip.order(pts, 500, start=0, workspace=ws, check=False)
    assert hip.order_status(ws) == hip.BS_ERR_INVALID_ARG
    assert (o.cpu().numpy() == -1).all()
