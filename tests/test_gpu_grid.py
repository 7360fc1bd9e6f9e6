"""GPU parity of the uniform-grid radius-pruned kernel against the CPU oracle.

The pruning must not change a single bit: orders and radii equal the plain
oracle's (small cases) or the exact grid oracle's (large cases, itself
pinned bit-exact to the plain oracle).  Both forms of the kernel are
covered: one pick per round (picks=1) and several exact picks per round
(picks=2..16, the default).
"""
import numpy as np
import pytest

import oracle
import synth
from tests import cases
from tests.test_gpu_scan import assert_parity, run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("picks", [1, 16])
@pytest.mark.parametrize("block", [256, 512, 1024])
@pytest.mark.parametrize("name", sorted(cases.ADVERSARIAL))
def test_grid_adversarial(hip, name, block, picks):
    for n in (1, 2, 3, 65, 1000, 4097):
        P = cases.ADVERSARIAL[name](n, 41 + n)
        st = (5 * n) // 7
        eo, er = oracle.greedy32(P, n, st)
        o, r = run(hip, P, n, start=st, tune=hip.tuning(kernel=hip.KERNEL_GRID, block=block, picks=picks))
        assert_parity(o, r, eo, er, "grid %s n=%d block=%d picks=%d" % (name, n, block, picks))


@pytest.mark.parametrize("picks", [2, 3, 7, 16, 24, 32])
def test_grid_picks_per_round(hip, picks):
    """Every read-ahead limit gives the same order (several superblock sizes)."""
    for n, cp in ((50000, 32.0), (20000, 4.0), (3000, 1.0)):
        P = synth.cad_part(n, seed=60 + n % 7).points.numpy()
        k = n // 2
        eo, er = oracle.greedy32_grid(P, k, 11)
        for block in (256, 512, 1024):
            o, r = run(hip, P, k, start=11,
                       tune=hip.tuning(kernel=hip.KERNEL_GRID, block=block, cell_points=cp, picks=picks))
            assert_parity(o, r, eo, er, "n=%d cell=%g block=%d picks=%d" % (n, cp, block, picks))


@pytest.mark.parametrize("cell_points", [1.0, 4.0, 32.0, 200.0])
def test_grid_cell_sizes(hip, cell_points):
    n = 30000
    P = synth.cad_part(n, seed=12).points.numpy()
    k = n // 3
    eo, er = oracle.greedy32_grid(P, k, 17)
    for block in (256, 512, 1024):
        o, r = run(hip, P, k, start=17,
                   tune=hip.tuning(kernel=hip.KERNEL_GRID, block=block, cell_points=cell_points))
        assert_parity(o, r, eo, er, "cell_points=%g block=%d" % (cell_points, block))


def test_grid_sphere_box_full_order(hip):
    s = synth.sphere_and_box(n=16384, seed=1)
    P = s.points.numpy()
    st = oracle.start_index(1, P.shape[0])
    eo, er = oracle.greedy32(P, 16384, st)
    o, r = run(hip, P, 16384, start=st, tune=hip.tuning(kernel=hip.KERNEL_GRID))
    assert_parity(o, r, eo, er, "grid sphere_and_box")


def test_grid_many_duplicates_and_ties(hip):
    # 40 distinct positions repeated: long runs of zero-distance picks
    P = cases.with_duplicates(20000, 5, groups=40)
    eo, er = oracle.greedy32_grid(P, 20000, 7)
    o, r = run(hip, P, 20000, start=7, tune=hip.tuning(kernel=hip.KERNEL_GRID))
    assert_parity(o, r, eo, er, "duplicates")
    L = cases.integer_lattice(30, 30, 30)
    eo, er = oracle.greedy32_grid(L, 27000, 0)
    o, r = run(hip, L, 27000, start=0, tune=hip.tuning(kernel=hip.KERNEL_GRID))
    assert_parity(o, r, eo, er, "lattice ties")


def test_grid_nonfinite(hip):
    import torch
    P = cases.random_cloud(50000, 2)
    P[777, 0] = np.inf
    Pt = torch.from_numpy(P).cuda()
    o, r = hip.order(Pt, 100, start=0, tune=hip.tuning(kernel=hip.KERNEL_GRID), check=False)
    torch.cuda.synchronize()
    assert (o.cpu().numpy() == -1).all() and np.isnan(r.cpu().numpy()).all()


def test_grid_repeat_and_agrees_with_resident(hip):
    n = 16000
    P = synth.cad_part(n, seed=21).points.numpy()
    a = run(hip, P, 4000, start=3, tune=hip.tuning(kernel=hip.KERNEL_WG))
    for _ in range(2):
        b = run(hip, P, 4000, start=3, tune=hip.tuning(kernel=hip.KERNEL_GRID))
        assert_parity(b[0], b[1], a[0], a[1], "grid vs resident")


def test_grid_cad_part_full_size(hip):
    """4,194,304 candidates to k = 262,144 through the grid kernel (16 picks
    per round after a leading scan of n / 1024 picks), through the automatic
    choice (the several-picks cooperative scan), and with one pick per round."""
    n, k = 4194304, 262144
    P = synth.cad_part(n, seed=2).points.numpy()
    st = oracle.start_index(2, n)
    o, r = run(hip, P, k, seed=2, tune=hip.tuning(kernel=hip.KERNEL_GRID))
    eo, er = oracle.greedy32_grid(P, k, st)
    assert_parity(o, r, eo, er, "grid cad_part full")
    assert hip.auto_kernel(n, k) == hip.KERNEL_COOP
    o, r = run(hip, P, k, seed=2)
    assert_parity(o, r, eo, er, "automatic cad_part full")
    o1, r1 = run(hip, P, k, seed=2, tune=hip.tuning(kernel=hip.KERNEL_GRID, picks=1))
    assert_parity(o1, r1, eo, er, "grid cad_part full, one pick per round")


@pytest.mark.parametrize("picks", [1, 16])
def test_grid_overflowing_distances(hip, picks):
    """Coordinates ~1e19: most squared distances are +inf, so a pick's ball
    reaches no box and whole blocks are never updated; their entries must
    still come from the grid build (regression: n = 23,004 read unset LDS)."""
    for n, seed in ((23004, 806), (60000, 807)):
        P = cases.huge_coords(n, seed)
        eo, er = oracle.greedy32_grid(P, n // 3, 5)
        for block in (256, 512, 1024):
            o, r = run(hip, P, n // 3, start=5,
                       tune=hip.tuning(kernel=hip.KERNEL_GRID, block=block, picks=picks))
            assert_parity(o, r, eo, er, "huge n=%d block=%d picks=%d" % (n, block, picks))


@pytest.mark.parametrize("name", ["random", "duplicates", "huge", "mixed_scale", "lattice"])
def test_grid_lead_scan_handoff(hip, name):
    """A leading cooperative full scan hands its distances to the grid kernel
    after 2, 3, 100, k-1 or k picks: the same order and radii."""
    n = 40000
    P = cases.ADVERSARIAL[name](n, 900)
    k = n // 2
    eo, er = oracle.greedy32_grid(P, k, 13)
    for lead in (2, 3, 100, k - 1, k):
        for block in (512, 1024):
            o, r = run(hip, P, k, start=13,
                       tune=hip.tuning(kernel=hip.KERNEL_GRID, block=block, picks=16, lead_picks=lead))
            assert_parity(o, r, eo, er, "%s lead=%d block=%d" % (name, lead, block))


def test_grid_lead_scan_cad_part(hip):
    """n = 300,000 (automatic lead of n / 1024 picks) and explicit leads, with
    several read-ahead limits and cell sizes."""
    n, k = 300000, 30000
    P = synth.cad_part(n, seed=33).points.numpy()
    eo, er = oracle.greedy32_grid(P, k, 101)
    for lead, picks, block, cp in ((0, 16, 1024, 0.0), (5000, 16, 1024, 0.0), (700, 2, 512, 4.0),
                                   (29999, 7, 256, 16.0), (-1, 16, 1024, 0.0), (3000, 1, 512, 0.0)):
        o, r = run(hip, P, k, start=101,
                   tune=hip.tuning(kernel=hip.KERNEL_GRID, block=block, picks=picks, cell_points=cp,
                                   lead_picks=lead))
        assert_parity(o, r, eo, er, "lead=%d picks=%d block=%d cells=%g" % (lead, picks, block, cp))
