"""The C-ABI library loads and exports what include/bluesurfels.h declares;
host-side logic (start index, argument validation) works without a GPU."""
import ctypes
import os

import pytest

import oracle
import paper_1904_08225_amd as bs


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(bs.LIB_PATH):
        from paper_1904_08225_amd import build
        build.build()
    return bs.load()


def test_exports_every_declared_function(lib):
    names = bs.header_functions()
    assert "bs_order" in names and "bs_order_ex" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_start_index_matches_splitmix64(lib):
    for n in (1, 2, 3, 1000, 16384, 4194304, 2**31 - 1):
        for seed in (0, 1, 2, 3, 99, 2**63, 2**64 - 1):
            assert bs.start_index(seed, n) == oracle.start_index(seed, n)
    assert bs.start_index(5, 0) == -1


def test_argument_validation_without_device(lib):
    vp = ctypes.c_void_p
    fake = vp(0x1000)
    # k == 0 is a no-op even with null pointers
    assert lib.bs_order(None, None, None, 10, 0, 0, None, None, None) == bs.BS_OK
    assert lib.bs_order(fake, None, None, 10, -1, 0, fake, None, None) == bs.BS_ERR_INVALID_ARG
    assert lib.bs_order_ex(fake, None, None, 10, 11, 0, -1, fake, None, fake, 1 << 20, None, None) == bs.BS_ERR_INVALID_ARG
    assert "k=11 > n=10" in bs.last_error()
    assert lib.bs_order_ex(None, None, None, 10, 5, 0, -1, fake, None, fake, 1 << 20, None, None) == bs.BS_ERR_INVALID_ARG
    assert lib.bs_order_ex(fake, None, None, 10, 5, 0, 10, fake, None, fake, 1 << 20, None, None) == bs.BS_ERR_INVALID_ARG
    assert lib.bs_order_ex(fake, None, None, 0, 5, 0, -1, fake, None, fake, 1 << 20, None, None) == bs.BS_ERR_INVALID_ARG
    assert lib.bs_order_ex(fake, None, None, 2**31, 5, 0, -1, fake, None, fake, 1 << 20, None, None) == bs.BS_ERR_INVALID_ARG
    bad = bs.Tuning()
    bad.reserved[0] = 1
    assert lib.bs_order_ex(fake, None, None, 10, 5, 0, -1, fake, None, fake, 1 << 20, ctypes.byref(bad), None) == bs.BS_ERR_INVALID_ARG
    # too small workspace is rejected before anything is enqueued
    assert lib.bs_order_ex(fake, None, None, 10, 5, 0, -1, fake, None, fake, 16, None, None) == bs.BS_ERR_INVALID_ARG
    assert lib.bs_workspace_size(10, 11, None) == 0
    assert lib.bs_workspace_size(16384, 16384, None) > 0
    assert bs.error_string(bs.BS_ERR_OVER_BUDGET) == "BS_ERR_OVER_BUDGET"


def test_batch_plan_validation_without_device(lib):
    import numpy as np
    plan = ctypes.c_void_p()
    offs = np.array([0, 5, 3], dtype=np.int64)   # decreasing
    ks = np.array([1, 1], dtype=np.int64)
    vp = ctypes.c_void_p
    rc = lib.bs_batch_plan_create(offs.ctypes.data_as(vp), ks.ctypes.data_as(vp), None, 2, None, ctypes.byref(plan))
    assert rc == bs.BS_ERR_INVALID_ARG
    offs = np.array([0, 5, 9], dtype=np.int64)
    ks = np.array([6, 1], dtype=np.int64)         # k > n
    rc = lib.bs_batch_plan_create(offs.ctypes.data_as(vp), ks.ctypes.data_as(vp), None, 2, None, ctypes.byref(plan))
    assert rc == bs.BS_ERR_INVALID_ARG and "k=6" in bs.last_error()
    offs = np.array([1, 5], dtype=np.int64)       # offsets[0] != 0
    ks = np.array([1], dtype=np.int64)
    rc = lib.bs_batch_plan_create(offs.ctypes.data_as(vp), ks.ctypes.data_as(vp), None, 1, None, ctypes.byref(plan))
    assert rc == bs.BS_ERR_INVALID_ARG
    offs = np.array([0, 5], dtype=np.int64)       # negative count of wide workgroups
    t = bs.tuning(groups=-1)
    rc = lib.bs_batch_plan_create(offs.ctypes.data_as(vp), ks.ctypes.data_as(vp), None, 1, ctypes.byref(t),
                                  ctypes.byref(plan))
    assert rc == bs.BS_ERR_INVALID_ARG
    t = bs.tuning(picks=33)                       # more picks per round than the grid kernel takes
    rc = lib.bs_batch_plan_create(offs.ctypes.data_as(vp), ks.ctypes.data_as(vp), None, 1, ctypes.byref(t),
                                  ctypes.byref(plan))
    assert rc == bs.BS_ERR_UNSUPPORTED and "picks" in bs.last_error()


def test_server_config_validation_without_device(lib):
    cfg = bs.ServerConfig(0, 0, 4, 16, 50, 0.0)
    srv = ctypes.c_void_p()
    assert lib.bs_server_create(ctypes.byref(cfg), ctypes.byref(srv)) == bs.BS_ERR_INVALID_ARG
    cfg = bs.ServerConfig(1 << 30, 0, 4, 16, 50, 0.0)
    cfg.reserved[2] = 5
    assert lib.bs_server_create(ctypes.byref(cfg), ctypes.byref(srv)) == bs.BS_ERR_INVALID_ARG


def test_autotune_validation_without_device(lib):
    fake = ctypes.c_void_p(0x1000)
    t = bs.Tuning()
    assert lib.bs_autotune(None, 10, 5, 0, ctypes.byref(t), None) == bs.BS_ERR_INVALID_ARG
    assert lib.bs_autotune(fake, 10, 0, 0, ctypes.byref(t), None) == bs.BS_ERR_INVALID_ARG
    assert lib.bs_autotune(fake, 10, 11, 0, ctypes.byref(t), None) == bs.BS_ERR_INVALID_ARG
    assert lib.bs_autotune(fake, 10, 5, 0, None, None) == bs.BS_ERR_INVALID_ARG
    # nothing tuned (and no device): the lookup reports not ready
    lib.bs_autotune_clear()
    assert lib.bs_autotune_lookup(4096, 100, ctypes.byref(t)) == bs.BS_ERR_NOT_READY
    assert lib.bs_batch_autotune(None, None, None, 0, fake, ctypes.byref(t), None) == bs.BS_ERR_INVALID_ARG
    # tuning fields: picks outside 0..128 is rejected like the reserved words;
    # the grid kernel takes at most 32 per round
    assert lib.bs_workspace_size(1000, 10, ctypes.byref(bs.tuning(kernel=3, picks=129))) == 0
    assert lib.bs_workspace_size(1000, 10, ctypes.byref(bs.tuning(kernel=3, picks=33))) == 0
    assert lib.bs_workspace_size(1000, 10, ctypes.byref(bs.tuning(kernel=3, picks=16))) > 0


def test_lead_picks_validation(lib):
    """lead_picks: -1 (none) and 0 (auto) are accepted, below -1 rejected; an
    explicit lead needs a cooperative scan that holds n (n = 10,000 fits one
    workgroup, so no cooperative shape exists)."""
    ws = lambda n, k, t: lib.bs_workspace_size(n, k, ctypes.byref(t))
    assert ws(1000, 10, bs.tuning(kernel=3, picks=16, lead_picks=-2)) == 0
    assert ws(1000, 10, bs.tuning(kernel=3, picks=16, lead_picks=-1)) > 0
    assert ws(1000, 10, bs.tuning(kernel=3, picks=16, lead_picks=0)) > 0
    assert ws(10000, 1000, bs.tuning(kernel=3, picks=16, lead_picks=100)) == 0
    assert ws(100000, 1000, bs.tuning(kernel=3, picks=16, lead_picks=100)) > 0
    # one pick per round ignores the lead
    assert ws(10000, 1000, bs.tuning(kernel=3, picks=1, lead_picks=100)) > 0
    # the struct keeps its size: 12 words
    assert ctypes.sizeof(bs.Tuning) == 48


def test_plan_describe(lib):
    """Automatic choices resolved: up to 256 workgroups of 1024 threads, the
    several-picks cooperative scan with 256 picks per step on the most
    workgroups that fit (fewest candidates per thread); above 4,194,304 the
    grid kernel with 16 picks per round (asked for at 4,194,304: with a
    leading scan of n / 1024 picks); up to 4,096 the resident workgroup."""
    lib.bs_autotune_clear()
    p = bs.plan_describe(4194304, 262144)
    assert (p.kernel, p.block, p.per_thread, p.groups, p.picks) == (bs.KERNEL_COOP, 1024, 16, 256, 256)
    p = bs.plan_describe(2097152, 1000)
    assert (p.kernel, p.per_thread, p.groups, p.picks) == (bs.KERNEL_COOP, 8, 256, 256)
    p = bs.plan_describe(100000, 1000)
    assert (p.kernel, p.per_thread, p.groups) == (bs.KERNEL_COOP, 1, 98)
    p = bs.plan_describe(500000, 1000)
    assert (p.kernel, p.per_thread, p.groups) == (bs.KERNEL_COOP, 2, 245)
    p = bs.plan_describe(100000, 1000, bs.tuning(kernel=2, per_thread=16, picks=8))
    assert (p.kernel, p.per_thread, p.groups, p.picks) == (bs.KERNEL_COOP, 16, 7, 8)
    p = bs.plan_describe(8000000, 262144)
    assert (p.kernel, p.block, p.picks, p.lead_picks) == (bs.KERNEL_GRID, 1024, 16, -1)  # no cooperative shape holds 8M
    p = bs.plan_describe(4194304, 262144, bs.tuning(kernel=3, picks=16))
    assert (p.kernel, p.block, p.picks, p.lead_picks) == (bs.KERNEL_GRID, 1024, 16, 4096)
    assert (p.per_thread, p.groups) == (16, 256)
    p = bs.plan_describe(4194304, 262144, bs.tuning(kernel=3, picks=16, lead_picks=-1))
    assert p.lead_picks == -1 and p.groups == 0
    p = bs.plan_describe(4194304, 2000, bs.tuning(kernel=3, picks=16))
    assert p.lead_picks == 2000  # capped at k
    p = bs.plan_describe(10000, 100)  # from two workgroups on, the several-picks scan
    assert (p.kernel, p.per_thread, p.groups, p.picks) == (bs.KERNEL_COOP, 1, 10, 128)  # few workgroups: 128
    p = bs.plan_describe(4096, 100)
    assert p.kernel == bs.KERNEL_WG and p.groups == 1
    # several picks per step need two workgroups at least
    with pytest.raises(Exception):
        bs.plan_describe(1000, 100, bs.tuning(kernel=2, picks=8))  # one workgroup even at 1 per thread
    out = bs.Tuning()
    assert lib.bs_plan_describe(10, 11, None, ctypes.byref(out)) == bs.BS_ERR_INVALID_ARG
    assert lib.bs_plan_describe(10, 5, None, None) == bs.BS_ERR_INVALID_ARG


def test_forced_kernel_override(lib, monkeypatch):
    """BS_FORCE_KERNEL replaces the automatic choice of calls that pass no
    tuning; an explicit tuning still wins, and an unknown value is an error."""
    lib.bs_autotune_clear()
    for name, kernel, picks in (("wg", bs.KERNEL_WG, None), ("scan", bs.KERNEL_COOP, 1),
                                ("several", bs.KERNEL_COOP, 256), ("grid", bs.KERNEL_GRID, 16)):
        monkeypatch.setenv("BS_FORCE_KERNEL", name)
        n = 4000 if name == "wg" else 100000
        p = bs.plan_describe(n, 1000)
        assert p.kernel == kernel, name
        if picks is not None:
            assert p.picks == picks, name
    monkeypatch.setenv("BS_FORCE_KERNEL", "grid")
    p = bs.plan_describe(100000, 1000, bs.tuning(kernel=2, per_thread=16, picks=8))
    assert p.kernel == bs.KERNEL_COOP and p.picks == 8
    monkeypatch.setenv("BS_FORCE_KERNEL", "fastest")
    out = bs.Tuning()
    assert lib.bs_plan_describe(100000, 1000, None, ctypes.byref(out)) == bs.BS_ERR_INVALID_ARG
    assert b"BS_FORCE_KERNEL" in lib.bs_last_error_message()
    monkeypatch.delenv("BS_FORCE_KERNEL")
    p = bs.plan_describe(100000, 1000)
    assert (p.kernel, p.per_thread, p.groups) == (bs.KERNEL_COOP, 1, 98)


def test_prefix_host_functions(lib):
    """bs_prefix_length equals the oracle's formula; bs_prefix_for_radius
    equals a linear scan over the oracle's radii (least t >= 1 with
    radius[t] <= r, else k); argument errors of bs_emit_surfels."""
    import numpy as np
    import oracle
    from tests import cases
    for r, rm, pm, k in ((0.1, 0.1, 1000, 10**6), (0.05, 0.1, 1000, 10**6), (0.3, 0.1, 1000, 10**6),
                         (1e-4, 0.1, 1000, 5000), (7.0, 0.1, 1000, 5000), (0.0, 0.1, 1000, 77), (0.02, 0.013, 250, 900)):
        assert bs.prefix_length(r, rm, pm, k) == oracle.prefix_length(r, rm, pm, k)
    P = cases.random_cloud(3000, 5)
    o, rad = oracle.greedy32(P, 800, 2)
    for r in (1e9, float(rad[1]), float(rad[57]), float(rad[57]) * 1.0001, float(rad[799]), float(rad[799]) * 0.5, 0.0):
        ok = [t for t in range(1, 800) if rad[t] <= r]
        assert bs.prefix_for_radius(rad, r) == (ok[0] if ok else 800)
    assert bs.prefix_for_radius(rad[:1], 0.0) == 1
    fake = ctypes.c_void_p(0x1000)
    assert lib.bs_emit_surfels(fake, None, None, 10, fake, -1, fake, None) == bs.BS_ERR_INVALID_ARG
    assert lib.bs_emit_surfels(None, None, None, 10, fake, 5, fake, None) == bs.BS_ERR_INVALID_ARG
    assert lib.bs_emit_surfels(None, None, None, 0, None, 0, None, None) == bs.BS_OK
    assert lib.bs_prefix_median_nn(fake, 10, fake, 1, fake, None) == bs.BS_ERR_INVALID_ARG
    assert lib.bs_prefix_median_nn(fake, 5000, fake, 4097, fake, None) == bs.BS_ERR_INVALID_ARG


def test_hier_plan_validation_on_cpu():
    """Plan creation is host-only: its checks and output offsets."""
    import paper_1904_08225_amd as bs
    bs.load()
    with pytest.raises(bs.BSError):
        bs.HierPlan([1, -1], [0, 10, 10], [3, 4])          # parent 1 has 3 candidates
    with pytest.raises(bs.BSError):
        bs.HierPlan([-1, 0], [0, 10, 20], [3, 1])          # a parent before its child
    with pytest.raises(bs.BSError):
        bs.HierPlan([2, 2, -1], [0, 10, 20, 25], [3, 3, 2])  # rows for an inner node
    p = bs.HierPlan([2, 2, -1], [0, 10, 20, 20], [3, 4, 7], [1, 2, 3])
    assert p.total_k == 14 and p.out_offsets.tolist() == [0, 3, 7, 14]
    assert p.workspace_bytes > 0
    p.close()
