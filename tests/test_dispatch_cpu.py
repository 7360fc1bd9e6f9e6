"""The serving dispatcher on a CPU stand-in device (no GPU): admission in
arrival order, budget accounting, micro-batching, overlap of jobs, and the
bound on a publication stuck behind resident workers (an in-order queue
shared by the preprocessing and the workers)."""
import ctypes
import os
import subprocess
import time

import numpy as np
import pytest

import oracle
import paper_1904_08225_amd as bs
from tests import cases, pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build(tmpdir, extra=()):
    obj = os.path.join(tmpdir, "oracle.o")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-c",
                           os.path.join(ROOT, "oracle", "bs_oracle.c"), "-o", obj, *extra])
    lib = os.path.join(tmpdir, "libfake_serve.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-pthread", *extra,
                           os.path.join(ROOT, "tests", "fake_serve_device.cpp"),
                           os.path.join(ROOT, "paper_1904_08225_amd", "csrc", "bs_dispatch.cpp"),
                           os.path.join(ROOT, "paper_1904_08225_amd", "csrc", "bs_error.cpp"), obj, "-o", lib])
    return lib


def _bind(path):
    L = ctypes.CDLL(path)
    vp, i32, i64, u64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    L.fake_server_create.argtypes = [sz, i32, i32, i32, i32, i32, i32, i32, i32]
    L.fake_server_create.restype = vp
    L.fake_server_submit.argtypes = [vp, vp, i64, i64, u64, vp, vp, ctypes.POINTER(u64)]
    L.fake_server_submit.restype = i32
    L.fake_server_wait.argtypes = [vp, u64, i64]
    L.fake_server_wait.restype = i32
    L.fake_server_poll.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_int)]
    L.fake_server_poll.restype = i32
    L.fake_server_drain.argtypes = [vp, i64]
    L.fake_server_drain.restype = i32
    L.fake_server_stats.argtypes = [vp, vp]
    L.fake_server_stats.restype = i32
    L.fake_server_stall_stops.argtypes = [vp]
    L.fake_server_stall_stops.restype = i64
    L.fake_server_launches.argtypes = [vp]
    L.fake_server_launches.restype = i64
    L.fake_server_take_peak.argtypes = [vp]
    L.fake_server_take_peak.restype = i32
    L.fake_server_destroy.argtypes = [vp]
    L.fake_server_destroy.restype = None
    return L


@pytest.fixture(scope="module")
def fake(tmp_path_factory):
    return _bind(_build(str(tmp_path_factory.mktemp("fake"))))


class _Srv:
    def __init__(self, L, budget, per_batch=64, workers=2, shared=False, delay_us=0, stall_us=2000, bpc=100,
                 idle_ms=2000, exit_us=0):
        self.L = L
        self.h = L.fake_server_create(budget, per_batch, workers, int(shared), delay_us, stall_us, bpc, idle_ms,
                                      exit_us)
        assert self.h
        self.keep = {}

    def submit(self, P, k, seed):
        o = np.full(max(k, 1), -9, np.int32)
        r = np.zeros(max(k, 1), np.float32)
        t = ctypes.c_uint64()
        rc = self.L.fake_server_submit(self.h, P.ctypes.data_as(ctypes.c_void_p), P.shape[0], k, seed,
                                       o.ctypes.data_as(ctypes.c_void_p), r.ctypes.data_as(ctypes.c_void_p),
                                       ctypes.byref(t))
        self.keep[t.value] = (P, o, r)
        return rc, t.value

    def wait(self, t, timeout_us=30_000_000):
        return self.L.fake_server_wait(self.h, t, timeout_us)

    def done(self, t):
        d = ctypes.c_int()
        self.L.fake_server_poll(self.h, t, ctypes.byref(d))
        return bool(d.value)

    def stats(self):
        st = bs.ServingStats()
        assert self.L.fake_server_stats(self.h, ctypes.byref(st)) == 0
        return st.as_dict()

    def close(self):
        self.L.fake_server_destroy(self.h)


def test_results_equal_oracle_and_batches(fake):
    srv = _Srv(fake, budget=10**9, per_batch=7, workers=3)
    jobs = []
    for i in range(30):
        n = 50 + 97 * i
        P = cases.random_cloud(n, 100 + i)
        k = 0 if i == 5 else max(1, n // 4)
        rc, t = srv.submit(P, k, 11 * i + 1)
        assert rc == 0
        jobs.append((t, P, k, 11 * i + 1))
    for t, P, k, seed in jobs:
        assert srv.wait(t) == 0
        if k:
            eo, er = oracle.greedy32(P, k, oracle.start_index(seed, P.shape[0]))
            _, o, r = srv.keep[t]
            assert np.array_equal(o[:k], eo) and pins.same_f32(r[:k], er)
    st = srv.stats()
    assert st["completed"] == 30 and st["admitted"] == 30 and st["rejected"] == 0
    assert st["batches"] >= 29 // 7          # at most 7 jobs per micro-batch
    assert st["hbm_in_use"] == 0
    srv.close()


def test_budget_accounting_and_rejection(fake):
    bpc = 100
    budget = 450_000                          # room for two 2,000-candidate jobs at a time
    srv = _Srv(fake, budget=budget, per_batch=64, workers=2, bpc=bpc)
    P = cases.random_cloud(2000, 5)
    ts = []
    for i in range(10):
        rc, t = srv.submit(P, 500, i)
        assert rc == 0
        ts.append(t)
    for t in ts:
        assert srv.wait(t) == 0
    st = srv.stats()
    assert st["hbm_peak"] <= budget and st["hbm_peak"] >= 2000 * bpc
    # the estimate (64 B per candidate) lets this one in, its exact plan (100 B) never fits
    Q = cases.random_cloud(6000, 6)
    rc, t = srv.submit(Q, 10, 1)
    assert rc == 0 and srv.wait(t) == bs.BS_ERR_OVER_BUDGET
    # the estimate alone is over the budget: refused at submit
    R = cases.random_cloud(8000, 7)
    rc, _ = srv.submit(R, 10, 1)
    assert rc == bs.BS_ERR_OVER_BUDGET
    st = srv.stats()
    assert st["rejected"] == 2 and st["completed"] == 10
    srv.close()


def test_later_job_finishes_while_earlier_runs(fake):
    srv = _Srv(fake, budget=10**9, workers=2)
    A = cases.random_cloud(60000, 1)
    rc, ta = srv.submit(A, 3000, 1)          # long: about a second on the host
    time.sleep(0.05)
    B = cases.random_cloud(300, 2)
    rc, tb = srv.submit(B, 100, 2)
    assert srv.wait(tb, 20_000_000) == 0
    assert not srv.done(ta), "the short job waited for the long one"
    assert srv.wait(ta) == 0
    srv.close()


@pytest.mark.parametrize("stall_us", [2000, 10_000_000])
def test_publication_behind_workers_is_bounded(fake, stall_us):
    """Shared queue: a batch admitted while the workers run cannot publish
    until they leave.  With the stall rule the dispatcher stops them once the
    publication is overdue, so the late job finishes right after the running
    one; without it (stall_us huge) it waits for the workers' idle time-out."""
    idle_ms = 1500
    srv = _Srv(fake, budget=10**9, workers=2, shared=True, stall_us=stall_us, idle_ms=idle_ms)
    A = cases.random_cloud(30000, 3)
    t0 = time.perf_counter()
    rc, ta = srv.submit(A, 2000, 1)
    time.sleep(0.05)                         # A is claimed and running
    B = cases.random_cloud(300, 4)
    rc, tb = srv.submit(B, 50, 2)
    assert srv.wait(ta) == 0
    ta_done = time.perf_counter() - t0
    assert srv.wait(tb) == 0
    tb_done = time.perf_counter() - t0
    stops = fake.fake_server_stall_stops(srv.h)
    srv.close()
    if stall_us < 1_000_000:
        assert stops >= 1
        assert tb_done < ta_done + 0.3, (ta_done, tb_done)
    else:
        assert stops == 0
        assert tb_done > ta_done + 0.8 * idle_ms / 1e3, (ta_done, tb_done)


def test_slow_preprocessing_is_not_a_stall(fake):
    """Preprocessing that takes long once it has begun (large batches, pool
    growth) is not a stall: with its own queue a 300 ms publication delay,
    far above stall_us, stops no workers."""
    srv = _Srv(fake, budget=10**9, workers=2, shared=False, delay_us=300_000, stall_us=2000)
    A = cases.random_cloud(30000, 3)
    rc, ta = srv.submit(A, 2000, 1)
    time.sleep(0.4)                          # A is published and running
    B = cases.random_cloud(300, 4)
    rc, tb = srv.submit(B, 50, 2)
    assert srv.wait(tb) == 0 and srv.wait(ta) == 0
    stops = fake.fake_server_stall_stops(srv.h)
    srv.close()
    assert stops == 0


def test_full_worker_set_after_each_stop(fake):
    """Rounds of four equal jobs, each round submitted as the last one ends:
    the dispatcher then stops the idle workers, and they notice it at
    staggered times.  No round may start while some of them are still
    leaving (the survivors would claim the whole round and no full set could
    start until the last of them left): every round must run four jobs at
    once.  (A dispatcher that admitted while the workers were leaving ran
    the rounds on 4, 3, 1, 1 and 1 workers here.)"""
    workers = 4
    srv = _Srv(fake, budget=10**9, per_batch=64, workers=workers, exit_us=30_000, idle_ms=5000)
    P = [cases.random_cloud(20000, 40 + i) for i in range(workers)]
    peaks = []
    for r in range(5):
        fake.fake_server_take_peak(srv.h)
        ts = [srv.submit(P[i], 1500, 10 * r + i)[1] for i in range(workers)]
        for t in ts:
            assert srv.wait(t) == 0
        peaks.append(fake.fake_server_take_peak(srv.h))
    for i in range(workers):  # outputs of the last round
        eo, er = oracle.greedy32(P[i], 1500, oracle.start_index(40 + i, P[i].shape[0]))
        _, o, r = srv.keep[ts[i]]
        assert np.array_equal(o[:1500], eo)
    launches = fake.fake_server_launches(srv.h)
    srv.close()
    assert peaks == [workers] * 5, peaks
    assert launches == 5


def test_dispatcher_under_sanitizers(tmp_path):
    """The dispatcher, fake device and oracle built with AddressSanitizer and
    UndefinedBehaviorSanitizer (host code only), driven through a short mixed
    scenario in a child process: any heap error or undefined behaviour fails."""
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    lib = _build(str(tmp_path), extra=("-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g"))
    script = (
        "import sys, ctypes, numpy as np\n"
        "sys.path.insert(0, %r)\n"
        "from tests import test_dispatch_cpu as T, cases\n"
        "L = T._bind(%r)\n"
        "s = T._Srv(L, budget=450000, per_batch=3, workers=2, shared=True, stall_us=1000, idle_ms=500)\n"
        "ts = [s.submit(cases.random_cloud(200 + 300 * i, i), 40, i)[1] for i in range(8)]\n"
        "rc, bad = s.submit(cases.random_cloud(8000, 9), 10, 1)\n"
        "assert rc == -4\n"
        "assert all(s.wait(t) == 0 for t in ts)\n"
        "s.close()\n"
        "print('sanitized run ok')\n") % (ROOT, lib)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = subprocess.run(["python", "-c", script], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0 and "sanitized run ok" in out.stdout, out.stdout[-2000:] + out.stderr[-4000:]
