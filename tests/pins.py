"""Checks that pin the CPU oracle to facts other than itself.

Each check takes an oracle implementation (the default library or a planted
mutant compiled from a modified copy of its source) and raises
AssertionError on failure.  The reference values come from the paper's
definition worked by hand (tests/golden/closed_forms.json), from an
independent numpy reformulation, from exhaustive search, or from
mathematical invariants -- never from the oracle itself.
"""
import itertools
import json
import math
import os

import numpy as np

import oracle
from tests import cases

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "closed_forms.json")


def load_golden():
    with open(GOLDEN) as f:
        return json.load(f)


# ---------------------------------------------------------------- brute force

def brute_greedy_f32(P, k, start):
    """From-scratch numpy binary32 greedy.

    Each step rebuilds the whole candidate-by-prefix distance matrix with
    the association ((dx*dx + dy*dy) + dz*dz) (numpy evaluates each binary
    float32 op separately, correctly rounded, without contraction), takes
    the row minimum, and the first maximal live row."""
    P = np.asarray(P, dtype=np.float32)
    n = P.shape[0]
    order = [start]
    rad = [np.float32(np.inf)]
    for _ in range(1, k):
        Q = P[np.array(order)]
        dx = P[:, None, 0] - Q[None, :, 0]
        dy = P[:, None, 1] - Q[None, :, 1]
        dz = P[:, None, 2] - Q[None, :, 2]
        d2 = (dx * dx + dy * dy) + dz * dz
        m = d2.min(axis=1)
        live = np.ones(n, dtype=bool)
        live[order] = False
        cand = np.where(live, m, np.float32(-1.0))
        c = int(np.argmax(cand))
        order.append(c)
        rad.append(np.sqrt(m[c]))
    return np.array(order, dtype=np.int32), np.array(rad, dtype=np.float32)


def same_f32(a, b):
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    return a.shape == b.shape and bool(np.all(a.view(np.uint32) == b.view(np.uint32)))


def check_bruteforce(lib=None, sizes=(1, 2, 3, 5, 9, 17, 40, 64)):
    for name, gen in cases.ADVERSARIAL.items():
        for n in sizes:
            P = gen(n, 100 + n)
            starts = range(n) if n <= 9 else (0, n // 2, n - 1)
            for s in starts:
                o, r = oracle.greedy32(P, n, s, lib=lib)
                bo, br = brute_greedy_f32(P, n, s)
                assert np.array_equal(o, bo), (name, n, s, o, bo)
                assert same_f32(r, br), (name, n, s, r, br)


def check_closed_forms(lib=None):
    g = load_golden()
    for case in g["cases"]:
        P = np.array(case["points"], dtype=np.float32)
        n = P.shape[0]
        exp_o = np.array(case["order"], dtype=np.int32)
        exp_r = np.array([np.inf if v == "inf" else math.sqrt(v) for v in case["radius_squared"]],
                         dtype=np.float32)
        for fn in (oracle.greedy32, oracle.greedy32_grid):
            o, r = fn(P, n, case["start"], lib=lib)
            assert np.array_equal(o, exp_o), (case["name"], fn.__name__, o)
            assert same_f32(r, exp_r), (case["name"], fn.__name__, r)
        o64, r64 = oracle.greedy64(P, n, case["start"], lib=lib)
        assert np.array_equal(o64, exp_o), (case["name"], "greedy64", o64)
        exp64 = np.array([math.sqrt(v) for v in case["radius_squared"][1:]])
        assert np.allclose(r64[1:], exp64, rtol=1e-15, atol=0)
        # prefixes: same order for every k
        for k in range(n + 1):
            o, r = oracle.greedy32(P, k, case["start"], lib=lib)
            assert np.array_equal(o, exp_o[:k])
    sm = g["splitmix64"]
    assert oracle.splitmix64_first(sm["seed"], lib=lib) == int(sm["first"], 16)


# ----------------------------------------------------------------- invariants

def nearest_prefix_d2_f32(P, prefix_idx, query_idx):
    """binary32 min over the prefix of d2(query, prefix point) (numpy)."""
    Q = P[prefix_idx]
    X = P[query_idx]
    dx = X[:, None, 0] - Q[None, :, 0]
    dy = X[:, None, 1] - Q[None, :, 1]
    dz = X[:, None, 2] - Q[None, :, 2]
    return ((dx * dx + dy * dy) + dz * dz).min(axis=1)


def check_invariants(P, order, radius, steps=None):
    """Exact binary32 properties of a greedy permutation prefix.

    - radius is non-increasing after the first two entries;
    - packing: every pair inside the (t+1)-prefix is at least radius[t] apart;
    - covering + greediness: at step t the farthest non-picked candidate
      (first one on ties) from the t-prefix is order[t], at radius[t].
    """
    P = np.asarray(P, dtype=np.float32)
    n = P.shape[0]
    k = len(order)
    assert len(set(order.tolist())) == k, "order repeats a candidate"
    assert np.all((order >= 0) & (order < n))
    if k >= 1:
        assert np.isinf(radius[0]) and radius[0] > 0
    if k >= 3:
        assert np.all(radius[2:] <= radius[1:-1]), "radius increased"
    if steps is None:
        steps = range(1, k)
    for t in steps:
        if t < 1 or t >= k:
            continue
        pre = order[:t]
        live = np.ones(n, dtype=bool)
        live[pre] = False
        idx = np.nonzero(live)[0]
        m = nearest_prefix_d2_f32(P, pre, idx)
        j = int(np.argmax(m))
        assert idx[j] == order[t], ("not the farthest", t, idx[j], order[t])
        assert np.sqrt(m[j]) == radius[t], ("radius", t)
        # packing inside the (t+1)-prefix
        pp = order[: t + 1]
        Q = P[pp]
        dx = Q[:, None, 0] - Q[None, :, 0]
        dy = Q[:, None, 1] - Q[None, :, 1]
        dz = Q[:, None, 2] - Q[None, :, 2]
        d2 = (dx * dx + dy * dy) + dz * dz
        np.fill_diagonal(d2, np.inf)
        assert np.sqrt(d2.min()) >= radius[t], ("packing", t)


def exhaustive_kcentre64(P, k):
    """Optimal discrete k-centre radius (centres among the points), binary64."""
    P = np.asarray(P, dtype=np.float64)
    D = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1))
    best = np.inf
    for S in itertools.combinations(range(P.shape[0]), k):
        r = D[:, list(S)].min(axis=1).max()
        if r < best:
            best = r
    return best


def check_two_approx(lib=None, trials=12):
    """Gonzalez: the first k picks cover every point within 2 * OPT_k."""
    for trial in range(trials):
        n = 6 + trial % 7  # 6..12
        P = cases.random_cloud(n, 500 + trial)
        s = trial % n
        o, _ = oracle.greedy32(P, n, s, lib=lib)
        P64 = P.astype(np.float64)
        D = np.sqrt(((P64[:, None, :] - P64[None, :, :]) ** 2).sum(-1))
        for k in range(1, n):
            cov = D[:, o[:k]].min(axis=1).max()
            opt = exhaustive_kcentre64(P, k)
            assert cov <= 2 * opt * (1 + 1e-6), (trial, k, cov, opt)


def check_fp64_bound(P, order, radius, lib=None, rel=1e-6):
    """|radius32 - r64| <= 1e-6 r64 along the binary32 order, and the pick is
    (1 - 1e-6)-greedy in binary64 at every step."""
    r64 = oracle.along_order64(P, order, lib=lib)
    k = len(order)
    for t in range(1, k):
        assert abs(float(radius[t]) - r64[t]) <= rel * r64[t] + 1e-300, (t, radius[t], r64[t])
    P64 = np.asarray(P, dtype=np.float64)
    n = P64.shape[0]
    m = np.full(n, np.inf)
    for t in range(1, k):
        d = np.sqrt(((P64 - P64[order[t - 1]]) ** 2).sum(1))
        m = np.minimum(m, d)
        live = np.ones(n, dtype=bool)
        live[order[:t]] = False
        best = m[live].max()
        assert r64[t] >= (1 - rel) * best, (t, r64[t], best)


def check_grid_equals_plain(P, k, start, lib=None, target=12.0):
    o1, r1 = oracle.greedy32(P, k, start, lib=lib)
    o2, r2 = oracle.greedy32_grid(P, k, start, target=target, lib=lib)
    assert np.array_equal(o1, o2), ("grid order differs", int(np.argmax(o1 != o2)))
    assert same_f32(r1, r2)


def pin_battery(lib=None):
    """The quick subset used against planted mistakes."""
    check_closed_forms(lib)
    check_bruteforce(lib, sizes=(2, 5, 17, 40))
    check_two_approx(lib, trials=4)
    P = cases.random_cloud(300, 9)
    o, r = oracle.greedy32(P, 300, 4, lib=lib)
    check_invariants(P, o, r, steps=(1, 2, 7, 50, 299))
    check_fp64_bound(P, o, r, lib=lib)
    for name in ("random", "duplicates", "mixed_scale"):
        Q = cases.ADVERSARIAL[name](700, 3)
        check_grid_equals_plain(Q, 700, 1, lib=lib)
