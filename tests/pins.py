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
        with np.errstate(over="ignore"):  # overflowing coordinates: +inf is the binary32 result
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
    with np.errstate(over="ignore"):  # overflowing coordinates: +inf is the binary32 result
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
        with np.errstate(over="ignore"):  # overflowing coordinates: +inf is the binary32 result
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


def brute_statistics_f32(P, order):
    """Per-update counts of a greedy order, recomputed from scratch (numpy).

    For the update with pick u (u = 0 .. k-2), c = order[u], the prefix
    order[:u] and the live set (everything outside order[:u + 1]):
      n_live  size of the live set;
      n_ball  live candidates with d2(p, c) < m(c), where m(c) is c's binary32
              squared distance to its nearest earlier pick (+inf for u = 0);
      n_dec   live candidates with d2(p, c) < their own nearest-prefix d2
              (+inf for u = 0): the min-distances this pick lowers.
    Each distance comes from the full matrix with the association
    ((dx*dx + dy*dy) + dz*dz), independently of the oracle's loop."""
    P = np.asarray(P, dtype=np.float32)
    n = P.shape[0]
    k = len(order)
    dx = P[:, None, 0] - P[None, :, 0]
    dy = P[:, None, 1] - P[None, :, 1]
    dz = P[:, None, 2] - P[None, :, 2]
    with np.errstate(over="ignore"):  # overflowing coordinates: +inf is the binary32 result
        D = (dx * dx + dy * dy) + dz * dz
    out = {key: np.zeros(max(k - 1, 0), dtype=np.int64) for key in ("n_live", "n_ball", "n_dec")}
    inf = np.float32(np.inf)
    for u in range(k - 1):
        c = int(order[u])
        prefix = np.asarray(order[:u], dtype=np.int64)
        live = np.ones(n, dtype=bool)
        live[np.asarray(order[:u + 1], dtype=np.int64)] = False
        m_before = D[:, prefix].min(axis=1) if u > 0 else np.full(n, inf, dtype=np.float32)
        mc = m_before[c]
        d = D[:, c]
        out["n_live"][u] = int(live.sum())
        out["n_ball"][u] = int((live & (d < mc)).sum())
        out["n_dec"][u] = int((live & (d < m_before)).sum())
    return out


def check_statistics(lib=None, sizes=(2, 9, 27, 64)):
    """The oracle's n_live / n_ball / n_dec (the ball populations that set
    the pruned method's algorithmic bytes) equal a from-scratch count, on
    adversarial sets including lattices where d2 == m(c) exactly; the grid
    oracle's n_ball equals it too."""
    for name, gen in cases.ADVERSARIAL.items():
        for n in sizes:
            P = gen(n, 300 + n)
            for s in sorted({0, n // 2, n - 1}):
                o, r, st = oracle.greedy32(P, n, s, stats=True, lib=lib)
                bf = brute_statistics_f32(P, o)
                for key in ("n_live", "n_ball", "n_dec"):
                    assert np.array_equal(st[key], bf[key]), (name, n, s, key, st[key], bf[key])
                _, _, sg = oracle.greedy32_grid(P, n, s, target=2.0, stats=True, lib=lib)
                assert np.array_equal(sg["n_ball"], bf["n_ball"]), (name, n, s, "grid n_ball")


def span_boundary_case(seed=0, S=16):
    """Four points and a cell side h that put a candidate q one cell beyond
    span = floor(sqrt(m(c)) / h) + 1 of the pick c (along x) while its binary32
    d2 to c is below m(c): the subtraction x_q - x_c rounds down to the float
    just under sqrt(m(c)) although the exact distance is just above.  A grid
    walk whose span carries no rounding margin misses q in the ball count.

    Points: A (the start), c (the farthest from A, so the first pick), q, and
    D0, which fixes the grid's lower x bound so that c sits just under the
    top of its cell.  Returns (P, h) or raises if the float conditions were
    not met within the trials."""
    rng = np.random.default_rng(seed)
    f32 = np.float32
    for _ in range(20000):
        a = f32(0.78 + 0.04 * rng.random())
        yA = f32(0.58 + 0.04 * rng.random())
        # c = (-eps, 0, 0) with eps set below; m(c) = d2(A, c) is nearly that of (a, yA)
        dxa = np.float32(a)
        mc = np.float32(np.float32(dxa * dxa) + np.float32(yA * yA))
        rr = float(np.sqrt(np.float64(mc)))
        f0 = np.float32(rr)
        if float(f0) > rr:
            f0 = np.nextafter(f0, f32(0))
        ulp = float(np.nextafter(f0, f32(np.inf))) - float(f0)
        gap = rr - float(f0)
        if not (0.2 * ulp < gap < 0.4 * ulp):
            continue
        if not (np.float32(f0 * f0) < mc):
            continue
        lo = np.float32(-(rr / S + gap))
        while -float(lo) <= rr / S + gap:
            lo = np.nextafter(lo, f32(-np.inf))
        eta = -float(lo) - rr / S - gap
        eps = np.float32(gap + eta * S / (S + 1) + 0.25 * (0.5 * ulp - gap))
        if not (gap + eta * S / (S + 1) < float(eps) < 0.5 * ulp):
            continue
        xc, xq = np.float32(-eps), f0
        if np.float32(xq - xc) != f0:
            continue
        A = np.array([a - eps, yA, 0], dtype=f32)  # so that A.x - c.x rounds like a
        c = np.array([xc, 0, 0], dtype=f32)
        q = np.array([xq, 0, 0], dtype=f32)
        D0 = np.array([lo, yA, 0], dtype=f32)
        P = np.stack([A, c, q, D0]).astype(f32)
        D = float(xc) - float(lo)
        hi_h = (float(xq) - float(lo)) / (S + 1)
        lo_h = max(D, rr / S)
        if not lo_h < hi_h:
            continue
        h = 0.5 * (lo_h + hi_h)
        # the construction's claims, checked here in binary64 / binary32
        m_c = np.float32(np.float32(np.float32(P[0, 0] - P[1, 0]) ** 2) + np.float32(P[0, 1] ** 2))
        rr = float(np.sqrt(np.float64(m_c)))
        if int(np.floor(rr / h)) + 1 != S:
            continue
        if not (np.float32(np.float32(xq - xc) ** 2) < m_c and float(xq) - float(xc) > rr):
            continue
        if int(np.floor((float(xq) - float(lo)) / h)) - int(np.floor((float(xc) - float(lo)) / h)) != S + 1:
            continue
        return P, h
    raise AssertionError("no span boundary case found")


def check_span_boundary(lib=None):
    """Grid oracle with the cell side of span_boundary_case: its ball counts
    (and order) equal the plain oracle's."""
    P, h = span_boundary_case()
    o1, r1, st = oracle.greedy32(P, 4, 0, stats=True, lib=lib)
    assert o1[1] == 1 and st["n_ball"][1] == 2, (o1, st)
    o2, r2, sg = oracle.greedy32_grid(P, 4, 0, stats=True, cell_side=h, lib=lib)
    assert np.array_equal(o1, o2) and same_f32(r1, r2)
    assert np.array_equal(sg["n_ball"], st["n_ball"]), ("span boundary", sg["n_ball"], st["n_ball"])


def check_grid_equals_plain(P, k, start, lib=None, target=12.0):
    o1, r1 = oracle.greedy32(P, k, start, lib=lib)
    o2, r2 = oracle.greedy32_grid(P, k, start, target=target, lib=lib)
    assert np.array_equal(o1, o2), ("grid order differs", int(np.argmax(o1 != o2)))
    assert same_f32(r1, r2)


def oct_decode64(code):
    """Inverse octahedral map in binary64 (written from the map's
    definition, independently of the encoder): unit normals [n, 3]."""
    p = np.asarray(code, dtype=np.float64).reshape(-1, 2) / 32767.0
    x, y = p[:, 0], p[:, 1]
    z = 1.0 - np.abs(x) - np.abs(y)
    neg = z < 0
    xn = np.where(neg, (1 - np.abs(y)) * np.where(x >= 0, 1.0, -1.0), x)
    yn = np.where(neg, (1 - np.abs(x)) * np.where(y >= 0, 1.0, -1.0), y)
    d = np.stack([xn, yn, z], 1)
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def check_surfel_records(lib=None):
    """Octahedral codes: hand-derived values at the axes, at an exact half
    (round to nearest even) and on the folded lower hemisphere; the inverse
    map recovers random unit normals within 4e-4 rad.  Records: byte layout,
    absent normals / colours, out-of-range order entries."""
    hand = {(0, 0, 1): (0, 0), (0, 0, -1): (32767, 32767), (1, 0, 0): (32767, 0), (-1, 0, 0): (-32767, 0),
            (0, 1, 0): (0, 32767), (0, -1, 0): (0, -32767), (0.5, -0.25, -0.25): (24575, -16384),
            (0.70710677, 0.70710677, 0.0): (16384, 16384), (0, 0, 0): (0, 0)}
    for n, c in hand.items():
        got = tuple(int(v) for v in oracle.oct_encode(np.array([n], dtype=np.float32), lib=lib)[0])
        assert got == c, "octahedral code of %s: %s, expected %s" % (n, got, c)
    rng = np.random.default_rng(11)
    v = rng.normal(size=(20000, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    v32 = v.astype(np.float32)
    d = oct_decode64(oracle.oct_encode(v32, lib=lib))
    ang = np.arccos(np.clip((d * v32.astype(np.float64)).sum(1), -1.0, 1.0))
    assert ang.max() < 4e-4, "octahedral round trip error %g rad" % ang.max()
    # records
    P = np.array([[1.5, -2.0, 3.25], [0.0, 0.0, 0.0], [7.0, 8.0, 9.0]], dtype=np.float32)
    N = np.array([[0, 0, -1], [1, 0, 0], [0, 0, 0]], dtype=np.float32)
    C = np.array([[10, 20, 30], [40, 50, 60], [70, 80, 90]], dtype=np.uint8)
    order = np.array([2, 0, -1, 1], dtype=np.int32)
    rec = oracle.emit_surfels(P, order, N, C, lib=lib)
    assert rec.shape == (4, 20)
    pos = rec[:, :12].copy().view(np.float32).reshape(4, 3)
    code = rec[:, 12:16].copy().view(np.int16).reshape(4, 2)
    col = rec[:, 16:20]
    assert np.array_equal(pos[[0, 1, 3]], P[[2, 0, 1]]) and np.isnan(pos[2]).all()
    assert code.tolist() == [[0, 0], [32767, 32767], [0, 0], [32767, 0]]
    assert col.tolist() == [[70, 80, 90, 255], [10, 20, 30, 255], [0, 0, 0, 0], [40, 50, 60, 255]]
    bare = oracle.emit_surfels(P, order[[0, 1]], None, None, lib=lib)
    assert (bare[:, 12:16] == 0).all() and (bare[:, 16:20] == 255).all()


def check_prefix_estimate(lib=None):
    """r_m on point sets whose nearest-neighbour distances are known: a unit
    lattice (every NN distance 1), points on a line with gaps 1, 2, 3, 4
    (median 2) and 1 .. 5 (even count: mean of the middle two, 2.5), only the
    first p_m ordered points counting; on a greedy order, r_m is at least the
    covering radius of the prefix (an r-net: no two prefix points closer).
    p(r) = p_m (r_m / r)^2 at r = r_m, r_m / 2, 2 r_m, and clamped to [1, k]."""
    L = np.stack(np.meshgrid(np.arange(10), np.arange(10), np.arange(10), indexing="ij"), -1)
    L = L.reshape(-1, 3).astype(np.float32)
    ident = np.arange(L.shape[0], dtype=np.int32)
    assert oracle.median_nn(L, ident, 1000, lib=lib) == 1.0
    assert oracle.median_nn(L, ident, 500, lib=lib) == 1.0
    line = np.array([[0, 0, 0], [1, 0, 0], [3, 0, 0], [6, 0, 0], [10, 0, 0], [15, 0, 0], [100, 0, 0]],
                    dtype=np.float32)
    o7 = np.array([4, 0, 3, 1, 2, 5, 6], dtype=np.int32)
    assert oracle.median_nn(line, o7, 5, lib=lib) == 2.0   # {10, 0, 6, 1, 3}: NN 4, 1, 3, 1, 2
    assert oracle.median_nn(line, o7, 6, lib=lib) == 2.5   # + 15: NN 4, 1, 3, 1, 2, 5
    P = cases.random_cloud(2000, 21)
    o, r = oracle.greedy32(P, 600, 3, lib=lib)
    for pm in (50, 200, 600):
        assert oracle.median_nn(P, o, pm, lib=lib) >= r[pm - 1]
    assert oracle.prefix_length(0.1, 0.1, 1000, 10**6, lib=lib) == 1000
    assert oracle.prefix_length(0.05, 0.1, 1000, 10**6, lib=lib) == 4000
    assert oracle.prefix_length(0.2, 0.1, 1000, 10**6, lib=lib) == 250
    assert oracle.prefix_length(0.001, 0.1, 1000, 5000, lib=lib) == 5000
    assert oracle.prefix_length(50.0, 0.1, 1000, 5000, lib=lib) == 1


def pin_battery(lib=None):
    """The quick subset used against planted mistakes."""
    check_closed_forms(lib)
    check_surfel_records(lib)
    check_prefix_estimate(lib)
    check_bruteforce(lib, sizes=(2, 5, 17, 40))
    check_two_approx(lib, trials=4)
    check_statistics(lib, sizes=(9, 27))
    check_span_boundary(lib)
    P = cases.random_cloud(300, 9)
    o, r = oracle.greedy32(P, 300, 4, lib=lib)
    check_invariants(P, o, r, steps=(1, 2, 7, 50, 299))
    check_fp64_bound(P, o, r, lib=lib)
    for name in ("random", "duplicates", "mixed_scale"):
        Q = cases.ADVERSARIAL[name](700, 3)
        check_grid_equals_plain(Q, 700, 1, lib=lib)
    sampler_battery(lib)


# ------------------------------------------------ randomized sampler (Sec. 3.2)

PHILOX_KAT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.json")
_M32 = 0xFFFFFFFF


def philox_py(ctr, key):
    """Philox4x32-10 in plain Python integers, written from the SC'11
    definition independently of the oracle's C (used by the brute force)."""
    x0, x1, x2, x3 = (int(v) & _M32 for v in ctr)
    k0, k1 = (int(v) & _M32 for v in key)
    for r in range(10):
        if r:
            k0 = (k0 + 0x9E3779B9) & _M32
            k1 = (k1 + 0xBB67AE85) & _M32
        p0 = 0xD2511F53 * x0
        p1 = 0xCD9E8D57 * x2
        x0, x1, x2, x3 = ((p1 >> 32) ^ x1 ^ k0) & _M32, p1 & _M32, ((p0 >> 32) ^ x3 ^ k1) & _M32, p0 & _M32
    return (x0, x1, x2, x3)


def check_philox_kat(lib=None):
    with open(PHILOX_KAT) as f:
        kat = json.load(f)
    for v in kat["vectors"]:
        ctr = [int(h, 16) for h in v["ctr"]]
        key = [int(h, 16) for h in v["key"]]
        exp = [int(h, 16) for h in v["out"]]
        got = [int(w) for w in oracle.philox4x32_10(ctr, key, lib=lib)]
        assert got == exp, ("philox", v, ["%08x" % g for g in got])
        assert list(philox_py(ctr, key)) == exp


def brute_sample_f32(P, k, seed, start, S, K, vicinity):
    """From-scratch numpy sampler: every pick recomputes each candidate's
    binary32 squared distance to the nearest chosen surfel from the full
    candidate-by-chosen matrix.  Rules as the sampler's readings: slot j of
    round i tries draws a = 0..15 (Philox counter (i, j, a, 0), key = seed
    halves, candidate floor(u0 * n / 2^32)) and keeps the first remaining one;
    S = 0 or an empty sample means the whole remaining set (one pick when
    the sample came up empty); round i makes 1 + i // K picks (K < 0: one)."""
    P = np.asarray(P, dtype=np.float32)
    n = P.shape[0]
    key = (seed & _M32, (seed >> 32) & _M32)
    alive = np.ones(n, dtype=bool)
    chosen = [start]
    rad = [np.float32(np.inf)]
    alive[start] = False

    def mind():
        Q = P[np.array(chosen)]
        dx = P[:, None, 0] - Q[None, :, 0]
        dy = P[:, None, 1] - Q[None, :, 1]
        dz = P[:, None, 2] - Q[None, :, 2]
        with np.errstate(over="ignore"):
            return ((dx * dx + dy * dy) + dz * dz).min(axis=1)

    rnd = 0
    while len(chosen) < k and alive.any():
        sample = []
        if S > 0:
            for j in range(S):
                for a in range(16):
                    u = philox_py((rnd, j, a, 0), key)[0]
                    idx = (u * n) >> 32
                    if alive[idx]:
                        if idx not in sample:
                            sample.append(idx)
                        break
        whole = S == 0 or not sample
        q = 1 if (K < 0 or (whole and S > 0)) else 1 + rnd // max(K, 1)
        d_first = None
        for _ in range(q):
            if len(chosen) >= k:
                break
            m = mind()
            pool = np.nonzero(alive)[0] if whole else np.array([i for i in sample if alive[i]], dtype=np.int64)
            if pool.size == 0:
                break
            vals = m[pool]
            best = pool[vals == vals.max()].min()
            if d_first is None:
                d_first = m[best]
            chosen.append(int(best))
            rad.append(np.sqrt(m[best]))
            alive[best] = False
        if vicinity > 0 and not whole and d_first is not None:
            m = mind()
            thr = np.float32(np.float32(vicinity) * np.float32(vicinity)) * d_first
            for i in sample:
                if alive[i] and m[i] < thr:
                    alive[i] = False
        rnd += 1
    cnt = len(chosen)
    order = np.full(k, -3, dtype=np.int32)
    radius = np.full(k, np.nan, dtype=np.float32)
    order[:cnt] = chosen
    radius[:cnt] = rad
    return order, radius, cnt


def check_sampler_bruteforce(lib=None, sizes=(2, 9, 40, 64)):
    """The oracle's sampler equals the from-scratch reformulation on small
    adversarial sets, over sample sizes (including ones the remaining set
    cannot fill), growth periods and vicinity removal."""
    configs = [(200, 500, 0.0), (3, 2, 0.0), (5, 1, 0.0), (8, -1, 0.0), (4, 3, 0.5), (6, 2, 1.0), (1, 1, 0.0)]
    for name, gen in cases.ADVERSARIAL.items():
        for n in sizes:
            P = gen(n, 700 + n)
            for ci, (S, K, v) in enumerate(configs):
                seed = (0x9E3779B97F4A7C15 * (n + 31 * ci)) & (2**64 - 1)
                start = (seed >> 7) % n
                k = n if ci % 2 == 0 else max(1, (2 * n) // 3)
                o, r, c = oracle.sample32(P, k, seed, start, S, K, v, lib=lib)
                bo, br, bc = brute_sample_f32(P, k, seed, start, S, K, v)
                assert c == bc, (name, n, ci, c, bc)
                assert np.array_equal(o, bo), (name, n, ci, o, bo)
                assert same_f32(r, br), (name, n, ci, r, br)


def check_sampler_whole_is_greedy(lib=None):
    """With the whole remaining set as the sample, every pick is the exact
    greedy one, however many picks a round takes."""
    for name in ("random", "lattice", "duplicates", "mixed_scale"):
        P = cases.ADVERSARIAL[name](300, 5)
        eo, er = oracle.greedy32(P, 300, 7, lib=lib)
        for K in (1, 2, 7, 500, -1):
            o, r, c = oracle.sample32(P, 300, 123, 7, 0, K, 0.0, lib=lib)
            assert c == 300 and np.array_equal(o, eo) and same_f32(r, er), (name, K)


def check_prefix_nn(lib=None):
    """Nearest-neighbour distances inside a prefix on sets where they are
    known: a unit lattice (all 1), a line with gaps 1, 2, 3, 4, 5, 85, a single
    point (+inf); on a greedy order every value is at least the prefix's
    covering radius (an r-net)."""
    L = np.stack(np.meshgrid(np.arange(6), np.arange(6), np.arange(6), indexing="ij"), -1)
    L = L.reshape(-1, 3).astype(np.float32)
    ident = np.arange(L.shape[0], dtype=np.int32)
    assert np.all(oracle.prefix_nn(L, ident, L.shape[0], lib=lib) == 1.0)
    line = np.array([[0, 0, 0], [1, 0, 0], [3, 0, 0], [6, 0, 0], [10, 0, 0], [15, 0, 0], [100, 0, 0]],
                    dtype=np.float32)
    o7 = np.array([4, 0, 3, 1, 2, 5, 6], dtype=np.int32)
    assert oracle.prefix_nn(line, o7, 5, lib=lib).tolist() == [4.0, 1.0, 3.0, 1.0, 2.0]
    assert oracle.prefix_nn(line, o7, 7, lib=lib).tolist() == [4.0, 1.0, 3.0, 1.0, 2.0, 5.0, 85.0]
    assert np.isinf(oracle.prefix_nn(line, o7, 1, lib=lib)[0])
    P = cases.random_cloud(1500, 8)
    o, r = oracle.greedy32(P, 500, 2, lib=lib)
    for p in (10, 100, 500):
        assert oracle.prefix_nn(P, o, p, lib=lib).min() >= r[p - 1]


def sampler_battery(lib=None):
    check_capture(lib, R=16)
    check_philox_kat(lib)
    check_sampler_bruteforce(lib, sizes=(9, 40))
    check_sampler_whole_is_greedy(lib)
    check_prefix_nn(lib)


# ------------------------------------------ hierarchical generation (Sec. 3.4)

def hier_reference(P, parents, leaf_offsets, ks, seeds, sampler=None):
    """Bottom-up generation (Sec. 3.4) composed from the oracle: a leaf's
    candidates are its own rows, an inner node's the positions its children
    chose (children in increasing node order, picks in order); each node is
    ordered by oracle_greedy32 (or oracle_sample32 with `sampler` = (S, K, v))
    with start = SplitMix64(seed) mod n.  Returns per node (order, radius,
    source rows)."""
    P = np.asarray(P, dtype=np.float32)
    m = len(parents)
    children = [[] for _ in range(m)]
    for j, p in enumerate(parents):
        if p >= 0:
            children[p].append(j)
    res = [None] * m
    for j in range(m):
        if children[j]:
            src = np.concatenate([res[c][2] for c in children[j]]) if any(ks[c] for c in children[j]) \
                else np.zeros(0, dtype=np.int64)
        else:
            src = np.arange(leaf_offsets[j], leaf_offsets[j + 1], dtype=np.int64)
        k = int(ks[j])
        if k == 0:
            res[j] = (np.zeros(0, np.int32), np.zeros(0, np.float32), np.zeros(0, np.int64))
            continue
        Q = P[src]
        st = oracle.start_index(seeds[j], Q.shape[0])
        if sampler is None:
            o, r = oracle.greedy32(Q, k, st)
        else:
            o, r, _ = oracle.sample32(Q, k, seeds[j], st, *sampler)
        res[j] = (o, r, src[o] if (o >= 0).all() else np.full(k, -1, np.int64))
    return res


# ------------------------------------------- visible-surface capture (Sec. 3.1)

def prims_arrays(prims):
    """synth.Primitives -> the capture's arrays (kind, center, rot, prm, rgb)
    in float32, and the bounding box of the primitives (float32 lo, hi)."""
    kind = prims.kind.cpu().numpy().astype(np.int32)
    center = prims.center.cpu().numpy().astype(np.float32)
    rot = prims.rot.cpu().numpy().astype(np.float32)
    prm = prims.prm.cpu().numpy().astype(np.float32)
    rgb = prims.color.cpu().numpy().astype(np.uint8)
    # corners of each primitive's local box, rotated: a conservative world box
    ext = np.where(kind[:, None] == 0, prm[:, :1].repeat(3, 1),
                   np.where(kind[:, None] == 1, prm, np.stack([prm[:, 0], prm[:, 0], prm[:, 1]], 1)))
    r64 = rot.astype(np.float64)
    half = np.abs(r64) @ ext.astype(np.float64)[:, :, None]
    lo = (center.astype(np.float64) - half[:, :, 0]).min(0).astype(np.float32)
    hi = (center.astype(np.float64) + half[:, :, 0]).max(0).astype(np.float32)
    return kind, center, rot, prm, rgb, lo, hi


def brute_capture64(kind, center, rot, prm, rgb, lo, hi, R):
    """Independent binary64 ray cast of the eight corner views (numpy, every
    pixel against every primitive).  Returns per pixel (view-major, row, column)
    the hit flag, t, the runner-up t, position, normal, colour and a graze
    margin (how far the hit is from a silhouette or face edge)."""
    lo = lo.astype(np.float64)
    hi = hi.astype(np.float64)
    c = 0.5 * (lo + hi)
    s = 0.5 * np.linalg.norm(hi - lo)
    out = []
    for v in range(8):
        corner = np.where([(v >> a) & 1 for a in range(3)], hi, lo)
        dv = c - corner
        L = np.linalg.norm(dv)
        if L == 0:
            continue
        d = dv / L
        u = np.cross(d, [0.0, 0.0, 1.0])
        if np.linalg.norm(u) < 1e-6:
            u = np.cross(d, [0.0, 1.0, 0.0])
        u /= np.linalg.norm(u)
        w = np.cross(u, d)
        f = (2 * np.arange(R) + 1) / R - 1.0
        A = np.repeat(f[None, :], R, 0) * s   # [j, i]
        B = np.repeat(f[:, None], R, 1) * s
        O = c + A[..., None] * u + B[..., None] * w - 2 * s * d   # [R, R, 3]
        O = O.reshape(-1, 3)
        best = np.full(O.shape[0], np.inf)
        second = np.full(O.shape[0], np.inf)
        bi = np.full(O.shape[0], -1)
        nrm = np.zeros_like(O)
        margin = np.full(O.shape[0], np.inf)
        for q in range(kind.shape[0]):
            Rm = rot[q].astype(np.float64)
            ol = (O - center[q]) @ Rm          # rot^T (o - center)
            dl = d @ Rm
            p = prm[q].astype(np.float64)
            t = np.full(O.shape[0], np.inf)
            nl = np.zeros_like(O)
            mg = np.full(O.shape[0], np.inf)
            if kind[q] == 0:
                b = ol @ dl
                cc = (ol * ol).sum(1) - p[0] ** 2
                disc = b * b - (dl @ dl) * cc
                ok = disc >= 0
                tt = (-b - np.sqrt(np.where(ok, disc, 0))) / (dl @ dl)
                ok &= tt > 0
                t = np.where(ok, tt, np.inf)
                hitp = ol + t[:, None] * dl
                nl = np.where(ok[:, None], hitp / p[0], 0)
                mg = np.abs(disc) / (p[0] ** 2)
            elif kind[q] == 1:
                with np.errstate(divide="ignore", invalid="ignore"):
                    t1 = (-p - ol) / dl
                    t2 = (p - ol) / dl
                tn = np.where(dl == 0, np.where(np.abs(ol) <= p, -np.inf, np.inf), np.minimum(t1, t2))
                tf = np.where(dl == 0, np.where(np.abs(ol) <= p, np.inf, -np.inf), np.maximum(t1, t2))
                ax = np.argmax(tn, 1)
                tnear = tn.max(1)
                tfar = tf.min(1)
                ok = (tnear <= tfar) & (tnear > 0)
                t = np.where(ok, tnear, np.inf)
                nl[np.arange(O.shape[0]), ax] = np.where(dl[ax] > 0, -1.0, 1.0)
                nl = np.where(ok[:, None], nl, 0)
                srt = np.sort(tn, 1)
                mg = np.minimum(np.abs(tfar - tnear), np.abs(srt[:, 2] - srt[:, 1])) / (np.abs(tnear) + 1e-30)
            else:
                r, h = p[0], p[1]
                a = dl[0] ** 2 + dl[1] ** 2
                tl = np.full(O.shape[0], np.inf)
                if a > 0:
                    b = ol[:, 0] * dl[0] + ol[:, 1] * dl[1]
                    cc = ol[:, 0] ** 2 + ol[:, 1] ** 2 - r * r
                    disc = b * b - a * cc
                    ok = disc >= 0
                    tt = (-b - np.sqrt(np.where(ok, disc, 0))) / a
                    z = ol[:, 2] + tt * dl[2]
                    ok &= (tt > 0) & (z >= -h) & (z <= h)
                    tl = np.where(ok, tt, np.inf)
                    mg = np.minimum(np.abs(disc) / (r * r), np.abs(np.abs(z) - h) / h)
                tcap = np.full(O.shape[0], np.inf)
                capn = np.zeros(O.shape[0])
                if dl[2] != 0:
                    for zc in (-h, h):
                        tt = (zc - ol[:, 2]) / dl[2]
                        x = ol[:, 0] + tt * dl[0]
                        y = ol[:, 1] + tt * dl[1]
                        rr = x * x + y * y
                        ok = (tt > 0) & (rr <= r * r) & (tt < tcap)
                        capn = np.where(ok, np.sign(zc), capn)
                        tcap = np.where(ok, tt, tcap)
                        mg = np.minimum(mg, np.where(np.isfinite(tt), np.abs(rr - r * r) / (r * r), np.inf))
                lat = tl <= tcap
                t = np.minimum(tl, tcap)
                hitp = ol + np.where(np.isfinite(t), t, 0)[:, None] * dl
                nl = np.where(lat[:, None], np.stack([hitp[:, 0] / r, hitp[:, 1] / r, 0 * hitp[:, 0]], 1),
                              np.stack([0 * capn, 0 * capn, capn], 1))
                nl = np.where(np.isfinite(t)[:, None], nl, 0)
            closer = t < best
            second = np.where(closer, best, np.minimum(second, t))
            nrm = np.where(closer[:, None], nl @ Rm.T, nrm)
            margin = np.where(closer, mg, margin)
            bi = np.where(closer, q, bi)
            best = np.where(closer, t, best)
        hit = bi >= 0
        pos = O + np.where(hit, best, 0)[:, None] * d
        colr = np.where(hit[:, None], rgb[np.maximum(bi, 0)], 0)
        out.append((hit, best, second, pos, nrm, colr, margin))
    cat = [np.concatenate([o[i] for o in out]) for i in range(7)]
    return cat


def check_capture_against_brute(P_arrays, R, lib=None, tol=2e-5, ntol=2e-3):
    """The oracle's capture against the independent binary64 ray cast: every
    pixel that is clearly hit or clearly missed (away from silhouettes and
    near-equal depths) agrees on coverage, and on covered pixels the position
    agrees within tol * scene size (binary32 intersection from the ray's
    closest approach: about 1e-6 of the scene), the normal within ntol (a
    position error divided by a small radius), the colour exactly."""
    kind, center, rot, prm, rgb, lo, hi = P_arrays
    pos, nrm, col = oracle.capture32(kind, center, rot, prm, rgb, lo, hi, R, lib=lib)
    hit, best, second, bpos, bnrm, bcol, margin = brute_capture64(kind, center, rot, prm, rgb, lo, hi, R)
    with np.errstate(invalid="ignore"):  # inf - inf where nothing is hit
        clear = (margin > 1e-3) & ((second - best) > 1e-4 * (np.abs(best) + 1))
    # rebuild the oracle's per-pixel coverage from its compacted output by
    # replaying the order: covered pixels in view/row/column order
    idx = np.nonzero(hit)[0]
    scene = float(np.linalg.norm(hi.astype(np.float64) - lo.astype(np.float64)))
    assert pos.shape[0] >= int((hit & clear).sum()) and pos.shape[0] <= int((hit | ~clear).sum()), \
        ("covered pixel count", pos.shape[0], int(hit.sum()))
    if pos.shape[0] == idx.shape[0]:
        ok = clear[idx]
        assert np.all(np.abs(pos[ok] - bpos[idx][ok]) <= tol * scene), "positions"
        assert np.all(np.abs(nrm[ok] - bnrm[idx][ok]) <= ntol), "normals"
        assert np.array_equal(col[ok], bcol[idx][ok]), "colours"
    else:
        raise AssertionError("covered pixels differ at silhouettes: %d against %d" % (pos.shape[0], idx.shape[0]))
    return pos.shape[0], int(hit.sum())


def capture_cases():
    import synth
    out = [pins_sphere_box()]
    for seed, cnt in ((7, 12), (3, 40)):
        out.append(prims_arrays(synth.cad_primitives(seed, count=cnt)))
    return out


def pins_sphere_box():
    """The unit sphere and the 1 x 0.5 x 0.25 box of the sphere_and_box
    workload, as capture primitives."""
    kind = np.array([0, 1], np.int32)
    center = np.array([[0, 0, 0], [2, 0, 0]], np.float32)
    rot = np.stack([np.eye(3, dtype=np.float32)] * 2)
    prm = np.array([[1, 0, 0], [0.5, 0.25, 0.125]], np.float32)
    rgb = np.array([[200, 60, 40], [40, 90, 210]], np.uint8)
    lo = np.array([-1, -1, -1], np.float32)
    hi = np.array([2.5, 1, 1], np.float32)
    return kind, center, rot, prm, rgb, lo, hi


def check_capture(lib=None, R=24):
    """Capture pins: the binary64 brute force on three scenes; a lone sphere's
    hits lie on it with unit normals and cover pi/12 of each view (its disc
    in the square of side 2 s, s = sqrt(3) r); an axis-aligned cube's hits
    lie on its faces with the face's normal and cover sqrt(3)/3 of each view
    (a regular hexagon of area sqrt(3) in a square of side sqrt(3))."""
    for case in capture_cases():
        check_capture_against_brute(case, R, lib=lib)
    kind = np.array([0], np.int32)
    center = np.array([[0.5, -1.0, 2.0]], np.float32)
    rot = np.eye(3, dtype=np.float32)[None]
    prm = np.array([[0.75, 0, 0]], np.float32)
    rgb = np.array([[1, 2, 3]], np.uint8)
    lo = center[0] - 0.75
    hi = center[0] + 0.75
    pos, nrm, col = oracle.capture32(kind, center, rot, prm, rgb, lo, hi, R, lib=lib)
    rad = np.linalg.norm(pos.astype(np.float64) - center[0], axis=1)
    assert np.all(np.abs(rad - 0.75) <= 1e-5), "sphere radius"
    assert np.all(np.abs(np.linalg.norm(nrm, axis=1) - 1) <= 1e-5)
    assert (col == [1, 2, 3]).all()
    # the projected disc covers pi r^2 / (2 s)^2 of each view, s = sqrt(3) r
    frac = pos.shape[0] / (8.0 * R * R)
    assert abs(frac - np.pi / 12) < 4.0 / R, ("sphere coverage", frac)
    kind = np.array([1], np.int32)
    center = np.zeros((1, 3), np.float32)
    prm = np.array([[0.5, 0.5, 0.5]], np.float32)
    pos, nrm, col = oracle.capture32(kind, center, rot, prm, rgb, -prm[0], prm[0], R, lib=lib)
    assert np.all(np.abs(np.abs(pos).max(1) - 0.5) <= 1e-6), "cube surface"
    assert np.all(np.isin(np.abs(nrm).sum(1), [1.0])), "axis normals"
    # each normal is the face the hit lies on: the coordinate at +-0.5 along it
    ax = np.argmax(np.abs(nrm), 1)
    assert np.all(np.abs(pos[np.arange(pos.shape[0]), ax] - 0.5 * nrm[np.arange(pos.shape[0]), ax]) <= 1e-6)
    frac = pos.shape[0] / (8.0 * R * R)
    assert abs(frac - np.sqrt(3) / 3) < 4.0 / R, ("cube coverage", frac)
