"""The oracle against what the paper's definition and mathematics fix (CPU)."""
import numpy as np
import pytest

import oracle
import synth
from tests import cases, pins


def test_closed_forms():
    pins.check_closed_forms()


def test_splitmix64_start():
    assert oracle.splitmix64_first(0) == 0xE220A8397B1DCDAF
    for n in (1, 2, 7, 16384, 4194304):
        for seed in (0, 1, 2, 12345, 2**64 - 1):
            s = oracle.start_index(seed, n)
            assert s == oracle.splitmix64_first(seed) % n
            assert 0 <= s < n


def test_bruteforce_numpy():
    pins.check_bruteforce()


def test_invariants_sampled_steps():
    P = synth.sphere_and_box(n=3000, seed=11).points.numpy()
    o, r = oracle.greedy32(P, 3000, 17)
    pins.check_invariants(P, o, r, steps=(1, 2, 3, 10, 100, 999, 2000, 2999))


@pytest.mark.parametrize("name", sorted(cases.ADVERSARIAL))
def test_invariants_adversarial(name):
    P = cases.ADVERSARIAL[name](400, 21)
    o, r = oracle.greedy32(P, 400, 5)
    pins.check_invariants(P, o, r, steps=range(1, 400, 7))


def test_prefix_stability():
    P = cases.random_cloud(500, 77)
    full, rf = oracle.greedy32(P, 500, 3)
    for k in (0, 1, 2, 50, 499):
        o, r = oracle.greedy32(P, k, 3)
        assert np.array_equal(o, full[:k])
        assert pins.same_f32(r, rf[:k])


def test_two_approximation():
    pins.check_two_approx()


def test_fp64_error_bound():
    P = synth.sphere_and_box(n=2000, seed=5).points.numpy()
    o, r = oracle.greedy32(P, 2000, 0)
    pins.check_fp64_bound(P, o, r)


def test_fp64_greedy_agrees_on_generic_input():
    # Away from near-ties the binary64 greedy picks the same candidates.
    P = cases.random_cloud(300, 4)
    o32, r32 = oracle.greedy32(P, 300, 0)
    o64, r64 = oracle.greedy64(P, 300, 0)
    assert np.array_equal(o32, o64)
    assert np.allclose(r32[1:], r64[1:], rtol=1e-6)


def test_grid_equals_plain_adversarial():
    for name, gen in cases.ADVERSARIAL.items():
        for n in (1, 2, 33, 1000):
            P = gen(n, 8 + n)
            for target in (1.0, 4.0, 30.0):
                pins.check_grid_equals_plain(P, n, n // 3, target=target)


def test_grid_equals_plain_clumped_outliers():
    # Far clumps of nearly coincident points: the grid's cells span both
    # the cube and the clumps, and the clumps are chosen first.
    for n in (40, 700):
        P = cases.clumped_outliers(n, 17)
        pins.check_grid_equals_plain(P, n, n // 2)
        o, r = oracle.greedy32(P, n, n // 2)
        pins.check_invariants(P, o, r)


@pytest.mark.parametrize("which", ["sphere_and_box", "cad_part"])
def test_grid_equals_plain_surfaces(which):
    if which == "sphere_and_box":
        P = synth.sphere_and_box(n=16384, seed=1).points.numpy()
        k = 16384
    else:
        P = synth.cad_part(65536, seed=2).points.numpy()
        k = 8192
    pins.check_grid_equals_plain(P, k, oracle.start_index(7, P.shape[0]))


def test_edge_cases():
    P = cases.random_cloud(5, 1)
    o, r = oracle.greedy32(P, 0, 0)
    assert o.size == 0 and r.size == 0
    o, r = oracle.greedy32(P[:1], 1, 0)
    assert o.tolist() == [0] and np.isinf(r[0])
    with pytest.raises(oracle.OracleError):
        oracle.greedy32(P, 6, 0)           # k > n
    with pytest.raises(oracle.OracleError):
        oracle.greedy32(P, 3, 5)           # start out of range
    Q = P.copy()
    Q[2, 1] = np.nan
    o, r = oracle.greedy32(Q, 4, 0)
    assert (o == -1).all() and np.isnan(r).all()
    Q[2, 1] = np.inf
    o, r = oracle.greedy32_grid(Q, 4, 0)
    assert (o == -1).all() and np.isnan(r).all()


def test_statistics_brute_force():
    pins.check_statistics()


def test_grid_span_boundary():
    pins.check_span_boundary()


def test_philox_known_answers():
    pins.check_philox_kat()


def test_sampler_bruteforce():
    pins.check_sampler_bruteforce()


def test_sampler_whole_set_is_exact_greedy():
    pins.check_sampler_whole_is_greedy()


def test_prefix_nn():
    pins.check_prefix_nn()


def test_sampler_edges():
    P = cases.random_cloud(50, 2)
    o, r, c = oracle.sample32(P, 0, 1, 0)
    assert c == 0 and o.size == 0
    o, r, c = oracle.sample32(P[:1], 1, 1, 0)
    assert c == 1 and o.tolist() == [0] and np.isinf(r[0])
    with pytest.raises(oracle.OracleError):
        oracle.sample32(P, 51, 1, 0)                      # k > n
    with pytest.raises(oracle.OracleError):
        oracle.sample32(P, 5, 1, 0, sample_size=0, vicinity=0.5)  # removal needs a sample
    Q = P.copy()
    Q[3, 0] = np.nan
    o, r, c = oracle.sample32(Q, 10, 1, 0)
    assert (o == -1).all() and np.isnan(r).all()
    # prefix stability holds for the sampler too (the rounds do not depend on k)
    full, rf, _ = oracle.sample32(P, 50, 99, 4, sample_size=7, growth_rounds=3)
    for k in (1, 2, 13, 49):
        o, r, c = oracle.sample32(P, k, 99, 4, sample_size=7, growth_rounds=3)
        assert c == k and np.array_equal(o, full[:k]) and pins.same_f32(r, rf[:k])
    # vicinity removal can exhaust the input: the tail is -3 / NaN
    o, r, c = oracle.sample32(P, 50, 5, 0, sample_size=50, growth_rounds=-1, vicinity=3.0)
    assert c < 50 and (o[c:] == -3).all() and np.isnan(r[c:]).all() and (o[:c] >= 0).all()


def test_sampler_quality_between_random_and_greedy():
    # Sec. 3.3: the sampler's prefixes cover the surface almost as evenly as
    # the greedy permutation's and far better than a random subset's
    import synth
    P = synth.cad_part(20000, seed=3).points.numpy()
    eo, _ = oracle.greedy32_grid(P, 2000, 0)
    so, _, _ = oracle.sample32(P, 2000, 7, 0)
    ro = np.random.default_rng(1).permutation(P.shape[0])[:2000].astype(np.int32)
    for p in (500, 2000):
        g, s, r = (np.median(oracle.prefix_nn(P, o, p)) for o in (eo, so, ro))
        assert g >= s > 1.5 * r, (p, g, s, r)


def test_capture_pins():
    pins.check_capture()


def test_statistics_consistent():
    P = cases.random_cloud(600, 3)
    o, r, st = oracle.greedy32(P, 600, 2, stats=True)
    # live count after u+1 picks
    assert np.array_equal(st["n_live"], 600 - 1 - np.arange(599))
    assert np.all(st["n_dec"] <= st["n_ball"]) and np.all(st["n_ball"] <= st["n_live"])
    _, _, sg = oracle.greedy32_grid(P, 600, 2, stats=True)
    assert np.array_equal(sg["n_ball"], st["n_ball"])
