"""Small adversarial inputs shared by the oracle pins and the GPU parity tests.

Plain numpy; no ordering arithmetic here.
"""
import numpy as np


def random_cloud(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return (scale * rng.random((n, 3))).astype(np.float32)


def integer_lattice(nx, ny, nz):
    """Lattice with integer coordinates: massive exact distance ties."""
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1)
    return g.reshape(-1, 3).astype(np.float32)


def with_duplicates(n, seed, groups=7):
    """n points drawn (with repetition) from `groups` distinct positions."""
    rng = np.random.default_rng(seed)
    base = rng.random((groups, 3)).astype(np.float32)
    return base[rng.integers(0, groups, n)].copy()


def collinear(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.random(n).astype(np.float32)
    return np.stack([x, 2 * x, -x], 1).astype(np.float32)


def subnormal_cluster(n, seed):
    """Coordinates ~1e-21: squared distances fall in the binary32 subnormal range."""
    rng = np.random.default_rng(seed)
    return (rng.random((n, 3)) * 1e-21).astype(np.float32)


def huge_coords(n, seed):
    """Coordinates ~1e19: squared distances overflow to +inf (ties at inf)."""
    rng = np.random.default_rng(seed)
    return ((rng.random((n, 3)) - 0.5) * 4e19).astype(np.float32)


def mixed_scale(n, seed):
    """Two tight clusters far apart plus scattered points."""
    rng = np.random.default_rng(seed)
    a = rng.random((n // 3, 3)) * 1e-3
    b = rng.random((n // 3, 3)) * 1e-3 + 100.0
    c = rng.random((n - 2 * (n // 3), 3)) * 100.0
    return np.concatenate([a, b, c]).astype(np.float32)


def clumped_outliers(n, seed, clumps=8, per=4):
    """A unit cube of points plus `clumps` tight clumps of `per` points far
    away: each clump sits consecutively in Morton order, so one wavefront
    of the several-picks scan holds all of its workgroup's best keys."""
    rng = np.random.default_rng(seed)
    m = clumps * per
    body = rng.random((n - m, 3))
    centres = 40.0 + 15.0 * rng.random((clumps, 3)) * np.array([1.0, -1.0, 1.0])
    clump = np.repeat(centres, per, 0) + 1e-3 * rng.random((m, 3))
    return np.concatenate([body, clump]).astype(np.float32)


ADVERSARIAL = {
    "random": lambda n, s: random_cloud(n, s),
    "lattice": lambda n, s: integer_lattice(*_lattice_dims(n))[:n],
    "duplicates": with_duplicates,
    "collinear": collinear,
    "subnormal": subnormal_cluster,
    "huge": huge_coords,
    "mixed_scale": mixed_scale,
}


def _lattice_dims(n):
    s = int(np.ceil(n ** (1 / 3)))
    return s, s, s
