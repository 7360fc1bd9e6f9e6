"""CPU oracle for the exact greedy permutation (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never links or
calls it, and it shares no code with the HIP path.

The arithmetic lives in ``bs_oracle.c`` (plain C, binary32 without FP
contraction, compiled here with gcc).  This module only marshals numpy
arrays through ctypes.  See the C file's header for the passages of the
paper each function follows (Sec. 3.2 progressive sampling, Sec. 3.3 greedy
permutation, Sec. 4.1 r-nets) and for the readings taken where the paper is
silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_bs_oracle.so")

# -O2 with contraction off: binary32 ops stay single correctly rounded ops.
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared", "-Wall", "-Wextra"]

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/_bs_oracle.so``."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _bind(path: str):
    lib = ctypes.CDLL(path)
    i64, u64 = ctypes.c_int64, ctypes.c_uint64
    vp = ctypes.c_void_p
    lib.oracle_splitmix64_first.argtypes = [u64]
    lib.oracle_splitmix64_first.restype = u64
    lib.oracle_start_index.argtypes = [u64, i64]
    lib.oracle_start_index.restype = i64
    lib.oracle_greedy32.argtypes = [vp, i64, i64, i64, vp, vp, vp, vp, vp]
    lib.oracle_greedy32.restype = ctypes.c_int
    lib.oracle_greedy64.argtypes = [vp, i64, i64, i64, vp, vp]
    lib.oracle_greedy64.restype = ctypes.c_int
    lib.oracle_along_order64.argtypes = [vp, i64, vp, i64, vp]
    lib.oracle_along_order64.restype = ctypes.c_int
    lib.oracle_greedy32_grid.argtypes = [vp, i64, i64, i64, vp, vp, ctypes.c_double, vp]
    lib.oracle_greedy32_grid.restype = ctypes.c_int
    lib.oracle_greedy32_grid_h.argtypes = [vp, i64, i64, i64, vp, vp, ctypes.c_double, ctypes.c_double, vp]
    lib.oracle_greedy32_grid_h.restype = ctypes.c_int
    lib.oracle_oct_encode_n.argtypes = [vp, i64, vp]
    lib.oracle_oct_encode_n.restype = ctypes.c_int
    lib.oracle_emit_surfels.argtypes = [vp, vp, vp, i64, vp, i64, vp]
    lib.oracle_emit_surfels.restype = ctypes.c_int
    lib.oracle_median_nn.argtypes = [vp, i64, vp, i64, vp]
    lib.oracle_median_nn.restype = ctypes.c_int
    lib.oracle_prefix_length.argtypes = [ctypes.c_double, ctypes.c_double, i64, i64]
    lib.oracle_prefix_length.restype = i64
    lib.oracle_philox4x32_10.argtypes = [vp, vp, vp]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_sample32.argtypes = [vp, i64, i64, u64, i64, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                    vp, vp, vp]
    lib.oracle_sample32.restype = ctypes.c_int
    lib.oracle_prefix_nn.argtypes = [vp, i64, vp, i64, vp]
    lib.oracle_prefix_nn.restype = ctypes.c_int
    lib.oracle_capture_view.argtypes = [vp, vp, ctypes.c_int, vp]
    lib.oracle_capture_view.restype = ctypes.c_int
    lib.oracle_capture32.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp, ctypes.c_int32, vp, vp, vp, vp]
    lib.oracle_capture32.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    _lib = _bind(_LIB_PATH)
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _points32(points) -> np.ndarray:
    p = np.ascontiguousarray(np.asarray(points, dtype=np.float32))
    if p.ndim != 2 or p.shape[1] != 3:
        raise ValueError("points must have shape [n, 3]")
    return p


def splitmix64_first(seed: int, lib=None) -> int:
    """First SplitMix64 output for ``seed`` (Steele, Lea and Flood 2014)."""
    return int((lib or _load()).oracle_splitmix64_first(ctypes.c_uint64(seed & (2**64 - 1))))


def start_index(seed: int, n: int, lib=None) -> int:
    """The random starting surfel (Sec. 3.2): SplitMix64(seed) mod n."""
    return int((lib or _load()).oracle_start_index(ctypes.c_uint64(seed & (2**64 - 1)), n))


class OracleError(RuntimeError):
    pass


def _check(rc: int, allow_nonfinite: bool = True):
    if rc == 0 or (rc == 1 and allow_nonfinite):
        return rc
    raise OracleError("oracle returned %d" % rc)


def greedy32(points, k: int, start: int, stats: bool = False, lib=None):
    """Plain binary32 greedy permutation (Sec. 3.2/3.3).

    Returns ``(order int32[k], radius float32[k])`` and, with ``stats``, a
    dict of per-update arrays ``n_live``, ``n_ball``, ``n_dec`` (length k-1).
    """
    p = _points32(points)
    n = p.shape[0]
    order = np.empty(max(k, 0), dtype=np.int32)
    radius = np.empty(max(k, 0), dtype=np.float32)
    st = {}
    if stats:
        for key in ("n_live", "n_ball", "n_dec"):
            st[key] = np.zeros(max(k - 1, 0), dtype=np.int64)
    rc = (lib or _load()).oracle_greedy32(_ptr(p), n, k, start, _ptr(order), _ptr(radius),
                                 _ptr(st.get("n_live")), _ptr(st.get("n_ball")),
                                 _ptr(st.get("n_dec")))
    _check(rc)
    return (order, radius, st) if stats else (order, radius)


def greedy32_grid(points, k: int, start: int, target: float = 12.0, stats: bool = False, lib=None,
                  cell_side: float = 0.0):
    """Exact grid-accelerated binary32 greedy; equal to :func:`greedy32`.
    ``cell_side`` > 0 fixes the grid's cell side (else it follows ``target``
    candidates per cell)."""
    p = _points32(points)
    n = p.shape[0]
    order = np.empty(max(k, 0), dtype=np.int32)
    radius = np.empty(max(k, 0), dtype=np.float32)
    ball = np.zeros(max(k - 1, 0), dtype=np.int64) if stats else None
    rc = (lib or _load()).oracle_greedy32_grid_h(_ptr(p), n, k, start, _ptr(order), _ptr(radius),
                                        float(target), float(cell_side), _ptr(ball))
    _check(rc)
    return (order, radius, {"n_ball": ball}) if stats else (order, radius)


def greedy64(points, k: int, start: int, lib=None):
    """The same greedy in binary64 on exactly widened coordinates."""
    p = np.ascontiguousarray(_points32(points).astype(np.float64))
    n = p.shape[0]
    order = np.empty(max(k, 0), dtype=np.int32)
    radius = np.empty(max(k, 0), dtype=np.float64)
    _check((lib or _load()).oracle_greedy64(_ptr(p), n, k, start, _ptr(order), _ptr(radius)), False)
    return order, radius


def along_order64(points, order, lib=None) -> np.ndarray:
    """Binary64 distance of each ``order[t]`` to its nearest earlier pick."""
    p = _points32(points)
    o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    r = np.empty(o.shape[0], dtype=np.float64)
    _check((lib or _load()).oracle_along_order64(_ptr(p), p.shape[0], _ptr(o), o.shape[0], _ptr(r)), False)
    return r


def oct_encode(normals, lib=None) -> np.ndarray:
    """Octahedral codes (int16 [n, 2]) of float32 normals [n, 3]."""
    nrm = np.ascontiguousarray(np.asarray(normals, dtype=np.float32).reshape(-1, 3))
    out = np.empty((nrm.shape[0], 2), dtype=np.int16)
    _check((lib or _load()).oracle_oct_encode_n(_ptr(nrm), nrm.shape[0], _ptr(out)), False)
    return out


def emit_surfels(points, order, normals=None, colors=None, lib=None) -> np.ndarray:
    """The ordered 20-byte surfel records (uint8 [k, 20]) of ``order``."""
    p = _points32(points)
    o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    nrm = None if normals is None else np.ascontiguousarray(np.asarray(normals, dtype=np.float32).reshape(-1, 3))
    col = None if colors is None else np.ascontiguousarray(np.asarray(colors, dtype=np.uint8).reshape(-1, 3))
    out = np.empty((o.shape[0], 20), dtype=np.uint8)
    _check((lib or _load()).oracle_emit_surfels(_ptr(p), _ptr(nrm), _ptr(col), p.shape[0], _ptr(o), o.shape[0],
                                                _ptr(out)), False)
    return out


def median_nn(points, order, pm: int, lib=None) -> float:
    """r_m: median over the first ``pm`` ordered surfels of each one's
    distance to its nearest other surfel of that prefix (Sec. 4.1)."""
    p = _points32(points)
    o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    out = np.empty(1, dtype=np.float32)
    _check((lib or _load()).oracle_median_nn(_ptr(p), p.shape[0], _ptr(o), int(pm), _ptr(out)), False)
    return out[0]


def prefix_length(r: float, r_m: float, pm: int, k: int, lib=None) -> int:
    """p(r) = pm (r_m / r)^2, rounded up, clamped to [1, k] (Sec. 4.1)."""
    return int((lib or _load()).oracle_prefix_length(float(r), float(r_m), int(pm), int(k)))


def philox4x32_10(ctr, key, lib=None):
    """Philox4x32-10 (Salmon et al., SC'11) of a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(4))
    kk = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
    out = np.empty(4, dtype=np.uint32)
    (lib or _load()).oracle_philox4x32_10(_ptr(c), _ptr(kk), _ptr(out))
    return out


def sample32(points, k: int, seed: int, start: int, sample_size: int = 200, growth_rounds: int = 500,
             vicinity: float = 0.0, lib=None):
    """The paper's randomized progressive sampler (Sec. 3.2).

    Returns ``(order int32[k], radius float32[k], count)``; entries past
    ``count`` (the input ran out, only with ``vicinity`` > 0) are -3 / NaN.
    ``sample_size`` 0 samples the whole remaining set (exact greedy)."""
    p = _points32(points)
    n = p.shape[0]
    order = np.empty(max(k, 0), dtype=np.int32)
    radius = np.empty(max(k, 0), dtype=np.float32)
    cnt = np.zeros(1, dtype=np.int64)
    rc = (lib or _load()).oracle_sample32(_ptr(p), n, k, ctypes.c_uint64(seed & (2**64 - 1)), start,
                                          int(sample_size), int(growth_rounds), float(vicinity),
                                          _ptr(order), _ptr(radius), _ptr(cnt))
    _check(rc)
    return order, radius, int(cnt[0])


def prefix_nn(points, order, p: int, lib=None) -> np.ndarray:
    """Each of the first ``p`` ordered surfels' distance to its nearest other
    surfel of that prefix (Sec. 3.3 quality measure)."""
    pts = _points32(points)
    o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    out = np.empty(int(p), dtype=np.float32)
    _check((lib or _load()).oracle_prefix_nn(_ptr(pts), pts.shape[0], _ptr(o), int(p), _ptr(out)), False)
    return out


def capture32(kind, center, rot, prm, rgb, lo, hi, resolution: int, lib=None):
    """The initial surfel set of Sec. 3.1: first hits of eight orthographic
    views from the bounding-box corners at ``resolution``^2 pixels each.

    kind int[P] (0 sphere, 1 box, 2 cylinder), center float[P,3], rot
    float[P,3,3] (local -> world), prm float[P,3], rgb uint8[P,3], lo / hi
    float[3].  Returns (positions float32[n,3], normals float32[n,3], colours
    uint8[n,3]) in view, row, column order."""
    k = np.ascontiguousarray(np.asarray(kind, dtype=np.int32))
    P = int(k.shape[0])
    c = np.ascontiguousarray(np.asarray(center, dtype=np.float32).reshape(P, 3))
    r = np.ascontiguousarray(np.asarray(rot, dtype=np.float32).reshape(P, 9))
    pr = np.ascontiguousarray(np.asarray(prm, dtype=np.float32).reshape(P, 3))
    col = np.ascontiguousarray(np.asarray(rgb, dtype=np.uint8).reshape(P, 3))
    lo = np.ascontiguousarray(np.asarray(lo, dtype=np.float32).reshape(3))
    hi = np.ascontiguousarray(np.asarray(hi, dtype=np.float32).reshape(3))
    cap = 8 * int(resolution) ** 2
    pos = np.empty((cap, 3), dtype=np.float32)
    nrm = np.empty((cap, 3), dtype=np.float32)
    oc = np.empty((cap, 3), dtype=np.uint8)
    cnt = np.zeros(1, dtype=np.int64)
    _check((lib or _load()).oracle_capture32(_ptr(k), _ptr(c), _ptr(r), _ptr(pr), _ptr(col), P, _ptr(lo), _ptr(hi),
                                             int(resolution), _ptr(pos), _ptr(nrm), _ptr(oc), _ptr(cnt)), False)
    n = int(cnt[0])
    return pos[:n].copy(), nrm[:n].copy(), oc[:n].copy()


def capture_view(lo, hi, v: int, lib=None):
    """Camera of view v: (d, u, w, c, s) or None for an empty box."""
    lo = np.ascontiguousarray(np.asarray(lo, dtype=np.float32).reshape(3))
    hi = np.ascontiguousarray(np.asarray(hi, dtype=np.float32).reshape(3))
    out = np.empty(13, dtype=np.float32)
    if not (lib or _load()).oracle_capture_view(_ptr(lo), _ptr(hi), int(v), _ptr(out)):
        return None
    return out[0:3], out[3:6], out[6:9], out[9:12], float(out[12])


def compile_variant(src_text: str, out_path: str):
    """Compile a (mutated) copy of the oracle source and bind it.

    Used only by the test that checks that planted mistakes in the oracle
    are caught by its pins."""
    c_path = out_path + ".c"
    with open(c_path, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", *CFLAGS, "-o", out_path, c_path, "-lm"])
    return _bind(out_path)


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()
