"""Python binding of libbluesurfels (MI355X greedy blue-noise surfel ordering).

Argument marshalling only: every step of the ordering runs in the HIP
kernels of ``libbluesurfels.so`` (built in-tree by
``python -m paper_1904_08225_amd.build``).  There is no CPU fallback; if the
library is missing, :func:`load` raises.

The ordering is the greedy permutation of the paper's progressive sampling
(Sec. 3.2) whose exact form Sec. 3.3 names as the goal: start at a random
candidate, then repeatedly append the remaining candidate farthest from its
nearest chosen surfel.  See ``include/bluesurfels.h`` for the exact
arithmetic contract.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbluesurfels.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "bluesurfels.h")

BS_OK = 0
BS_ERR_INVALID_ARG = -1
BS_ERR_OUT_OF_MEMORY = -2
BS_ERR_HIP = -3
BS_ERR_OVER_BUDGET = -4
BS_ERR_NOT_READY = -5
BS_ERR_UNSUPPORTED = -6
BS_ERR_TIMEOUT = -7
BS_ERR_DEVICE = -8

KERNEL_AUTO, KERNEL_WG, KERNEL_COOP, KERNEL_GRID = 0, 1, 2, 3

_lib = None


class BSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (error_string(code) if _lib else code, msg))
        self.code = code


class Tuning(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("block", ctypes.c_int32),
                ("per_thread", ctypes.c_int32), ("groups", ctypes.c_int32),
                ("cell_points", ctypes.c_float), ("picks", ctypes.c_int32),
                ("lead_picks", ctypes.c_int32), ("batch_wide", ctypes.c_int32),
                ("spin_limit", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


def tuning(kernel: int = 0, block: int = 0, per_thread: int = 0, groups: int = 0,
           cell_points: float = 0.0, picks: int = 0, lead_picks: int = 0, batch_wide: int = 0,
           spin_limit: int = 0) -> Tuning:
    return Tuning(kernel, block, per_thread, groups, cell_points, picks, lead_picks, batch_wide, spin_limit)


class Sampler(ctypes.Structure):
    _fields_ = [("sample_size", ctypes.c_int32), ("growth_rounds", ctypes.c_int32), ("vicinity", ctypes.c_float),
                ("reserved", ctypes.c_int32 * 5)]


def sampler(sample_size: int = 200, growth_rounds: int = 500, vicinity: float = 0.0) -> Sampler:
    """Sampler parameters (``bs_sampler``); the defaults are the paper's."""
    return Sampler(int(sample_size), int(growth_rounds), float(vicinity))


def header_functions():
    """Names of the functions declared in include/bluesurfels.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bs_[a-z0-9_]+)\s*\(", text)))


def load():
    """Load libbluesurfels.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libbluesurfels.so is not built (run: python -m paper_1904_08225_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, u64, vp, sz = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_size_t
    tp = ctypes.POINTER(Tuning)
    lib.bs_error_string.argtypes = [i32]
    lib.bs_error_string.restype = ctypes.c_char_p
    lib.bs_last_error_message.argtypes = []
    lib.bs_last_error_message.restype = ctypes.c_char_p
    lib.bs_version.restype = ctypes.c_char_p
    lib.bs_start_index.argtypes = [u64, i64]
    lib.bs_start_index.restype = i64
    lib.bs_auto_kernel.argtypes = [i64, i64]
    lib.bs_auto_kernel.restype = i32
    lib.bs_plan_describe.argtypes = [i64, i64, vp, vp]
    lib.bs_plan_describe.restype = i32
    lib.bs_emit_surfels.argtypes = [vp, vp, vp, i64, vp, i64, vp, vp]
    lib.bs_emit_surfels.restype = i32
    lib.bs_prefix_median_nn.argtypes = [vp, i64, vp, i64, vp, vp]
    lib.bs_prefix_median_nn.restype = i32
    lib.bs_prefix_length.argtypes = [ctypes.c_double, ctypes.c_double, i64, i64]
    lib.bs_prefix_length.restype = i64
    lib.bs_prefix_for_radius.argtypes = [vp, i64, ctypes.c_float]
    lib.bs_prefix_for_radius.restype = i64
    lib.bs_autotune.argtypes = [vp, i64, i64, u64, tp, vp]
    lib.bs_autotune.restype = i32
    lib.bs_autotune_lookup.argtypes = [i64, i64, tp]
    lib.bs_autotune_lookup.restype = i32
    lib.bs_autotune_clear.argtypes = []
    lib.bs_autotune_clear.restype = None
    lib.bs_batch_autotune.argtypes = [vp, vp, vp, i32, vp, tp, vp]
    lib.bs_batch_autotune.restype = i32
    lib.bs_workspace_size.argtypes = [i64, i64, tp]
    lib.bs_workspace_size.restype = sz
    lib.bs_order.argtypes = [vp, vp, vp, i64, i64, u64, vp, vp, vp]
    lib.bs_order.restype = i32
    lib.bs_order_ex.argtypes = [vp, vp, vp, i64, i64, u64, i64, vp, vp, vp, sz, tp, vp]
    lib.bs_order_ex.restype = i32
    lib.bs_order_profile.argtypes = [vp, i64, i64, i64, vp, vp, vp, vp, vp, vp, sz, tp, vp]
    lib.bs_order_profile.restype = i32
    lib.bs_sampler_defaults.argtypes = []
    lib.bs_sampler_defaults.restype = Sampler
    lib.bs_sample_workspace_size.argtypes = [i64]
    lib.bs_sample_workspace_size.restype = sz
    lib.bs_sample.argtypes = [vp, i64, i64, u64, i64, ctypes.POINTER(Sampler), vp, vp, vp, vp, sz, vp]
    lib.bs_sample.restype = i32
    lib.bs_prefix_nn.argtypes = [vp, i64, vp, i64, vp, vp]
    lib.bs_prefix_nn.restype = i32
    lib.bs_batch_plan_execute_sample.argtypes = [vp, ctypes.POINTER(Sampler), vp, vp, vp, vp, vp, sz, vp]
    lib.bs_batch_plan_execute_sample.restype = i32
    lib.bs_hier_plan_create.argtypes = [ctypes.c_int32, vp, vp, vp, vp, tp, ctypes.POINTER(vp)]
    lib.bs_hier_plan_create.restype = i32
    lib.bs_hier_workspace_size.argtypes = [vp]
    lib.bs_hier_workspace_size.restype = sz
    lib.bs_hier_total_k.argtypes = [vp]
    lib.bs_hier_total_k.restype = i64
    lib.bs_hier_out_offsets.argtypes = [vp, vp]
    lib.bs_hier_out_offsets.restype = i32
    lib.bs_hier_plan_execute.argtypes = [vp, vp, ctypes.POINTER(Sampler), vp, vp, vp, vp, sz, vp]
    lib.bs_hier_plan_execute.restype = i32
    lib.bs_hier_plan_destroy.argtypes = [vp]
    lib.bs_hier_plan_destroy.restype = None
    lib.bs_capture_workspace_size.argtypes = [ctypes.c_int32]
    lib.bs_capture_workspace_size.restype = sz
    lib.bs_capture.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_int32, vp, vp, vp, vp, vp, sz, vp]
    lib.bs_capture.restype = i32
    lib.bs_order_noalloc.argtypes = [vp, i64, i64, u64, i64, vp, vp, tp, vp]
    lib.bs_order_noalloc.restype = i32
    lib.bs_noalloc_max_bytes.argtypes = []
    lib.bs_noalloc_max_bytes.restype = sz
    lib.bs_order_status.argtypes = [vp, vp]
    lib.bs_order_status.restype = i32
    lib.bs_wall_clock_hz.argtypes = []
    lib.bs_wall_clock_hz.restype = ctypes.c_double
    lib.bs_batch_plan_create.argtypes = [vp, vp, vp, ctypes.c_int32, tp, ctypes.POINTER(vp)]
    lib.bs_batch_plan_create.restype = i32
    lib.bs_batch_workspace_size.argtypes = [vp]
    lib.bs_batch_workspace_size.restype = sz
    lib.bs_batch_total_k.argtypes = [vp]
    lib.bs_batch_total_k.restype = i64
    lib.bs_batch_out_offsets.argtypes = [vp, vp]
    lib.bs_batch_out_offsets.restype = i32
    lib.bs_batch_plan_execute.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    lib.bs_batch_plan_execute.restype = i32
    lib.bs_batch_morton_order.argtypes = [vp, vp, vp, vp, sz, vp]
    lib.bs_batch_morton_order.restype = i32
    lib.bs_morton_workspace_size.argtypes = [i64]
    lib.bs_morton_workspace_size.restype = sz
    lib.bs_morton_order.argtypes = [vp, i64, vp, vp, sz, vp]
    lib.bs_morton_order.restype = i32
    lib.bs_batch_plan_destroy.argtypes = [vp]
    lib.bs_batch_plan_destroy.restype = None
    lib.bs_server_create.argtypes = [vp, ctypes.POINTER(vp)]
    lib.bs_server_create.restype = i32
    lib.bs_server_submit.argtypes = [vp, vp, ctypes.POINTER(u64)]
    lib.bs_server_submit.restype = i32
    lib.bs_server_poll.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_int)]
    lib.bs_server_poll.restype = i32
    lib.bs_server_wait.argtypes = [vp, u64, i64]
    lib.bs_server_wait.restype = i32
    lib.bs_server_drain.argtypes = [vp, i64]
    lib.bs_server_drain.restype = i32
    lib.bs_server_stats.argtypes = [vp, vp]
    lib.bs_server_stats.restype = i32
    lib.bs_server_destroy.argtypes = [vp]
    lib.bs_server_destroy.restype = None
    _lib = lib
    return lib


def error_string(code: int) -> str:
    return load().bs_error_string(code).decode()


def last_error() -> str:
    return load().bs_last_error_message().decode()


def _check(rc: int):
    if rc != BS_OK:
        raise BSError(rc, last_error())


def start_index(seed: int, n: int) -> int:
    return int(load().bs_start_index(ctypes.c_uint64(seed & (2**64 - 1)), n))


def auto_kernel(n: int, k: int) -> int:
    return int(load().bs_auto_kernel(n, k))


def plan_describe(n: int, k: int, tune: Optional[Tuning] = None) -> Tuning:
    """The plan ``order`` follows for (n, k, tune), automatic choices resolved
    (``bs_plan_describe``)."""
    out = Tuning()
    _check(load().bs_plan_describe(n, k, ctypes.byref(tune) if tune is not None else None, ctypes.byref(out)))
    return out


def autotune(points, k: int, seed: int = 0, stream=None) -> Tuning:
    """Time candidate configurations for ordering ``points`` to ``k`` (a
    prefix of the ordering) and record the fastest for this size; later
    calls without a tuning use it (``bs_autotune``)."""
    lib = load()
    points = _prep_points(points)
    t = Tuning()
    _check(lib.bs_autotune(_ptr(points), int(points.shape[0]), int(k), ctypes.c_uint64(seed & (2**64 - 1)),
                           ctypes.byref(t), _stream_handle(stream)))
    return t


def autotune_lookup(n: int, k: int) -> Optional[Tuning]:
    """The recorded configuration for (n, k), or None."""
    t = Tuning()
    rc = load().bs_autotune_lookup(int(n), int(k), ctypes.byref(t))
    return t if rc == 0 else None


def autotune_clear() -> None:
    load().bs_autotune_clear()


def batch_autotune(points, offsets, ks, seeds=None, stream=None) -> Tuning:
    """Grid cell occupancy for a batch, timed on a sample of its objects
    (``bs_batch_autotune``); pass the result to ``BatchPlan``."""
    import numpy as np
    lib = load()
    points = _prep_points(points)
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    kk = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
    sd = None if seeds is None else np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    t = Tuning()
    _check(lib.bs_batch_autotune(offs.ctypes.data_as(ctypes.c_void_p), kk.ctypes.data_as(ctypes.c_void_p),
                                 None if sd is None else sd.ctypes.data_as(ctypes.c_void_p), int(kk.shape[0]),
                                 _ptr(points), ctypes.byref(t), _stream_handle(stream)))
    return t


def workspace_size(n: int, k: int, tune: Optional[Tuning] = None) -> int:
    return int(load().bs_workspace_size(n, k, ctypes.byref(tune) if tune is not None else None))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _prep_points(points):
    import torch
    if not isinstance(points, torch.Tensor) or not points.is_cuda:
        raise TypeError("points must be a CUDA (HIP) torch tensor")
    if points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] != 3:
        raise TypeError("points must be float32 [n, 3]")
    if not points.is_contiguous():
        raise ValueError("points must be contiguous")
    return points


def order(points, k: Optional[int] = None, seed: int = 0, *, normals=None, colors=None,
          start: Optional[int] = None, tune: Optional[Tuning] = None, workspace=None,
          out_order=None, out_radius=None, stream=None, check: bool = True
          ) -> Tuple["torch.Tensor", "torch.Tensor"]:
    """Greedy permutation of ``points`` (float32 [n, 3] on the GPU).

    Returns ``(order int32[k], radius float32[k])`` on the same device.  With
    ``start`` or ``tune`` or ``workspace`` given, calls ``bs_order_ex`` with a
    torch-allocated workspace; otherwise ``bs_order``.  ``check`` synchronises
    and raises ValueError if the device flagged non-finite coordinates.
    """
    import torch
    lib = load()
    points = _prep_points(points)
    n = int(points.shape[0])
    k = n if k is None else int(k)
    dev = points.device
    if out_order is None:
        out_order = torch.empty(max(k, 0), dtype=torch.int32, device=dev)
    if out_radius is None:
        out_radius = torch.empty(max(k, 0), dtype=torch.float32, device=dev)
    st = _stream_handle(stream)
    if start is None and tune is None and workspace is None:
        rc = lib.bs_order(_ptr(points), _ptr(normals), _ptr(colors), n, k,
                          ctypes.c_uint64(seed & (2**64 - 1)), _ptr(out_order), _ptr(out_radius), st)
    else:
        tp = ctypes.byref(tune) if tune is not None else None
        if workspace is None:
            need = int(lib.bs_workspace_size(n, k, tp)) if k > 0 else 0
            if k > 0 and need == 0:
                _check(lib.bs_order_ex(_ptr(points), None, None, n, k, 0, -1 if start is None else start,
                                       _ptr(out_order), _ptr(out_radius), None, 0, tp, st))
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        rc = lib.bs_order_ex(_ptr(points), _ptr(normals), _ptr(colors), n, k,
                             ctypes.c_uint64(seed & (2**64 - 1)), -1 if start is None else int(start),
                             _ptr(out_order), _ptr(out_radius), _ptr(workspace),
                             int(workspace.numel()), tp, st)
    _check(rc)
    if check and k > 0:
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        _check_outputs(int(out_order[0]))
    return out_order, out_radius


def _check_outputs(first: int):
    # the device's error contract: -1 everywhere for non-finite input, -2 when
    # a cooperative kernel's bounded wait gave up
    if first == -1:
        raise ValueError("non-finite candidate coordinates")
    if first == -2:
        raise BSError(BS_ERR_TIMEOUT, "a cooperative kernel's bounded wait gave up; the outputs are invalid")


def order_status(workspace, stream=None) -> int:
    """Status of the last ordering enqueued on ``workspace`` (``bs_order_status``):
    BS_OK, BS_ERR_INVALID_ARG (non-finite input) or BS_ERR_TIMEOUT (a bounded
    wait gave up).  Synchronises the stream."""
    return int(load().bs_order_status(_ptr(workspace), _stream_handle(stream)))


def order_noalloc(points, k: Optional[int] = None, seed: int = 0, *, start: Optional[int] = None,
                  tune: Optional[Tuning] = None, out_order=None, out_radius=None, stream=None,
                  check: bool = True) -> Tuple["torch.Tensor", "torch.Tensor"]:
    """``bs_order_noalloc``: the ordering with the library's per-GPU scratch
    array as workspace (no device allocation by the library; the outputs are
    allocated here unless given).  Calls on one GPU must not overlap."""
    import torch
    lib = load()
    points = _prep_points(points)
    n = int(points.shape[0])
    k = n if k is None else int(k)
    dev = points.device
    if out_order is None:
        out_order = torch.empty(max(k, 0), dtype=torch.int32, device=dev)
    if out_radius is None:
        out_radius = torch.empty(max(k, 0), dtype=torch.float32, device=dev)
    tp = ctypes.byref(tune) if tune is not None else None
    _check(lib.bs_order_noalloc(_ptr(points), n, k, ctypes.c_uint64(seed & (2**64 - 1)),
                                -1 if start is None else int(start), _ptr(out_order), _ptr(out_radius), tp,
                                _stream_handle(stream)))
    if check and k > 0:
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        _check_outputs(int(out_order[0]))
    return out_order, out_radius


def sample(points, k: Optional[int] = None, seed: int = 0, *, start: Optional[int] = None,
           sample_size: int = 200, growth_rounds: int = 500, vicinity: float = 0.0, workspace=None,
           out_order=None, out_radius=None, stream=None, check: bool = True):
    """The paper's randomized progressive sampler (``bs_sample``, Sec. 3.2).

    Returns ``(order int32[k], radius float32[k], count)``; ``count`` (picks
    made; less than k only when ``vicinity`` removal empties the input) is read
    back after a sync."""
    import torch
    lib = load()
    points = _prep_points(points)
    n = int(points.shape[0])
    k = n if k is None else int(k)
    dev = points.device
    prm = sampler(sample_size, growth_rounds, vicinity)
    if out_order is None:
        out_order = torch.empty(max(k, 0), dtype=torch.int32, device=dev)
    if out_radius is None:
        out_radius = torch.empty(max(k, 0), dtype=torch.float32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    if workspace is None:
        need = int(lib.bs_sample_workspace_size(n)) if n > 0 else 0
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _check(lib.bs_sample(_ptr(points), n, k, ctypes.c_uint64(seed & (2**64 - 1)), -1 if start is None else int(start),
                         ctypes.byref(prm), _ptr(out_order), _ptr(out_radius), _ptr(cnt), _ptr(workspace),
                         int(workspace.numel()), _stream_handle(stream)))
    count = 0
    if k > 0:
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        count = int(cnt.cpu()[0])
        if check and int(out_order[0]) == -1:
            raise ValueError("non-finite candidate coordinates")
    return out_order, out_radius, count


def prefix_nn(points, order, p: int, stream=None):
    """Each of the first ``p`` ordered surfels' distance to its nearest other
    surfel of the prefix (``bs_prefix_nn``, the Sec. 3.3 measure): float32 [p]."""
    import torch
    lib = load()
    pts = _prep_points(points)
    o = (order if order.dtype == torch.int32 else order.to(torch.int32)).contiguous()
    out = torch.empty(int(p), dtype=torch.float32, device=pts.device)
    _check(lib.bs_prefix_nn(_ptr(pts), int(pts.shape[0]), _ptr(o), int(p), _ptr(out), _stream_handle(stream)))
    return out


def morton_order(points, stream=None):
    """The candidates' indices in the Morton layout of the ordering kernels
    (``bs_morton_order``): int32 [n] on the points' device."""
    import torch
    lib = load()
    pts = _prep_points(points)
    n = int(pts.shape[0])
    out = torch.empty(max(n, 1), dtype=torch.int32, device=pts.device)
    ws = torch.empty(max(int(lib.bs_morton_workspace_size(n)), 1), dtype=torch.uint8, device=pts.device)
    _check(lib.bs_morton_order(_ptr(pts), n, _ptr(out), _ptr(ws), int(ws.numel()), _stream_handle(stream)))
    return out[:n]


def primitive_records(kind, center, rot, prm, rgb):
    """Pack primitives into the 68-byte ``bs_primitive`` records (numpy
    structured array): kind int[P] (0 sphere, 1 box, 2 cylinder), center
    [P,3], rot [P,3,3] local -> world, prm [P,3], rgb uint8 [P,3]."""
    import numpy as np
    dt = np.dtype([("kind", "<i4"), ("center", "<f4", 3), ("rot", "<f4", 9), ("prm", "<f4", 3),
                   ("rgb", "u1", 4)])
    assert dt.itemsize == 68
    k = np.asarray(kind)
    rec = np.zeros(k.shape[0], dtype=dt)
    rec["kind"] = k
    rec["center"] = np.asarray(center, dtype=np.float32).reshape(-1, 3)
    rec["rot"] = np.asarray(rot, dtype=np.float32).reshape(-1, 9)
    rec["prm"] = np.asarray(prm, dtype=np.float32).reshape(-1, 3)
    rec["rgb"][:, :3] = np.asarray(rgb, dtype=np.uint8).reshape(-1, 3)
    return rec


def capture(records, lo, hi, resolution: int = 1024, stream=None, device="cuda"):
    """The visible-surface candidates of a node (``bs_capture``, Sec. 3.1):
    ``(points float32[n,3], normals float32[n,3], colors uint8[n,3])`` on the
    GPU, from primitive records (:func:`primitive_records`) and the node's
    bounding box."""
    import numpy as np
    import torch
    lib = load()
    R = int(resolution)
    raw = torch.from_numpy(np.ascontiguousarray(records).view(np.uint8).copy()).to(device)
    cap = 8 * R * R
    pts = torch.empty((cap, 3), dtype=torch.float32, device=device)
    nrm = torch.empty((cap, 3), dtype=torch.float32, device=device)
    col = torch.empty((cap, 3), dtype=torch.uint8, device=device)
    cnt = torch.zeros(1, dtype=torch.int64, device=device)
    ws = torch.empty(max(int(lib.bs_capture_workspace_size(R)), 1), dtype=torch.uint8, device=device)
    lo32 = np.ascontiguousarray(np.asarray(lo, dtype=np.float32).reshape(3))
    hi32 = np.ascontiguousarray(np.asarray(hi, dtype=np.float32).reshape(3))
    _check(lib.bs_capture(_ptr(raw), int(records.shape[0]), lo32.ctypes.data_as(ctypes.c_void_p),
                          hi32.ctypes.data_as(ctypes.c_void_p), R, _ptr(pts), _ptr(nrm), _ptr(col), _ptr(cnt),
                          _ptr(ws), int(ws.numel()), _stream_handle(stream)))
    n = int(cnt.cpu()[0])
    return pts[:n], nrm[:n], col[:n]


def noalloc_max_bytes() -> int:
    return int(load().bs_noalloc_max_bytes())


def emit_surfels(points, order, normals=None, colors=None, stream=None, out=None):
    """The ordered 20-byte surfel records (``bs_emit_surfels``) of ``order``:
    a uint8 tensor [k, 20] on the points' device (position f32 x 3,
    octahedral normal code int16 x 2, RGBA8)."""
    import torch
    lib = load()
    pts = _prep_points(points)
    o = order if order.dtype == torch.int32 else order.to(torch.int32)
    o = o.contiguous()
    k = int(o.shape[0])
    if out is None:
        out = torch.empty((k, 20), dtype=torch.uint8, device=pts.device)
    nrm = None if normals is None else normals.to(torch.float32).contiguous()
    col = None if colors is None else colors.to(torch.uint8).contiguous()
    _check(lib.bs_emit_surfels(_ptr(pts), _ptr(nrm) if nrm is not None else None,
                               _ptr(col) if col is not None else None, int(pts.shape[0]), _ptr(o), k, _ptr(out),
                               _stream_handle(stream)))
    return out


def prefix_median_nn(points, order, pm: int = 1000, stream=None) -> float:
    """r_m (``bs_prefix_median_nn``): median nearest-neighbour distance within
    the first ``pm`` ordered surfels (paper Sec. 4.1)."""
    import torch
    lib = load()
    pts = _prep_points(points)
    o = (order if order.dtype == torch.int32 else order.to(torch.int32)).contiguous()
    out = torch.empty(1, dtype=torch.float32, device=pts.device)
    _check(lib.bs_prefix_median_nn(_ptr(pts), int(pts.shape[0]), _ptr(o), int(pm), _ptr(out), _stream_handle(stream)))
    return float(out.cpu()[0])


def prefix_length(r: float, r_m: float, pm: int, k: int) -> int:
    """p(r) = pm (r_m / r)^2 rounded up, in [1, k] (``bs_prefix_length``)."""
    return int(load().bs_prefix_length(float(r), float(r_m), int(pm), int(k)))


def prefix_for_radius(radius, r: float) -> int:
    """Least prefix whose covering radius is <= r (``bs_prefix_for_radius``);
    ``radius`` is an ordering's radius array (host copy taken if needed)."""
    import numpy as np
    h = radius.detach().cpu().numpy() if hasattr(radius, "detach") else np.asarray(radius)
    h = np.ascontiguousarray(h, dtype=np.float32)
    return int(load().bs_prefix_for_radius(h.ctypes.data_as(ctypes.c_void_p), int(h.shape[0]), float(r)))


def wall_clock_hz() -> float:
    return float(load().bs_wall_clock_hz())


def _event_handle(ev):
    if ev is None:
        return None
    h = int(ev.cuda_event)
    if h == 0:
        raise ValueError("event not created yet: record it once before passing it")
    return ctypes.c_void_p(h)


def order_profile(points, k: int, start: int = -1, tune: Optional[Tuning] = None, stream=None,
                  ticks: bool = True, events=None, workspace=None, out_order=None, out_radius=None):
    """Ordering plus instruments (``bs_order_profile``).

    Returns ``(order, radius, ticks)``; ``ticks`` (when requested) is uint64
    [k] (as an int64 tensor) of the device wall clock after each pick, else
    None.  ``events`` = (begin, end) ``torch.cuda.Event`` objects, each
    already recorded once (so that the handle exists), are recorded on the
    stream right before and after the ordering kernel itself."""
    import torch
    lib = load()
    points = _prep_points(points)
    n = int(points.shape[0])
    dev = points.device
    tp = ctypes.byref(tune) if tune is not None else None
    if workspace is None:
        need = int(lib.bs_workspace_size(n, k, tp))
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    o = torch.empty(k, dtype=torch.int32, device=dev) if out_order is None else out_order
    r = torch.empty(k, dtype=torch.float32, device=dev) if out_radius is None else out_radius
    tk = torch.zeros(k, dtype=torch.int64, device=dev) if ticks else None
    eb, ee = (None, None) if events is None else (_event_handle(events[0]), _event_handle(events[1]))
    _check(lib.bs_order_profile(_ptr(points), n, k, start, _ptr(o), _ptr(r), _ptr(tk), eb, ee,
                                _ptr(workspace), int(workspace.numel()), tp, _stream_handle(stream)))
    return o, r, tk


class BatchPlan:
    """Batched ordering of many objects in CSR form (``bs_batch_plan_*``).

    ``offsets``: int sequence [m+1] of candidate row offsets, ``ks``: [m]
    picks per object, ``seeds``: [m] start seeds (default 0).  ``execute``
    takes the concatenated float32 [N, 3] candidates on the GPU and returns
    ``(order, radius)`` of length ``total_k``; object j's picks are
    ``order[out_offsets[j]:out_offsets[j+1]]`` (local indices).
    """

    def __init__(self, offsets, ks, seeds=None, tune: Optional[Tuning] = None):
        import numpy as np
        lib = load()
        self._lib = lib
        offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        kk = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
        m = int(kk.shape[0])
        if offs.shape[0] != m + 1:
            raise ValueError("offsets must have m + 1 entries")
        sd = None if seeds is None else np.ascontiguousarray(
            np.asarray([int(s) & (2**64 - 1) for s in seeds], dtype=np.uint64))
        self.m = m
        self._plan = ctypes.c_void_p()
        tp = ctypes.byref(tune) if tune is not None else None
        _check(lib.bs_batch_plan_create(offs.ctypes.data_as(ctypes.c_void_p), kk.ctypes.data_as(ctypes.c_void_p),
                                        None if sd is None else sd.ctypes.data_as(ctypes.c_void_p),
                                        m, tp, ctypes.byref(self._plan)))
        self.total_k = int(lib.bs_batch_total_k(self._plan))
        self.workspace_bytes = int(lib.bs_batch_workspace_size(self._plan))
        oo = np.zeros(m + 1, dtype=np.int64)
        _check(lib.bs_batch_out_offsets(self._plan, oo.ctypes.data_as(ctypes.c_void_p)))
        self.out_offsets = oo
        self._ws = None

    def execute(self, points, out_order=None, out_radius=None, workspace=None, stream=None):
        import torch
        points = _prep_points(points) if points.shape[0] > 0 else points
        dev = points.device
        if out_order is None:
            out_order = torch.empty(max(self.total_k, 1), dtype=torch.int32, device=dev)
        if out_radius is None:
            out_radius = torch.empty(max(self.total_k, 1), dtype=torch.float32, device=dev)
        if workspace is None:
            if self._ws is None or self._ws.numel() < self.workspace_bytes:
                self._ws = torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8, device=dev)
            workspace = self._ws
        _check(self._lib.bs_batch_plan_execute(self._plan, _ptr(points), _ptr(out_order), _ptr(out_radius),
                                               _ptr(workspace), int(workspace.numel()), _stream_handle(stream)))
        return out_order[: self.total_k], out_radius[: self.total_k]

    def morton_order(self, points, stream=None):
        """Each object's candidates in the Morton layout, indices local to
        the object, at the object's rows (``bs_batch_morton_order``)."""
        import torch
        points = _prep_points(points)
        dev = points.device
        n = int(points.shape[0])
        out = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        if self._ws is None or self._ws.numel() < self.workspace_bytes:
            self._ws = torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8, device=dev)
        _check(self._lib.bs_batch_morton_order(self._plan, _ptr(points), _ptr(out), _ptr(self._ws),
                                               int(self._ws.numel()), _stream_handle(stream)))
        return out[:n]

    def execute_sample(self, points, sample_size: int = 200, growth_rounds: int = 500, vicinity: float = 0.0,
                       out_order=None, out_radius=None, out_count=None, workspace=None, stream=None):
        """The randomized sampler (Sec. 3.2) over the plan's objects
        (``bs_batch_plan_execute_sample``): ``(order, radius, count int32[m])``."""
        import torch
        points = _prep_points(points) if points.shape[0] > 0 else points
        dev = points.device
        if out_order is None:
            out_order = torch.empty(max(self.total_k, 1), dtype=torch.int32, device=dev)
        if out_radius is None:
            out_radius = torch.empty(max(self.total_k, 1), dtype=torch.float32, device=dev)
        if out_count is None:
            out_count = torch.zeros(max(self.m, 1), dtype=torch.int32, device=dev)
        if workspace is None:
            if self._ws is None or self._ws.numel() < self.workspace_bytes:
                self._ws = torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8, device=dev)
            workspace = self._ws
        prm = sampler(sample_size, growth_rounds, vicinity)
        _check(self._lib.bs_batch_plan_execute_sample(self._plan, ctypes.byref(prm), _ptr(points), _ptr(out_order),
                                                      _ptr(out_radius), _ptr(out_count), _ptr(workspace),
                                                      int(workspace.numel()), _stream_handle(stream)))
        return out_order[: self.total_k], out_radius[: self.total_k], out_count[: self.m]

    def close(self):
        if getattr(self, "_plan", None):
            self._lib.bs_batch_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HierPlan:
    """Bottom-up generation over a scene hierarchy (``bs_hier_plan_*``, Sec. 3.4).

    ``parents``: int [m] (-1 for roots; a parent after its children);
    ``leaf_offsets``: int [m+1] rows of each leaf in the candidate array
    (inner nodes empty); ``ks``: picks per node; ``seeds``: [m] or None.
    ``execute`` returns ``(order, radius, source)`` of length ``total_k``;
    node j's picks are at ``out_offsets[j]:out_offsets[j+1]``; ``source`` is
    the candidate row each pick came from."""

    def __init__(self, parents, leaf_offsets, ks, seeds=None, tune: Optional[Tuning] = None):
        import numpy as np
        lib = load()
        self._lib = lib
        par = np.ascontiguousarray(np.asarray(parents, dtype=np.int32))
        offs = np.ascontiguousarray(np.asarray(leaf_offsets, dtype=np.int64))
        kk = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
        m = int(par.shape[0])
        if offs.shape[0] != m + 1 or kk.shape[0] != m:
            raise ValueError("leaf_offsets must have m + 1 entries and ks m")
        sd = None if seeds is None else np.ascontiguousarray(
            np.asarray([int(s) & (2**64 - 1) for s in seeds], dtype=np.uint64))
        self.m = m
        self._plan = ctypes.c_void_p()
        tp = ctypes.byref(tune) if tune is not None else None
        _check(lib.bs_hier_plan_create(m, par.ctypes.data_as(ctypes.c_void_p), offs.ctypes.data_as(ctypes.c_void_p),
                                       kk.ctypes.data_as(ctypes.c_void_p),
                                       None if sd is None else sd.ctypes.data_as(ctypes.c_void_p), tp,
                                       ctypes.byref(self._plan)))
        self.total_k = int(lib.bs_hier_total_k(self._plan))
        self.workspace_bytes = int(lib.bs_hier_workspace_size(self._plan))
        oo = np.zeros(m + 1, dtype=np.int64)
        _check(lib.bs_hier_out_offsets(self._plan, oo.ctypes.data_as(ctypes.c_void_p)))
        self.out_offsets = oo
        self._ws = None

    def execute(self, points, sampler_params: Optional[Sampler] = None, stream=None):
        import torch
        points = _prep_points(points)
        dev = points.device
        o = torch.empty(max(self.total_k, 1), dtype=torch.int32, device=dev)
        r = torch.empty(max(self.total_k, 1), dtype=torch.float32, device=dev)
        s = torch.empty(max(self.total_k, 1), dtype=torch.int32, device=dev)
        if self._ws is None or self._ws.numel() < self.workspace_bytes:
            self._ws = torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8, device=dev)
        sp = ctypes.byref(sampler_params) if sampler_params is not None else None
        _check(self._lib.bs_hier_plan_execute(self._plan, _ptr(points), sp, _ptr(o), _ptr(r), _ptr(s),
                                              _ptr(self._ws), int(self._ws.numel()), _stream_handle(stream)))
        return o[: self.total_k], r[: self.total_k], s[: self.total_k]

    def close(self):
        if getattr(self, "_plan", None):
            self._lib.bs_hier_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("device", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("max_jobs_per_batch", ctypes.c_int32),
                ("poll_us", ctypes.c_int32), ("cell_points", ctypes.c_float),
                ("workgroups", ctypes.c_int32), ("stall_us", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]


class Job(ctypes.Structure):
    _fields_ = [("d_points", ctypes.c_void_p), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("d_out_order", ctypes.c_void_p), ("d_out_radius", ctypes.c_void_p),
                ("ready_event", ctypes.c_void_p)]


class ServingStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("queued", ctypes.c_int64), ("inflight_batches", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("ordered_surfels", ctypes.c_int64),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double), ("mean_us", ctypes.c_double),
                ("max_us", ctypes.c_double), ("elapsed_s", ctypes.c_double), ("surfels_per_s", ctypes.c_double),
                ("hbm_in_use", ctypes.c_size_t), ("hbm_peak", ctypes.c_size_t),
                ("worker_launches", ctypes.c_int64), ("stall_stops", ctypes.c_int64)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class Server:
    """Serving loop with continuous batching (``bs_server_*``).

    ``submit`` takes device tensors (points float32 [n, 3], order int32 [k],
    radius float32 [k]) which must stay alive until the job is done."""

    def __init__(self, hbm_budget_bytes: int, device: int = 0, max_inflight: int = 0,
                 max_jobs_per_batch: int = 512, poll_us: int = 50, cell_points: float = 0.0,
                 workgroups: int = 0, stall_us: int = 0):
        lib = load()
        self._lib = lib
        cfg = ServerConfig(int(hbm_budget_bytes), device, max_inflight, max_jobs_per_batch, poll_us, cell_points,
                           workgroups, stall_us)
        self._srv = ctypes.c_void_p()
        _check(lib.bs_server_create(ctypes.byref(cfg), ctypes.byref(self._srv)))
        self._keep = {}

    def submit(self, points, k: int, seed: int, out_order, out_radius=None, ready=True) -> int:
        """Queue a job.  With ``ready`` (default) an event recorded on the
        current stream orders the server's read of ``points`` after the work
        already queued there (e.g. the kernel that generated them)."""
        import torch
        n = int(points.shape[0])
        ev = None
        if ready and n:
            ev = torch.cuda.Event()
            ev.record(torch.cuda.current_stream(points.device))
        job = Job(ctypes.c_void_p(points.data_ptr()) if n else None, n, int(k), seed & (2**64 - 1),
                  _ptr(out_order) if k else None, _ptr(out_radius) if (out_radius is not None and k) else None,
                  ctypes.c_void_p(int(ev.cuda_event)) if ev is not None else None)
        t = ctypes.c_uint64()
        _check(self._lib.bs_server_submit(self._srv, ctypes.byref(job), ctypes.byref(t)))
        self._keep[t.value] = (points, out_order, out_radius, ev)
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1):
        _check(self._lib.bs_server_wait(self._srv, ctypes.c_uint64(ticket), timeout_us))
        self._keep.pop(ticket, None)

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int()
        _check(self._lib.bs_server_poll(self._srv, ctypes.c_uint64(ticket), ctypes.byref(d)))
        return bool(d.value)

    def drain(self, timeout_us: int = -1):
        _check(self._lib.bs_server_drain(self._srv, timeout_us))

    def stats(self) -> dict:
        st = ServingStats()
        _check(self._lib.bs_server_stats(self._srv, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_srv", None):
            self._lib.bs_server_destroy(self._srv)
            self._srv = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
