"""Seeded synthetic surfel-candidate workloads.

This module is shared by the tests, the benchmark and the scripts that write
stored expected values.  It only makes inputs: it holds none of the
ordering method's arithmetic.

The paper's candidates are the visible-surface pixels of a node rendered
from the eight corners of its bounding box (Sec. 3.1); its scenes (Stanford
bunny, UNC power plant, Pompeii, car factory, bakery) are not available
here.  The stand-ins sample surfaces of analytic primitives uniformly by
area and keep only samples on the boundary of the union (a sample strictly
inside another primitive of the same object is rejected), each with its
analytic normal and an RGB8 colour per primitive.  All draws come from
``torch.Generator`` objects seeded from the caller's seed, on the device the
caller names (host: Mersenne twister; GPU: Philox4x32-10), so a given
(seed, device) always produces the same surfels.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import torch

SPHERE, BOX, CYLINDER, TORUS = 0, 1, 2, 3


@dataclass
class Surfels:
    """Candidate set of one object: AoS float32 xyz, normals, RGB8."""
    points: torch.Tensor   # [n, 3] float32
    normals: torch.Tensor  # [n, 3] float32
    colors: torch.Tensor   # [n, 3] uint8

    @property
    def n(self) -> int:
        return int(self.points.shape[0])


@dataclass
class Primitives:
    kind: torch.Tensor     # [P] int64
    center: torch.Tensor   # [P, 3] float64
    rot: torch.Tensor      # [P, 3, 3] float64 (local -> world)
    prm: torch.Tensor      # [P, 3] float64 (see _area)
    color: torch.Tensor    # [P, 3] uint8


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    return g


def _rand(g, shape, device):
    return torch.rand(shape, generator=g, device=device, dtype=torch.float64)


def _log_uniform(g, shape, lo, hi, device):
    u = _rand(g, shape, device)
    return torch.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))


def _random_rotations(g, m, device):
    """Uniform random rotations from normalised Gaussian quaternions."""
    q = torch.randn((m, 4), generator=g, device=device, dtype=torch.float64)
    q = q / q.norm(dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    r = torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], dim=1)
    return r.view(m, 3, 3)


def _area(prims: Primitives) -> torch.Tensor:
    a, b, c = prims.prm.unbind(1)
    k = prims.kind
    sphere = 4 * math.pi * a * a                     # a = radius
    box = 8 * (a * b + a * c + b * c)                # a, b, c = half extents
    cyl = 2 * math.pi * a * (2 * b) + 2 * math.pi * a * a  # a = r, b = h/2
    torus = 4 * math.pi * math.pi * a * b            # a = R, b = r
    return torch.where(k == SPHERE, sphere, torch.where(k == BOX, box,
                       torch.where(k == CYLINDER, cyl, torus)))


def _bound_radius(prims: Primitives) -> torch.Tensor:
    a, b, c = prims.prm.unbind(1)
    k = prims.kind
    return torch.where(k == SPHERE, a, torch.where(k == BOX, torch.sqrt(a * a + b * b + c * c),
                       torch.where(k == CYLINDER, torch.sqrt(a * a + b * b), a + b)))


def _sample_local(g, prims: Primitives, pid: torch.Tensor, device):
    """Area-uniform samples on primitive surfaces, in local coordinates.

    Returns (q, nrm, ok): ok is False where the torus area-element rejection
    refused the sample."""
    m = pid.shape[0]
    u = _rand(g, (m, 4), device)
    kind = prims.kind[pid]
    a, b, c = prims.prm[pid].unbind(1)
    two_pi = 2 * math.pi
    q = torch.zeros((m, 3), dtype=torch.float64, device=device)
    nrm = torch.zeros_like(q)
    ok = torch.ones(m, dtype=torch.bool, device=device)

    # sphere: z = 1 - 2u, phi = 2 pi v
    s = kind == SPHERE
    if s.any():
        z = 1 - 2 * u[s, 0]
        phi = two_pi * u[s, 1]
        rho = torch.sqrt(torch.clamp(1 - z * z, min=0))
        d = torch.stack([rho * torch.cos(phi), rho * torch.sin(phi), z], 1)
        q[s] = d * a[s, None]
        nrm[s] = d

    # box: face chosen proportionally to its area, uniform within the face
    s = kind == BOX
    if s.any():
        A, B, C = a[s], b[s], c[s]
        w = torch.stack([B * C, A * C, A * B], 1)
        cw = torch.cumsum(w, 1) / w.sum(1, keepdim=True)
        axis = (u[s, 2:3] >= cw).sum(1).clamp(max=2)
        sign = torch.where(u[s, 3] < 0.5, -1.0, 1.0).to(torch.float64)
        half = torch.stack([A, B, C], 1)
        # free coordinates: the two axes other than `axis`
        f0 = 2 * u[s, 0] - 1
        f1 = 2 * u[s, 1] - 1
        ax0 = torch.where(axis == 0, 1, 0)
        ax1 = torch.where(axis == 2, 1, 2)
        p = torch.zeros_like(half)
        ar = torch.arange(p.shape[0], device=device)
        p[ar, axis] = sign * half[ar, axis]
        p[ar, ax0] = f0 * half[ar, ax0]
        p[ar, ax1] = f1 * half[ar, ax1]
        nn = torch.zeros_like(p)
        nn[ar, axis] = sign
        q[s] = p
        nrm[s] = nn

    # cylinder along local z: lateral 2 pi r h, two caps pi r^2
    s = kind == CYLINDER
    if s.any():
        R, H = a[s], b[s]
        lat = 2 * math.pi * R * 2 * H
        cap = math.pi * R * R
        tot = lat + 2 * cap
        v = u[s, 2] * tot
        th = two_pi * u[s, 0]
        is_lat = v < lat
        is_top = v >= lat + cap
        rho = torch.where(is_lat, R, R * torch.sqrt(u[s, 1]))
        th2 = torch.where(is_lat, th, two_pi * u[s, 0])
        zz = torch.where(is_lat, H * (2 * u[s, 1] - 1), torch.where(is_top, H, -H))
        p = torch.stack([rho * torch.cos(th2), rho * torch.sin(th2), zz], 1)
        nn = torch.where(is_lat[:, None],
                         torch.stack([torch.cos(th2), torch.sin(th2), torch.zeros_like(th2)], 1),
                         torch.stack([torch.zeros_like(th2), torch.zeros_like(th2),
                                      torch.where(is_top, 1.0, -1.0).to(torch.float64)], 1))
        q[s] = p
        nrm[s] = nn

    # torus around local z: area element (R + r cos v), accepted by rejection
    s = kind == TORUS
    if s.any():
        R, r = a[s], b[s]
        uu = two_pi * u[s, 0]
        vv = two_pi * u[s, 1]
        ring = R + r * torch.cos(vv)
        ok[s] = u[s, 2] * (R + r) < ring
        p = torch.stack([ring * torch.cos(uu), ring * torch.sin(uu), r * torch.sin(vv)], 1)
        nn = torch.stack([torch.cos(vv) * torch.cos(uu), torch.cos(vv) * torch.sin(uu),
                          torch.sin(vv)], 1)
        q[s] = p
        nrm[s] = nn
    return q, nrm, ok


def _inside(prims: Primitives, i: int, pts: torch.Tensor) -> torch.Tensor:
    """Strictly-inside test of world points against primitive i."""
    qq = (pts - prims.center[i]) @ prims.rot[i]
    a, b, c = [float(v) for v in prims.prm[i]]
    kind = int(prims.kind[i])
    x, y, z = qq.unbind(1)
    if kind == SPHERE:
        return x * x + y * y + z * z < a * a
    if kind == BOX:
        return (x.abs() < a) & (y.abs() < b) & (z.abs() < c)
    if kind == CYLINDER:
        return (x * x + y * y < a * a) & (z.abs() < b)
    rr = torch.sqrt(x * x + y * y) - a
    return rr * rr + z * z < b * b


def sample_union_boundary(prims: Primitives, n: int, seed: int, device="cpu") -> Surfels:
    """n area-uniform samples on the boundary of the union of `prims`."""
    device = torch.device(device)
    g = _gen(seed, device)
    area = _area(prims)
    cdf = torch.cumsum(area, 0) / area.sum()
    cdf[-1] = 1.0
    bound = _bound_radius(prims)
    P = prims.kind.shape[0]
    got_p: List[torch.Tensor] = []
    got_n: List[torch.Tensor] = []
    got_c: List[torch.Tensor] = []
    have = 0
    batch = max(1024, int(n * 1.3) + 64)
    while have < n:
        pid = torch.searchsorted(cdf, _rand(g, (batch,), device), right=True).clamp(max=P - 1)
        q, nrm, ok = _sample_local(g, prims, pid, device)
        rot = prims.rot[pid]
        pts = torch.einsum("mij,mj->mi", rot, q) + prims.center[pid]
        nw = torch.einsum("mij,mj->mi", rot, nrm)
        keep = ok.clone()
        if P > 1:
            for i in range(P):
                near = ((pts - prims.center[i]).pow(2).sum(1) < float(bound[i]) ** 2) & (pid != i) & keep
                idx = near.nonzero().squeeze(1)
                if idx.numel():
                    ins = _inside(prims, i, pts[idx])
                    keep[idx[ins]] = False
        idx = keep.nonzero().squeeze(1)
        got_p.append(pts[idx])
        got_n.append(nw[idx])
        got_c.append(prims.color[pid[idx]])
        have += int(idx.numel())
        rate = max(have / max(batch * len(got_p), 1), 0.05)
        batch = max(1024, int((n - have) / rate * 1.1) + 64)
    pts = torch.cat(got_p)[:n].to(torch.float32).contiguous()
    nw = torch.cat(got_n)[:n].to(torch.float32).contiguous()
    col = torch.cat(got_c)[:n].contiguous()
    return Surfels(pts, nw, col)


def _prims(kind, center, rot, prm, color) -> Primitives:
    return Primitives(kind, center, rot, prm, color)


def sphere_and_box(n: int = 16384, seed: int = 1, device="cpu") -> Surfels:
    """Unit sphere at the origin plus a 1 x 0.5 x 0.25 box centred at (2,0,0)."""
    device = torch.device(device)
    kind = torch.tensor([SPHERE, BOX], device=device)
    center = torch.tensor([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0]], dtype=torch.float64, device=device)
    rot = torch.eye(3, dtype=torch.float64, device=device).repeat(2, 1, 1)
    prm = torch.tensor([[1.0, 0.0, 0.0], [0.5, 0.25, 0.125]], dtype=torch.float64, device=device)
    color = torch.tensor([[200, 60, 40], [40, 90, 210]], dtype=torch.uint8, device=device)
    return sample_union_boundary(_prims(kind, center, rot, prm, color), n, seed, device)


def cad_primitives(seed: int, count: int = 200, device="cpu") -> Primitives:
    """`count` random boxes / cylinders (Bernoulli 1/2): box edges and
    cylinder radius and height log-uniform in [0.01, 1], uniform random
    rotation, centres uniform in [0, 2]^3 (so they overlap)."""
    device = torch.device(device)
    g = _gen(seed * 7919 + 17, device)
    kind = torch.where(_rand(g, (count,), device) < 0.5, BOX, CYLINDER)
    dims = _log_uniform(g, (count, 3), 0.01, 1.0, device)
    prm = torch.where((kind == BOX)[:, None], dims / 2,
                      torch.stack([dims[:, 0] / 2, dims[:, 1] / 2, torch.zeros_like(dims[:, 0])], 1))
    center = 2 * _rand(g, (count, 3), device)
    rot = _random_rotations(g, count, device)
    color = (255 * _rand(g, (count, 3), device)).to(torch.uint8)
    return _prims(kind, center, rot, prm, color)


def cad_part(n: int, seed: int = 2, count: int = 200, device="cpu") -> Surfels:
    """One CAD-like part: union boundary of `count` random boxes/cylinders."""
    return sample_union_boundary(cad_primitives(seed, count, device), n, seed, device)


def log_uniform_sizes(m: int, lo: int, hi: int, seed: int) -> List[int]:
    """m integers log-uniform in [lo, hi] (host generator)."""
    g = _gen(seed * 104729 + 3, "cpu")
    v = _log_uniform(g, (m,), float(lo), float(hi), "cpu")
    return [int(min(max(round(float(x)), lo), hi)) for x in v]


def scene_object(kind: int, n: int, seed: int, device="cpu") -> Surfels:
    """Objects of the heterogeneous scene: 0 = thin two-sided sheet (one
    dimension 1e-3..1e-2), 1 = torus, 2 = cluster of dense small boxes
    (edges 0.01..0.05)."""
    device = torch.device(device)
    g = _gen(seed * 31 + 5, device)
    if kind == 0:
        dims = _log_uniform(g, (1, 3), 0.2, 1.0, device)
        dims[0, 2] = float(_log_uniform(g, (1,), 1e-3, 1e-2, device))
        prims = _prims(torch.tensor([BOX], device=device), torch.zeros((1, 3), dtype=torch.float64, device=device),
                       _random_rotations(g, 1, device), dims / 2,
                       (255 * _rand(g, (1, 3), device)).to(torch.uint8))
    elif kind == 1:
        R = float(_log_uniform(g, (1,), 0.2, 1.0, device))
        r = R * float(0.1 + 0.3 * _rand(g, (1,), device))
        prims = _prims(torch.tensor([TORUS], device=device), torch.zeros((1, 3), dtype=torch.float64, device=device),
                       _random_rotations(g, 1, device),
                       torch.tensor([[R, r, 0.0]], dtype=torch.float64, device=device),
                       (255 * _rand(g, (1, 3), device)).to(torch.uint8))
    else:
        cnt = 24
        dims = _log_uniform(g, (cnt, 3), 0.01, 0.05, device)
        prims = _prims(torch.full((cnt,), BOX, device=device), 0.15 * _rand(g, (cnt, 3), device),
                       _random_rotations(g, cnt, device), dims / 2,
                       (255 * _rand(g, (cnt, 3), device)).to(torch.uint8))
    return sample_union_boundary(prims, n, seed, device)


def poisson_arrivals(count: int, rate_hz: float, seed: int) -> List[float]:
    """Arrival times (s) of a Poisson process with the given mean rate."""
    g = _gen(seed * 7 + 11, "cpu")
    u = _rand(g, (count,), "cpu")
    gaps = -torch.log1p(-u) / rate_hz
    return torch.cumsum(gaps, 0).tolist()


def concat(objs: List[Surfels]):
    """Concatenate objects into CSR form: (points, normals, colors, offsets)."""
    offs = [0]
    for o in objs:
        offs.append(offs[-1] + o.n)
    pts = torch.cat([o.points for o in objs]) if objs else torch.zeros((0, 3))
    nrm = torch.cat([o.normals for o in objs]) if objs else torch.zeros((0, 3))
    col = torch.cat([o.colors for o in objs]) if objs else torch.zeros((0, 3), dtype=torch.uint8)
    return pts, nrm, col, offs


def _inside_batched(kind, prm, center, rot, pts):
    """Strictly-inside test of points against one primitive each (batched):
    kind [S], prm [S,3], center [S,3], rot [S,3,3], pts [S,3]."""
    q = torch.einsum("sji,sj->si", rot, pts - center)  # rot^T (p - c)
    x, y, z = q.unbind(1)
    a, b, c = prm.unbind(1)
    sphere = x * x + y * y + z * z < a * a
    box = (x.abs() < a) & (y.abs() < b) & (z.abs() < c)
    cyl = (x * x + y * y < a * a) & (z.abs() < b)
    rr = torch.sqrt(x * x + y * y) - a
    tor = rr * rr + z * z < b * b
    return torch.where(kind == SPHERE, sphere, torch.where(kind == BOX, box,
                       torch.where(kind == CYLINDER, cyl, tor)))


def cad_parts_batch(sizes: List[int], seed: int = 3, count: int = 200, device="cpu",
                    chunk: int = 1 << 24):
    """Many CAD-like parts at once: object j is the union boundary of its own
    `count` random boxes/cylinders (the recipe of :func:`cad_part`), with
    sizes[j] area-uniform samples.  Returns (points [N,3] float32, offsets
    list of m+1).  Vectorised over objects and processed in chunks of
    samples, so thousands of objects take seconds on a GPU."""
    device = torch.device(device)
    m = len(sizes)
    g = _gen(seed * 7919 + 29, device)
    kind = torch.where(_rand(g, (m, count), device) < 0.5, BOX, CYLINDER)
    dims = _log_uniform(g, (m, count, 3), 0.01, 1.0, device)
    prm = torch.where((kind == BOX)[..., None], dims / 2,
                      torch.stack([dims[..., 0] / 2, dims[..., 1] / 2, torch.zeros_like(dims[..., 0])], -1))
    center = 2 * _rand(g, (m, count, 3), device)
    rot = _random_rotations(g, m * count, device).view(m, count, 3, 3)
    flat = Primitives(kind.reshape(-1), center.reshape(-1, 3), rot.reshape(-1, 3, 3), prm.reshape(-1, 3),
                      torch.zeros((m * count, 3), dtype=torch.uint8, device=device))
    area = _area(flat).view(m, count)
    cdf = torch.cumsum(area, 1) / area.sum(1, keepdim=True)
    cdf[:, -1] = 1.0
    flat_cdf = (cdf + torch.arange(m, device=device, dtype=torch.float64)[:, None]).reshape(-1)
    bound = _bound_radius(flat).view(m, count)
    sizes_t = torch.tensor(sizes, dtype=torch.int64, device=device)
    need = sizes_t.clone()
    got: List[List[torch.Tensor]] = [[] for _ in range(m)]
    have = torch.zeros(m, dtype=torch.int64, device=device)
    over = 1.35
    rounds = 0
    while bool((need > 0).any()) and rounds < 12:
        rounds += 1
        want = torch.clamp((need.double() * over).ceil().long() + 16, min=0) * (need > 0)
        obj_all = torch.repeat_interleave(torch.arange(m, device=device), want)
        for s0 in range(0, int(obj_all.numel()), chunk):
            obj = obj_all[s0:s0 + chunk]
            u = _rand(g, (obj.numel(),), device) * 0.999999999 + obj.double()
            pid_flat = torch.searchsorted(flat_cdf, u, right=True).clamp(max=m * count - 1)
            pid_flat = torch.maximum(pid_flat, obj * count)
            q, nrm, ok = _sample_local(g, flat, pid_flat, device)
            r = flat.rot[pid_flat]
            pts = torch.einsum("mij,mj->mi", r, q) + flat.center[pid_flat]
            keep = ok.clone()
            own = pid_flat - obj * count
            for p in range(count):
                fp = obj * count + p
                near = keep & (own != p) & ((pts - flat.center[fp]).pow(2).sum(1) < bound.view(-1)[fp] ** 2)
                idx = near.nonzero().squeeze(1)
                if idx.numel():
                    f = fp[idx]
                    ins = _inside_batched(flat.kind[f], flat.prm[f], flat.center[f], flat.rot[f], pts[idx])
                    keep[idx[ins]] = False
            kept = keep.nonzero().squeeze(1)
            ko = obj[kept]
            kp = pts[kept].to(torch.float32)
            # take at most `need` more per object, in sample order
            order = torch.argsort(ko, stable=True)
            ko = ko[order]
            kp = kp[order]
            counts = torch.bincount(ko, minlength=m)
            starts = torch.cumsum(counts, 0) - counts
            rank = torch.arange(ko.numel(), device=device) - starts[ko]
            take = rank < (sizes_t - have)[ko]
            ko = ko[take]
            kp = kp[take]
            taken = torch.bincount(ko, minlength=m)
            if ko.numel():
                for j, part in enumerate(torch.split(kp, taken.tolist())):
                    if part.shape[0]:
                        got[j].append(part)
            have += taken
        need = sizes_t - have
        over *= 1.5
    pts = torch.cat([torch.cat(gj) if gj else torch.zeros((0, 3), device=device) for gj in got]).contiguous()
    offs = [0]
    for n in sizes:
        offs.append(offs[-1] + n)
    assert pts.shape[0] == offs[-1], "generator did not reach the requested sizes"
    return pts, offs


def scene_batch(sizes: List[int], seed: int = 5, device="cpu", chunk: int = 1 << 24, pad: int = 24):
    """The heterogeneous scene's objects at once: object j is kind j % 3 of
    :func:`scene_object` (0 thin two-sided sheet, 1 torus, 2 cluster of 24
    small boxes), drawn with its own parameters, with sizes[j] area-uniform
    union-boundary samples in its local frame.  Returns (points [N,3]
    float32, offsets list of m+1), like :func:`cad_parts_batch`, but writes
    samples straight into their object's rows so that 10^4 objects and 10^9
    samples stay cheap."""
    device = torch.device(device)
    m = len(sizes)
    g = _gen(seed * 7919 + 31, device)
    P = pad
    kind = torch.full((m, P), BOX, dtype=torch.int64, device=device)
    prm = torch.zeros((m, P, 3), dtype=torch.float64, device=device)  # zero size: never drawn, never inside
    center = torch.zeros((m, P, 3), dtype=torch.float64, device=device)
    rot = _random_rotations(g, m * P, device).view(m, P, 3, 3)
    ok_kind = torch.arange(m, device=device) % 3
    # sheets: one thin box
    dims = _log_uniform(g, (m, 3), 0.2, 1.0, device)
    dims[:, 2] = _log_uniform(g, (m,), 1e-3, 1e-2, device)
    sheet = ok_kind == 0
    prm[sheet, 0] = dims[sheet] / 2
    # tori: R in [0.2, 1], r = R * U(0.1, 0.4)
    R = _log_uniform(g, (m,), 0.2, 1.0, device)
    r = R * (0.1 + 0.3 * _rand(g, (m,), device))
    tor = ok_kind == 1
    kind[tor, 0] = TORUS
    prm[tor, 0] = torch.stack([R, r, torch.zeros_like(R)], 1)[tor]
    # clusters: `pad` small boxes, edges 0.01..0.05, centres in a 0.15 cube
    cl = ok_kind == 2
    cd = _log_uniform(g, (m, P, 3), 0.01, 0.05, device)
    cc = 0.15 * _rand(g, (m, P, 3), device)
    prm[cl] = cd[cl] / 2
    center[cl] = cc[cl]
    flat = Primitives(kind.reshape(-1), center.reshape(-1, 3), rot.reshape(-1, 3, 3), prm.reshape(-1, 3),
                      torch.zeros((m * P, 3), dtype=torch.uint8, device=device))
    area = _area(flat).view(m, P)
    cdf = torch.cumsum(area, 1) / area.sum(1, keepdim=True)
    cdf[:, -1] = 1.0
    flat_cdf = (cdf + torch.arange(m, device=device, dtype=torch.float64)[:, None]).reshape(-1)
    bound = _bound_radius(flat).view(m, P)
    nprim = (area > 0).sum(1)
    sizes_t = torch.tensor(sizes, dtype=torch.int64, device=device)
    offs_t = torch.cumsum(sizes_t, 0) - sizes_t
    out = torch.empty((int(sizes_t.sum()), 3), dtype=torch.float32, device=device)
    have = torch.zeros(m, dtype=torch.int64, device=device)
    over = 1.2
    rounds = 0
    need = sizes_t.clone()
    while bool((need > 0).any()) and rounds < 16:
        rounds += 1
        want = torch.clamp((need.double() * over).ceil().long() + 16, min=0) * (need > 0)
        obj_all = torch.repeat_interleave(torch.arange(m, device=device), want)
        for s0 in range(0, int(obj_all.numel()), chunk):
            obj = obj_all[s0:s0 + chunk]
            u = _rand(g, (obj.numel(),), device) * 0.999999999 + obj.double()
            pid = torch.searchsorted(flat_cdf, u, right=True).clamp(max=m * P - 1)
            pid = torch.maximum(pid, obj * P)
            q, nrm, okk = _sample_local(g, flat, pid, device)
            pts = torch.einsum("mij,mj->mi", flat.rot[pid], q) + flat.center[pid]
            keep = okk.clone()
            own = pid - obj * P
            multi = nprim[obj] > 1
            for p in range(P):
                fp = obj * P + p
                near = keep & multi & (own != p) & \
                    ((pts - flat.center[fp]).pow(2).sum(1) < bound.view(-1)[fp] ** 2)
                idx = near.nonzero().squeeze(1)
                if idx.numel():
                    f = fp[idx]
                    ins = _inside_batched(flat.kind[f], flat.prm[f], flat.center[f], flat.rot[f], pts[idx])
                    keep[idx[ins]] = False
            kept = keep.nonzero().squeeze(1)
            ko = obj[kept]  # non-decreasing: samples are drawn object by object
            counts = torch.bincount(ko, minlength=m)
            starts = torch.cumsum(counts, 0) - counts
            rank = torch.arange(ko.numel(), device=device) - starts[ko]
            take = rank < (sizes_t - have)[ko]
            pos = offs_t[ko[take]] + have[ko[take]] + rank[take]
            out[pos] = pts[kept[take]].to(torch.float32)
            have += torch.bincount(ko[take], minlength=m)
        need = sizes_t - have
        over *= 1.5
    assert bool((need == 0).all()), "generator did not reach the requested sizes"
    offs = [0]
    for n in sizes:
        offs.append(offs[-1] + n)
    return out, offs


def scene_sizes(m: int = 10000, total: int = 1_500_000_000, lo: int = 5000, hi: int = 1_000_000,
                seed: int = 5) -> List[int]:
    """Object sizes of the heterogeneous scene: log-uniform in [lo, hi], then
    scaled so that they sum to `total` exactly."""
    s = log_uniform_sizes(m, lo, hi, seed)
    f = total / float(sum(s))
    out = [max(1, int(round(x * f))) for x in s]
    out[max(range(m), key=lambda j: out[j])] += total - sum(out)
    return out
