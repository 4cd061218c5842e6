"""Seeded edit streams, cameras, layer operations and request mixes.

The paper edits a layer with a tool placed by the user in window space and a
camera that also produces the depth texture (§4.3.1).  The workloads here draw
the equivalent inputs at random: brush spheres centred on the surface, lasso
polygons in normalised device coordinates seen from random cameras, layer
operations over random layer pairs, and Poisson request arrivals.  Cameras are
built in fp64 (look-at + GL perspective) and rounded once to a row-major fp32
4x4 matrix M with clip = M @ [x, y, z, 1].
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .mesh import (Mesh, vessel, scan_mesh, batch_model_mesh, max_model_mesh)

# layer algebra op codes (same numbering as the C library's uvl_op)
AND, OR, XOR, REMAP = 0, 1, 2, 3
U8, U16 = 1, 2


def look_at_perspective(eye, target, up, fovy_deg: float = 60.0, aspect: float = 1.0,
                        near: float = 0.1, far: float = 100.0) -> np.ndarray:
    """GL-style view-projection, fp64, rounded to fp32 row-major [16]."""
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    s = np.cross(f, np.asarray(up, dtype=np.float64))
    s /= np.linalg.norm(s)
    u = np.cross(s, f)
    V = np.eye(4)
    V[0, :3], V[1, :3], V[2, :3] = s, u, -f
    V[0, 3], V[1, 3], V[2, 3] = -s @ eye, -u @ eye, f @ eye
    g = 1.0 / math.tan(math.radians(fovy_deg) / 2.0)
    P = np.zeros((4, 4))
    P[0, 0] = g / aspect
    P[1, 1] = g
    P[2, 2] = (far + near) / (near - far)
    P[2, 3] = 2.0 * far * near / (near - far)
    P[3, 2] = -1.0
    return (P @ V).astype(np.float32).reshape(16)


def random_camera(rng: np.random.Generator, target, dist: float, aspect: float = 1.0) -> np.ndarray:
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    up = (0.0, 0.0, 1.0) if abs(d[2]) <= 0.99 else (1.0, 0.0, 0.0)
    return look_at_perspective(np.asarray(target) + dist * d, target, up, aspect=aspect)


def star_polygon(rng: np.random.Generator, n: int) -> np.ndarray:
    """Star-shaped NDC polygon: centre U[-.5,.5]^2, angle (k+U[0,.8]) 2pi/n, radius U[.1,.6]."""
    c = rng.uniform(-0.5, 0.5, size=2)
    ang = (np.arange(n) + rng.uniform(0.0, 0.8, size=n)) * (2.0 * math.pi / n)
    rad = rng.uniform(0.1, 0.6, size=n)
    pts = c[None, :] + rad[:, None] * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    return pts.astype(np.float32)


def area_cdf(mesh: Mesh) -> np.ndarray:
    p = mesh.pos.astype(np.float64)
    t = mesh.tri.astype(np.int64)
    a = 0.5 * np.linalg.norm(np.cross(p[t[:, 1]] - p[t[:, 0]], p[t[:, 2]] - p[t[:, 0]]), axis=1)
    return np.cumsum(a)


def surface_points(rng: np.random.Generator, mesh: Mesh, k: int, cdf=None) -> np.ndarray:
    """k points uniform on the surface: area-weighted triangle, uniform barycentric."""
    p = mesh.pos.astype(np.float64) if cdf is None else mesh.pos
    t = mesh.tri.astype(np.int64) if cdf is None else mesh.tri
    if cdf is None:
        cdf = area_cdf(mesh)
    pick = np.searchsorted(cdf, rng.uniform(0.0, cdf[-1], size=k), side="right")
    pick = np.minimum(pick, t.shape[0] - 1)
    r1 = np.sqrt(rng.uniform(size=k))
    r2 = rng.uniform(size=k)
    w0, w1, w2 = 1.0 - r1, r1 * (1.0 - r2), r1 * r2
    tp = t[pick].astype(np.int64)
    P = [p[tp[:, c]].astype(np.float64) for c in range(3)]
    pts = w0[:, None] * P[0] + w1[:, None] * P[1] + w2[:, None] * P[2]
    return pts.astype(np.float32)


def bounding_sphere(mesh: Mesh):
    lo = mesh.pos.min(axis=0).astype(np.float64)
    hi = mesh.pos.max(axis=0).astype(np.float64)
    c = 0.5 * (lo + hi)
    r = float(np.sqrt(((mesh.pos.astype(np.float64) - c) ** 2).sum(axis=1).max()))
    return c, r


@dataclass
class BrushEdit:
    layer: int
    centre: np.ndarray      # float32 [3]
    radius: np.float32
    label: int
    kind: str = "brush"


@dataclass
class LassoEdit:
    layer: int
    camera: int             # index into the workload's camera list
    poly: np.ndarray        # float32 [n, 2] NDC
    label: int
    kind: str = "lasso"


@dataclass
class LayerOp:
    op: int
    dst: int
    a: int
    b: int                  # ignored for REMAP
    sel_a: int
    sel_b: int
    out_label: int
    lut: Optional[np.ndarray] = None   # uint16 [256 | 65536], REMAP only


@dataclass
class Workload:
    name: str
    mesh: Mesh
    W: int
    H: int
    layer_dtypes: List[int]
    edits: list
    cameras: List[np.ndarray]
    depth_w: int
    depth_h: int
    bias: float
    ops: List[LayerOp] = field(default_factory=list)
    rho: int = 0


def _label(rng, dt):
    return int(rng.integers(1, 256 if dt == U8 else 65536))


def make_ops(rng: np.random.Generator, dtypes: List[int], n_ops: int) -> List[LayerOp]:
    """Random AND/OR/XOR/REMAP over random layer pairs (a != b)."""
    ops = []
    L = len(dtypes)
    for _ in range(n_ops):
        op = int(rng.integers(0, 4))
        a, b = (int(x) for x in rng.choice(L, size=2, replace=False))
        dst = int(rng.integers(0, L))
        sel_a = 0 if rng.uniform() < 0.5 else _label(rng, dtypes[a])
        sel_b = 0 if rng.uniform() < 0.5 else _label(rng, dtypes[b])
        out = _label(rng, dtypes[dst])
        lut = None
        if op == REMAP:
            na = 256 if dtypes[a] == U8 else 65536
            if dtypes[a] == dtypes[dst]:
                lut = np.concatenate([[0], 1 + rng.permutation(na - 1)]).astype(np.uint16)
            else:
                top = 256 if dtypes[dst] == U8 else 65536
                lut = rng.integers(1, top, size=na).astype(np.uint16)
                lut[0] = 0
            b = a
        ops.append(LayerOp(op, dst, a, b, sel_a, sel_b, out, lut))
    return ops


def _edit_stream(rng_e, rng_c, mesh, dtypes, n_brush, n_lasso, r_lo, r_hi,
                 n_poly, cam_dist, lassos_per_camera, label_max=None):
    kinds = np.array([0] * n_brush + [1] * n_lasso)
    kinds = kinds[rng_e.permutation(kinds.size)]
    centres = surface_points(rng_e, mesh, n_brush)
    c, _ = bounding_sphere(mesh)
    edits, cams = [], []
    bi = li = 0
    for k in kinds:
        layer = int(rng_e.integers(0, len(dtypes)))
        if label_max is not None:
            label = int(rng_e.integers(1, label_max + 1))
        else:
            label = _label(rng_e, dtypes[layer])
        if k == 0:
            r = np.float32(rng_e.uniform(r_lo, r_hi))
            edits.append(BrushEdit(layer, centres[bi], r, label))
            bi += 1
        else:
            if li % lassos_per_camera == 0:
                cams.append(random_camera(rng_c, c, cam_dist))
            n = n_poly if isinstance(n_poly, int) else int(rng_e.integers(n_poly[0], n_poly[1] + 1))
            edits.append(LassoEdit(layer, len(cams) - 1, star_polygon(rng_e, n), label))
            li += 1
    return edits, cams


def tiny_workload(noise_amp: float = 0.02) -> Workload:
    """Plain tiny case: 128^2-vertex vessel, 512^2 atlas, one u8 layer, 64 edits.

    32 brushes (r ~ U[0.05, 0.3], label 1..7) and 32 lassos (8-vertex stars,
    camera at distance 4 in a random direction, 256^2 depth map, bias 1e-4).
    """
    mesh = vessel(seed=0, noise_amp=noise_amp)
    rng_e = np.random.default_rng(1)
    rng_c = np.random.default_rng(2)
    dtypes = [U8]
    edits, cams = _edit_stream(rng_e, rng_c, mesh, dtypes, 32, 32, 0.05, 0.3, 8, 4.0, 1,
                               label_max=7)
    return Workload("vessel-512", mesh, 512, 512, dtypes, edits, cams, 256, 256, 1e-4)


def scan_workload(n_brush: int = 1000, n_lasso: int = 1000, n_ops: int = 256,
                  W: int = 8192, n_charts: int = 64, nx: int = 256, ny: int = 128,
                  depth: int = 2048) -> Workload:
    """Scan-scale case: 64 displaced 256x128 charts (4,145,280 tris) in 8192^2.

    8 u8 layers + 1 u16 layer; 1000 brushes (r ~ U[0.01, 0.2]) and 1000
    lassos (3-32 vertex stars, one camera per 8 lassos, 2048^2 depth maps);
    256 layer operations.  Smaller sizes keep the same structure.
    """
    mesh, rho = scan_mesh(seed=1000, n_charts=n_charts, nx=nx, ny=ny, W=W, H=W)
    rng_e = np.random.default_rng(1001)
    rng_c = np.random.default_rng(1002)
    rng_o = np.random.default_rng(1003)
    dtypes = [U8] * 8 + [U16]
    _, rad = bounding_sphere(mesh)
    edits, cams = _edit_stream(rng_e, rng_c, mesh, dtypes, n_brush, n_lasso, 0.01, 0.2,
                               (3, 32), 2.5 * rad, 8)
    ops = make_ops(rng_o, dtypes, n_ops)
    wl = Workload(f"scan-{W}", mesh, W, W, dtypes, edits, cams, depth, depth, 1e-4, ops, rho)
    return wl


def batch_workload(n_models: int = 256, t_lo: float = 1e4, t_hi: float = 1e6,
                   max_edits: int = 64, depth: int = 1024, seed: int = 2000):
    """Many independent models of uneven size, each with 1..max_edits pending edits.

    Triangle counts are log-uniform in [t_lo, t_hi]; half the edits are
    brushes (r ~ U[0.01, 0.2] of the model's bounding radius), half lassos
    (3-32 vertex stars, one camera per 8 lassos).  Returns a list of
    Workload, one per model, each with one u8 layer.
    """
    rng = np.random.default_rng(seed)
    out = []
    tris = np.exp(rng.uniform(math.log(t_lo), math.log(t_hi), size=n_models))
    for m in range(n_models):
        mesh, side = batch_model_mesh(seed + 10 + m, int(tris[m]))
        rng_e = np.random.default_rng(seed * 10 + 2 * m + 1)
        rng_c = np.random.default_rng(seed * 10 + 2 * m + 2)
        k = int(rng.integers(1, max_edits + 1))
        nb = int(rng.binomial(k, 0.5))
        _, rad = bounding_sphere(mesh)
        edits, cams = _edit_stream(rng_e, rng_c, mesh, [U8], nb, k - nb,
                                   0.01 * rad, 0.2 * rad, (3, 32), 2.5 * rad, 8)
        out.append(Workload(f"batch-{m}", mesh, side, side, [U8], edits, cams,
                            depth, depth, 1e-4))
    return out


def serve_workload(n_requests: int, qps: float, n_models: int, seed: int = 3004):
    """Poisson request stream over n_models: 60% brush, 25% lasso, 10% area, 5% algebra.

    Returns arrival times (seconds from start), request kinds (0 brush,
    1 lasso, 2 area, 3 algebra) and target models.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=n_requests)
    t = np.cumsum(gaps)
    kind = rng.choice(4, size=n_requests, p=[0.60, 0.25, 0.10, 0.05])
    model = rng.integers(0, n_models, size=n_requests)
    return t, kind, model


def serve_stream(meshes, layer_dtypes, n_requests: int, qps: float, seed: int = 3004,
                 n_cameras: int = 8, r_frac=(0.01, 0.2)):
    """Request stream for a serving run over several resident models.

    Poisson arrivals at `qps`; kinds 60% brush / 25% lasso / 10% area / 5%
    layer operation; uniform model choice.  Each model has n_cameras cameras
    (2.5x its bounding radius); brushes have r ~ U[r_frac] x bounding radius.
    Returns (cameras per model, list of request dicts with keys t, model,
    kind and edit | op | layer).
    """
    rng = np.random.default_rng(seed)
    t, kind, model = serve_workload(n_requests, qps, len(meshes), seed)
    cams, spheres, cdfs = [], [], []
    for k, m in enumerate(meshes):
        c, rad = bounding_sphere(m)
        rc = np.random.default_rng(seed * 7 + k)
        cams.append([random_camera(rc, c, 2.5 * rad) for _ in range(n_cameras)])
        spheres.append(rad)
        cdfs.append(area_cdf(m))
    out = []
    for i in range(n_requests):
        m = int(model[i])
        dts = layer_dtypes[m]
        L = int(rng.integers(0, len(dts)))
        req = {"t": float(t[i]), "model": m}
        if kind[i] == 0:
            c = surface_points(rng, meshes[m], 1, cdfs[m])[0]
            r = np.float32(rng.uniform(*r_frac) * spheres[m])
            req.update(kind="brush", edit=BrushEdit(L, c, r, _label(rng, dts[L])))
        elif kind[i] == 1:
            n = int(rng.integers(3, 33))
            req.update(kind="lasso", edit=LassoEdit(L, int(rng.integers(0, n_cameras)), star_polygon(rng, n),
                                                    _label(rng, dts[L])))
        elif kind[i] == 2:
            req.update(kind="area", layer=L)
        else:
            req.update(kind="algebra", op=make_ops(rng, dts, 1)[0] if len(dts) > 1 else None)
            if req["op"] is None:
                req.update(kind="area", layer=L)
        out.append(req)
    return cams, out


def max_workload(n_edits: int = 10000) -> Workload:
    """Largest single model: 16384^2 atlas, 8,258,048 triangles, 32 u8 layers."""
    mesh, rho = max_model_mesh()
    rng_e = np.random.default_rng(4001)
    rng_c = np.random.default_rng(4002)
    rng_o = np.random.default_rng(4003)
    dtypes = [U8] * 32
    _, rad = bounding_sphere(mesh)
    edits, cams = _edit_stream(rng_e, rng_c, mesh, dtypes, n_edits // 2, n_edits - n_edits // 2,
                               0.01, 0.2, (3, 32), 2.5 * rad, 8)
    ops = make_ops(rng_o, dtypes, 80)
    return Workload("max-16384", mesh, 16384, 16384, dtypes, edits, cams, 2048, 2048, 1e-4,
                    ops, rho)
