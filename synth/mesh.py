"""Seeded synthetic meshes with texture coordinates.

The paper stores every thematic layer as a 2D texture addressed by the mesh's
texture coordinates (§4.1, §4.2).  Its test models (scanned vessel, excavation,
statues; Fig. 5) are not available, so these generators stand in for them:

* ``vessel``   - a surface of revolution with one chart covering [0,1]^2, the
  shape class of the paper's vessel model;
* ``scan_mesh`` - many height-displaced grid charts, shelf-packed into one atlas
  with gutters, the structure of a scanned model's UV atlas;
* ``sphere`` / ``plane_grid`` - shapes with closed-form areas and positions,
  used to pin the oracle.

Everything here is fp64 numpy rounded once to fp32 at the end.  Nothing here
rasterises, selects or measures area.
"""

from __future__ import annotations

import math
from typing import NamedTuple, Sequence

import numpy as np


class Mesh(NamedTuple):
    pos: np.ndarray   # float32 [V, 3]
    nrm: np.ndarray   # float32 [V, 3]
    uv: np.ndarray    # float32 [V, 2]
    tri: np.ndarray   # int32   [T, 3]

    @property
    def nv(self) -> int:
        return int(self.pos.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tri.shape[0])


def grid_triangles(nx: int, ny: int) -> np.ndarray:
    """Triangles of an nx-by-ny vertex grid (vertex index j*nx + i).

    Each quad (i,j)-(i+1,j+1) is split on that diagonal.  With u growing with
    i and v with j both triangles are counter-clockwise in (u, v).
    """
    i, j = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="xy")
    v00 = (j * nx + i).ravel()
    v10 = v00 + 1
    v11 = v00 + nx + 1
    v01 = v00 + nx
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    tri = np.empty((2 * v00.size, 3), dtype=np.int64)
    tri[0::2] = t1
    tri[1::2] = t2
    return tri.astype(np.int32)


def vertex_normals(pos: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """Area-weighted average of incident face normals, fp64, normalised."""
    p = pos.astype(np.float64)
    t = tri.astype(np.int64)
    fn = np.cross(p[t[:, 1]] - p[t[:, 0]], p[t[:, 2]] - p[t[:, 0]])
    acc = np.zeros_like(p)
    for k in range(3):
        for c in range(3):
            acc[:, c] += np.bincount(t[:, k], weights=fn[:, c], minlength=p.shape[0])
    ln = np.linalg.norm(acc, axis=1, keepdims=True)
    ln[ln == 0] = 1.0
    return acc / ln


def _finish(pos64, nrm64, uv64, tri) -> Mesh:
    return Mesh(np.ascontiguousarray(pos64, dtype=np.float32),
                np.ascontiguousarray(nrm64, dtype=np.float32),
                np.ascontiguousarray(uv64, dtype=np.float32),
                np.ascontiguousarray(tri, dtype=np.int32))


def vessel(seed: int = 0, n: int = 128, noise_amp: float = 0.02) -> Mesh:
    """Vessel-like surface of revolution r(z) = 1 + 0.3 sin(3z) + noise.

    theta_i = 2 pi i/(n-1) (the seam column is duplicated at u = 1),
    z_j = pi j/(n-1); UV = (theta/2pi, z/pi) is a single chart over [0,1]^2.
    The radial noise is U[-amp, amp] per vertex and equal on both seam columns.
    128 x 128 vertices give 2 * 127^2 = 32,258 triangles.
    """
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.float64)
    j = np.arange(n, dtype=np.float64)
    theta = 2.0 * math.pi * i / (n - 1)
    z = math.pi * j / (n - 1)
    noise = rng.uniform(-noise_amp, noise_amp, size=(n, n)) if noise_amp > 0 else np.zeros((n, n))
    noise[:, n - 1] = noise[:, 0]
    r = 1.0 + 0.3 * np.sin(3.0 * z)[:, None] + noise           # [j, i]
    th = np.broadcast_to(theta[None, :], (n, n))
    zz = np.broadcast_to(z[:, None], (n, n))
    pos = np.stack([r * np.cos(th), r * np.sin(th), zz], axis=-1).reshape(-1, 3)
    uv = np.stack([np.broadcast_to(i[None, :] / (n - 1), (n, n)),
                   np.broadcast_to(j[:, None] / (n - 1), (n, n))], axis=-1).reshape(-1, 2)
    tri = grid_triangles(n, n)
    pos32 = pos.astype(np.float32)
    nrm = vertex_normals(pos32, tri)
    # the seam columns are one geometric vertex: give them the same normal
    nr = nrm.reshape(n, n, 3)
    s = nr[:, 0] + nr[:, n - 1]
    s /= np.maximum(np.linalg.norm(s, axis=1, keepdims=True), 1e-300)
    nr[:, 0] = s
    nr[:, n - 1] = s
    return _finish(pos, nr.reshape(-1, 3), uv, tri)


def sphere(radius: float = 1.0, n_theta: int = 257, n_phi: int = 129,
           centre=(0.0, 0.0, 0.0)) -> Mesh:
    """UV sphere: phi_j = pi j/(n_phi-1) from the south pole, theta_i = 2 pi i/(n_theta-1).

    UV = (theta/2pi, phi/pi); normals are the exact radial directions.
    """
    i = np.arange(n_theta, dtype=np.float64)
    j = np.arange(n_phi, dtype=np.float64)
    th = (2.0 * math.pi * i / (n_theta - 1))[None, :]
    ph = (math.pi * j / (n_phi - 1))[:, None]
    d = np.stack([np.sin(ph) * np.cos(th), np.sin(ph) * np.sin(th),
                  -np.cos(ph) * np.ones_like(th)], axis=-1).reshape(-1, 3)
    pos = d * radius + np.asarray(centre, dtype=np.float64)
    uv = np.stack([np.broadcast_to(i[None, :] / (n_theta - 1), (n_phi, n_theta)),
                   np.broadcast_to(j[:, None] / (n_phi - 1), (n_phi, n_theta))],
                  axis=-1).reshape(-1, 2)
    return _finish(pos, d, uv, grid_triangles(n_theta, n_phi))


def plane_grid(nx: int, ny: int, uv0=(0.0, 0.0), uv1=(1.0, 1.0),
               A=((1.0, 0.0), (0.0, 1.0), (0.0, 0.0)), b=(0.0, 0.0, 0.0),
               mirror: bool = False) -> Mesh:
    """Planar grid whose positions are an affine map of its texture coordinates.

    pos = A @ (u, v) + b for every vertex, so every point of the surface obeys
    the same map.  ``mirror`` reverses every triangle's winding.
    """
    u = np.linspace(uv0[0], uv1[0], nx)
    v = np.linspace(uv0[1], uv1[1], ny)
    uu, vv = np.meshgrid(u, v, indexing="xy")
    uv = np.stack([uu.ravel(), vv.ravel()], axis=1)
    A = np.asarray(A, dtype=np.float64)
    pos = uv @ A.T + np.asarray(b, dtype=np.float64)
    tri = grid_triangles(nx, ny)
    if mirror:
        tri = tri[:, [0, 2, 1]]
    n = np.cross(A[:, 0], A[:, 1])
    n = n / np.linalg.norm(n)
    if mirror:
        n = -n
    nrm = np.broadcast_to(n, pos.shape)
    return _finish(pos, nrm, uv, tri)


# ---------------------------------------------------------------------------
# displaced grid charts and atlas packing (scan-like models)


def value_noise(rng: np.random.Generator, s: np.ndarray, t: np.ndarray,
                extent=(2.0, 1.0), octaves: int = 4, base_freq: float = 4.0,
                gain: float = 0.5) -> np.ndarray:
    """Sum of octaves of lattice value noise (values U[-1,1], quintic fade)."""
    out = np.zeros(np.broadcast(s, t).shape, dtype=np.float64)
    amp = 1.0
    for o in range(octaves):
        f = base_freq * (2.0 ** o)
        nx = int(math.ceil(extent[0] * f)) + 2
        ny = int(math.ceil(extent[1] * f)) + 2
        lat = rng.uniform(-1.0, 1.0, size=(ny, nx))
        x = s * f
        y = t * f
        x0 = np.clip(np.floor(x).astype(np.int64), 0, nx - 2)
        y0 = np.clip(np.floor(y).astype(np.int64), 0, ny - 2)
        fx = x - x0
        fy = y - y0
        fx = fx * fx * fx * (fx * (fx * 6.0 - 15.0) + 10.0)
        fy = fy * fy * fy * (fy * (fy * 6.0 - 15.0) + 10.0)
        a = lat[y0, x0] * (1 - fx) + lat[y0, x0 + 1] * fx
        c = lat[y0 + 1, x0] * (1 - fx) + lat[y0 + 1, x0 + 1] * fx
        out += amp * (a * (1 - fy) + c * fy)
        amp *= gain
    return out


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def displaced_chart(rng: np.random.Generator, nx: int, ny: int,
                    extent=(2.0, 1.0), amp: float = 0.05, box: float = 8.0):
    """One height-displaced grid chart, rigidly placed inside a box^3 cube.

    Returns (pos64 [nx*ny,3], param [nx*ny,2] in chart units, tri [T,3]).
    """
    s = np.linspace(0.0, extent[0], nx)
    t = np.linspace(0.0, extent[1], ny)
    ss, tt = np.meshgrid(s, t, indexing="xy")
    h = amp * value_noise(rng, ss, tt, extent=extent)
    local = np.stack([ss - extent[0] / 2, tt - extent[1] / 2, h], axis=-1).reshape(-1, 3)
    R = random_rotation(rng)
    c = rng.uniform(1.0, box - 1.0, size=3)
    pos = local @ R.T + c
    param = np.stack([ss.ravel(), tt.ravel()], axis=1)
    return pos, param, grid_triangles(nx, ny)


def shelf_pack(rects: Sequence[tuple[int, int]], W: int, H: int, gutter: int = 2):
    """Shelf packing of integer rectangles (w, h) into W x H with gutters.

    Rectangles are placed tallest first, left to right, each shelf as tall as
    its first rectangle.  Returns the [x0, y0] corner per input rectangle, or
    None if they do not fit.
    """
    order = sorted(range(len(rects)), key=lambda k: (-rects[k][1], k))
    out = [None] * len(rects)
    x, y, shelf = gutter, gutter, 0
    for k in order:
        w, h = rects[k]
        if x + w + gutter > W:
            y += shelf + gutter
            x, shelf = gutter, 0
        if x + w + gutter > W or y + h + gutter > H:
            return None
        out[k] = (x, y)
        x += w + gutter
        shelf = max(shelf, h)
    return out


def atlas_mesh(charts, W: int, H: int, gutter: int = 2) -> tuple[Mesh, int]:
    """Pack charts (pos64, param, tri) with integer extents into one atlas.

    All charts get the same texel density rho (texels per chart unit), the
    largest one for which the shelf packing fits.  Each chart's rectangle
    starts on an integer texel boundary.  Returns (mesh, rho).
    """
    ext = [(int(round(p[:, 0].max())), int(round(p[:, 1].max()))) for _, p, _ in charts]
    lo, hi = 1, max(W, H)
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if shelf_pack([(e[0] * mid, e[1] * mid) for e in ext], W, H, gutter) is None:
            hi = mid - 1
        else:
            lo = mid
    rho = lo
    corners = shelf_pack([(e[0] * rho, e[1] * rho) for e in ext], W, H, gutter)
    if corners is None:
        raise ValueError("charts do not fit the atlas")
    pos_l, uv_l, tri_l, nrm_l = [], [], [], []
    base = 0
    for (pos, param, tri), (x0, y0) in zip(charts, corners):
        uv = np.stack([(x0 + param[:, 0] * rho) / W, (y0 + param[:, 1] * rho) / H], axis=1)
        pos_l.append(pos)
        uv_l.append(uv)
        tri_l.append(tri.astype(np.int64) + base)
        nrm_l.append(vertex_normals(pos.astype(np.float32), tri))
        base += pos.shape[0]
    pos = np.concatenate(pos_l)
    tri = np.concatenate(tri_l)
    return _finish(pos, np.concatenate(nrm_l), np.concatenate(uv_l), tri), rho


def merge_meshes(meshes: Sequence[Mesh]) -> Mesh:
    base = 0
    tris = []
    for m in meshes:
        tris.append(m.tri.astype(np.int64) + base)
        base += m.nv
    return Mesh(np.concatenate([m.pos for m in meshes]),
                np.concatenate([m.nrm for m in meshes]),
                np.concatenate([m.uv for m in meshes]),
                np.concatenate(tris).astype(np.int32))


def scan_mesh(seed: int = 1000, n_charts: int = 64, nx: int = 256, ny: int = 128,
              W: int = 8192, H: int = 8192, gutter: int = 2, amp: float = 0.05):
    """Scan-scale model: n_charts displaced 2x1 grid charts in one atlas.

    The default 64 charts of 256 x 128 vertices give 64 * 255 * 127 * 2 =
    4,145,280 triangles packed into 8192^2 with 2-texel gutters.
    Returns (mesh, rho).
    """
    rng = np.random.default_rng(seed)
    charts = [displaced_chart(rng, nx, ny, extent=(2.0, 1.0), amp=amp) for _ in range(n_charts)]
    return atlas_mesh(charts, W, H, gutter)


def batch_model_mesh(seed: int, n_tris: int, amp: float = 0.05):
    """A model of roughly n_tris triangles from ceil(n_tris/32258) square charts.

    The atlas side is 2^round(log2 sqrt(64 n_tris)) clamped to [1024, 8192].
    Returns (mesh, side).
    """
    rng = np.random.default_rng(seed)
    n_charts = max(1, math.ceil(n_tris / 32258))
    n = max(2, int(round(math.sqrt(n_tris / (2.0 * n_charts)))) + 1)
    side = 2 ** int(round(math.log2(math.sqrt(64.0 * n_tris))))
    side = min(8192, max(1024, side))
    charts = [displaced_chart(rng, n, n, extent=(1.0, 1.0), amp=amp) for _ in range(n_charts)]
    mesh, _ = atlas_mesh(charts, side, side, 2)
    return mesh, side


def max_model_mesh(seed: int = 4000, n_charts: int = 256, n: int = 128, side: int = 16384):
    """Largest single model: 256 charts of 128^2 vertices (8,258,048 triangles), 16384^2 atlas."""
    rng = np.random.default_rng(seed)
    charts = [displaced_chart(rng, n, n, extent=(1.0, 1.0), amp=0.05, box=16.0)
              for _ in range(n_charts)]
    return atlas_mesh(charts, side, side, 2)
