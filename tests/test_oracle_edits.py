"""Pins of the oracle's depth texture, brush and lasso selection (§4.3.1).

Closed forms: window depth of a tilted plane and of a sphere by exact ray
casting, of a floor that reaches behind the eye (clipped at the near plane)
and of a wall far beyond the guard band; a near occluder hiding a sphere;
an eye inside a closed mesh seeing it everywhere; Archimedes' cap (a ball of radius r centred on a sphere cuts a cap of
area pi r^2); the visible cap 2 pi R^2 (1 - R/d) seen from distance d; the
world-space rectangle a square lasso cuts from a plane facing the camera.
Brute force: even-odd crossing number against a winding-number angle sum.
"""

import math

import numpy as np
import pytest

import synth
from synth.edits import look_at_perspective

NEAR, FAR = 0.1, 100.0


def _window_depth(M64, p):
    c = M64 @ np.append(p, 1.0)
    return 0.5 * c[2] / c[3] + 0.5


def _pixel_ray(M64, x, y):
    Mi = np.linalg.inv(M64)
    a = Mi @ np.array([x, y, -1.0, 1.0])
    b = Mi @ np.array([x, y, 1.0, 1.0])
    a, b = a[:3] / a[3], b[:3] / b[3]
    return a, b - a


def test_depth_of_tilted_plane(orc):
    d = 4.0
    M = look_at_perspective((0.3, -0.2, d), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0))
    M64 = M.reshape(4, 4).astype(np.float64)
    A = np.array([[8.0, 0.0], [0.0, 6.0], [0.0, 4.0]])
    b = np.array([-4.0, -3.0, -2.0])
    m = synth.plane_grid(9, 9, A=A, b=b)
    Wd, Hd = 64, 48
    D = orc.depth_map(m, M, Wd, Hd)
    n = np.cross(A[:, 0], A[:, 1])
    checked = 0
    for iy in range(Hd):
        for ix in range(Wd):
            x = (2 * ix + 1) / Wd - 1
            y = (2 * iy + 1) / Hd - 1
            o, r = _pixel_ray(M64, x, y)
            t = n @ (b - o) / (n @ r)
            h = o + t * r
            uvh = np.linalg.lstsq(A, h - b, rcond=None)[0]
            if uvh.min() < 0.02 or uvh.max() > 0.98:
                continue
            assert abs(D[iy, ix] - _window_depth(M64, h)) < 2e-6, (ix, iy)
            checked += 1
    assert checked > 0.5 * Wd * Hd


@np.errstate(all="ignore")
def test_depth_of_sphere_and_background(orc):
    R, d = 1.0, 4.0
    m = synth.sphere(radius=R, n_theta=257, n_phi=129)
    M = look_at_perspective((0.0, -d, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    M64 = M.reshape(4, 4).astype(np.float64)
    Wd = Hd = 256
    D = orc.depth_map(m, M, Wd, Hd)
    iy, ix = np.mgrid[0:Hd, 0:Wd]
    x = (2 * ix + 1) / Wd - 1
    y = (2 * iy + 1) / Hd - 1
    Mi = np.linalg.inv(M64)
    ndc = lambda z: np.stack([x, y, np.full_like(x, z), np.ones_like(x)], -1) @ Mi.T
    a, b = ndc(-1.0), ndc(1.0)
    o = a[..., :3] / a[..., 3:]
    r = b[..., :3] / b[..., 3:] - o
    r /= np.linalg.norm(r, axis=-1, keepdims=True)
    bq = (o * r).sum(-1)
    disc = bq * bq - ((o * o).sum(-1) - R * R)
    assert (D[disc < -0.02] == 1.0).all()          # rays that miss see the clear value
    hit = disc > 0.02                               # away from the silhouette
    h = o + (-bq - np.sqrt(np.maximum(disc, 0)))[..., None] * r
    wd = lambda p: (lambda c: 0.5 * c[..., 2] / c[..., 3] + 0.5)(
        np.concatenate([p, np.ones(p.shape[:-1] + (1,))], -1) @ M64.T)
    err = D - wd(h)
    # The inscribed polyhedron lies at most one sagitta (< 2.5e-4 R at these
    # angular steps) inside the sphere, i.e. sagitta / cos(incidence) along
    # the ray; the 1/256-pixel vertex snap moves it sideways by < 1/256 px,
    # i.e. by that times tan(incidence) along the ray.
    cosi = np.abs((r * h).sum(-1)) / R
    px = 2 * np.linalg.norm(h - o, axis=-1) * math.tan(math.radians(30)) / Wd
    lat = px / 256 * np.sqrt(1 - cosi ** 2) / cosi
    hi = wd(h + ((2.5e-4 * R / cosi) + lat)[..., None] * r) - wd(h)
    lo = wd(h) - wd(h - lat[..., None] * r)
    tol = 3e-7                                      # fp32 vertex depths
    assert (err[hit] < hi[hit] + tol).all()
    assert (err[hit] > -lo[hit] - tol).all()
    assert hit.sum() > 5000


def test_depth_plane_seen_edge_on_is_not_drawn(orc):
    m = synth.plane_grid(3, 3, A=((8.0, 0.0), (0.0, 8.0), (0.0, 0.0)), b=(-4.0, -4.0, 0.0))
    # the eye lies in the plane, looking along it: the plane projects to a
    # line (zero screen area), so nothing is drawn even though its triangles
    # reach behind the eye and are clipped
    M = look_at_perspective((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    assert (orc.depth_map(m, M, 16, 16) == 1.0).all()


def _floor(x0=-10.0, x1=50.0, half=30.0, z=-1.0, n=3):
    return synth.plane_grid(n, n, A=((x1 - x0, 0.0), (0.0, 2 * half), (0.0, 0.0)), b=(x0, -half, z))


def _ray_plane_depth(M64, Wd, Hd, z0):
    """Window depth of the plane z = z0 along every pixel's ray (nan where
    the ray does not meet it in front of the eye)."""
    out = np.full((Hd, Wd), np.nan)
    for iy in range(Hd):
        for ix in range(Wd):
            x = (2 * ix + 1) / Wd - 1
            y = (2 * iy + 1) / Hd - 1
            o, r = _pixel_ray(M64, x, y)
            if abs(r[2]) < 1e-12:
                continue
            t = (z0 - o[2]) / r[2]
            if t <= 0:
                continue
            out[iy, ix] = _window_depth(M64, o + t * r)
    return out


def test_depth_floor_through_the_near_plane(orc):
    """A floor whose triangles reach behind the eye (every one crosses the
    near plane): clipped, not dropped, so every pixel whose ray meets the
    floor within the far plane holds the floor's exact window depth."""
    m = _floor()
    M = look_at_perspective((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    M64 = M.reshape(4, 4).astype(np.float64)
    Wd, Hd = 48, 32
    D = orc.depth_map(m, M, Wd, Hd)
    want = _ray_plane_depth(M64, Wd, Hd, -1.0)
    # the floor spans x in [-10, 50], |y| <= 30: rays hitting it beyond
    # x = 45 or |y| = 25 are left out (its far edge), as are grazing ones
    ok = np.isfinite(want) & (want < 0.999)
    # Window depth of a plane is affine on the screen, so its gradient per
    # pixel g is one vector; each vertex snap moves a vertex by at most
    # sqrt(2)/512 pixel, which moves the interpolated depth by at most
    # |g| sqrt(2)/512 inside the triangle (the barycentrics sum to 1); the
    # vertices' fp32 window depths add 2^-24 at most.
    g = np.array([np.nanmedian(np.diff(want, axis=1)), np.nanmedian(np.diff(want, axis=0))])
    tol = np.hypot(*g) * math.sqrt(2) / 512 * 1.01 + 2.0 ** -24 + 1e-7
    checked = 0
    for j, i in zip(*np.nonzero(ok)):
        x = (2 * i + 1) / Wd - 1
        y = (2 * j + 1) / Hd - 1
        o, r = _pixel_ray(M64, x, y)
        h = o + (-1.0 - o[2]) / r[2] * r
        if h[0] > 45 or abs(h[1]) > 25:
            continue
        assert abs(D[j, i] - want[j, i]) < tol, (i, j, tol)
        checked += 1
    assert checked > 0.25 * Wd * Hd
    # the upper half of the view sees nothing
    assert (D[Hd // 2 + 1:] == 1.0).all()


def test_depth_near_occluder_hides_what_is_behind(orc):
    """A sphere below the floor of the previous case: the floor, clipped at
    the near plane, stays in front of it wherever both are seen, so the depth
    texture equals the floor's alone."""
    floor = _floor()
    ball = synth.sphere(radius=1.5, n_theta=65, n_phi=33)
    ball = synth.Mesh(ball.pos + np.array([6.0, 0.0, -3.0], np.float32), ball.nrm, ball.uv, ball.tri)
    both = synth.mesh.merge_meshes([floor, ball])
    M = look_at_perspective((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    Wd, Hd = 64, 64
    D_floor = orc.depth_map(floor, M, Wd, Hd)
    D_ball = orc.depth_map(ball, M, Wd, Hd)
    D = orc.depth_map(both, M, Wd, Hd)
    assert (D_ball < 1.0).sum() > 50                # the ball alone is in view
    assert np.array_equal(D, D_floor)


def test_depth_wall_beyond_the_guard_band(orc):
    """A wall facing the eye at distance 2 whose corners project to |ndc| of
    about 900: clipped to the guard band and drawn, every pixel at the
    wall's window depth."""
    m = synth.plane_grid(3, 3, A=((0.0, 0.0), (2000.0, 0.0), (0.0, 2000.0)), b=(2.0, -1000.0, -1000.0))
    M = look_at_perspective((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    M64 = M.reshape(4, 4).astype(np.float64)
    D = orc.depth_map(m, M, 32, 32)
    assert np.abs(D - _window_depth(M64, np.array([2.0, 0.0, 0.0]))).max() < 1e-6


def test_depth_eye_inside_a_closed_mesh(orc):
    """The eye at the centre of a sphere: triangles behind it and beside it
    are clipped at the near plane and the guard band; every pixel is drawn
    (no cracks where clipped triangles meet) at the depth of a point
    between the inscribed polyhedron's faces and the sphere."""
    R = 5.0
    m = synth.sphere(radius=R, n_theta=65, n_phi=33)
    M = look_at_perspective((0.0, 0.0, 0.0), (1.0, 0.3, 0.2), (0.0, 0.0, 1.0))
    M64 = M.reshape(4, 4).astype(np.float64)
    Wd = Hd = 64
    D = orc.depth_map(m, M, Wd, Hd).astype(np.float64)
    assert (D < 1.0).all()
    # along each pixel's ray from the eye, the faces lie between R - sag and
    # R (sag = R (1 - cos(pi / 32)) at these angular steps, generously);
    # window depth grows with the distance along a ray
    sag = R * (1 - math.cos(math.pi / 32))
    for iy in range(0, Hd, 3):
        for ix in range(0, Wd, 3):
            a, _ = _pixel_ray(M64, (2 * ix + 1) / Wd - 1, (2 * iy + 1) / Hd - 1)
            r = a / np.linalg.norm(a)
            lo, hi = _window_depth(M64, (R - sag) * r), _window_depth(M64, R * r)
            assert lo - 1e-5 <= D[iy, ix] <= hi + 1e-5, (ix, iy)


def _sphere_geom(orc, W=1024):
    m = synth.sphere(radius=1.0, n_theta=257, n_phi=129)
    return m, orc.geometry_image(m, W, W)


@pytest.fixture(scope="module")
def sphere_geom(orc):
    return _sphere_geom(orc)


def test_brush_spherical_cap(orc, sphere_geom):
    m, g = sphere_geom
    c = np.array([0.3, 0.5, math.sqrt(1 - 0.34)], np.float32)
    for r in (0.25, 0.6, 1.1):
        L = np.zeros(g.tri_id.size, np.uint8)
        n = orc.brush(g.pos32, L, c, r, 3)
        assert n == (L == 3).sum() > 0
        a = orc.area(g, L)
        assert abs(a[3] / (math.pi * r * r) - 1) < 1e-2, r
        # same set as the fp64 distance away from a thin boundary band
        dist = np.linalg.norm(g.pos - c.astype(np.float64)[:, None], axis=0)
        far = np.abs(dist - r) > 1e-5
        cov = g.tri_id >= 0
        assert ((L == 3)[far & cov] == (dist <= r)[far & cov]).all()
        assert not (L[~cov]).any()


def test_brush_idempotent_and_extremes(orc, sphere_geom):
    m, g = sphere_geom
    c = np.array([0.0, 0.0, 1.0], np.float32)
    L1 = np.zeros(g.tri_id.size, np.uint8)
    orc.brush(g.pos32, L1, c, 0.5, 9)
    L2 = L1.copy()
    orc.brush(g.pos32, L2, c, 0.5, 9)
    assert np.array_equal(L1, L2)
    # erase with label 0 restores the empty layer
    orc.brush(g.pos32, L2, c, 0.5, 0)
    assert not L2.any()
    # an infinite radius selects exactly the covered texels
    L3 = np.zeros(g.tri_id.size, np.uint16)
    orc.brush(g.pos32, L3, c, 1e30, 65535)
    assert np.array_equal(L3 == 65535, g.tri_id >= 0)


def _winding(x, y, poly):
    ang = np.arctan2(poly[:, 1] - y, poly[:, 0] - x)
    d = np.diff(np.append(ang, ang[0]))
    d = (d + np.pi) % (2 * np.pi) - np.pi
    return int(round(d.sum() / (2 * np.pi)))


def _seg_dist(x, y, poly):
    p = poly.astype(np.float64)
    q = np.roll(p, -1, axis=0)
    v = q - p
    t = np.clip(((x - p[:, 0]) * v[:, 0] + (y - p[:, 1]) * v[:, 1]) / (v ** 2).sum(1), 0, 1)
    return np.hypot(p[:, 0] + t * v[:, 0] - x, p[:, 1] + t * v[:, 1] - y).min()


def test_point_in_polygon_even_odd_vs_winding(orc):
    rng = np.random.default_rng(11)
    polys = [synth.star_polygon(rng, n) for n in (3, 5, 8, 17, 32)]
    # a pentagram: its inner pentagon has winding number 2 (even-odd: outside)
    k = np.arange(5)
    polys.append(np.stack([np.cos(4 * np.pi * k / 5), np.sin(4 * np.pi * k / 5)], 1).astype(np.float32) * 0.8)
    for poly in polys:
        pts = rng.uniform(-1.2, 1.2, size=(3000, 2)).astype(np.float32)
        for x, y in pts:
            if _seg_dist(float(x), float(y), poly) < 1e-4:
                continue
            w = _winding(float(x), float(y), poly.astype(np.float64))
            assert orc.point_in_polygon(x, y, poly) == (w % 2 == 1)
    assert not orc.point_in_polygon(0.0, 0.0, polys[-1])      # pentagram centre


def test_lasso_visible_cap(orc, sphere_geom):
    m, g = sphere_geom
    rng = np.random.default_rng(5)
    square = np.array([[-1.5, -1.5], [1.5, -1.5], [1.5, 1.5], [-1.5, 1.5]], np.float32)
    cov = g.tri_id >= 0
    for d, Wd in ((4.0, 2048), (2.5, 1024)):
        M = synth.random_camera(rng, (0.0, 0.0, 0.0), d)
        D = orc.depth_map(m, M, Wd, Wd)
        L = np.zeros(g.tri_id.size, np.uint8)
        orc.lasso(g.pos32, L, M, square, D, 1e-4, 1)
        # eye position from the matrix: the point mapped to clip w = 0, x = y = 0
        eye = np.linalg.solve(M.reshape(4, 4).astype(np.float64)[[0, 1, 3], :3],
                              -M.reshape(4, 4).astype(np.float64)[[0, 1, 3], 3])
        assert abs(np.linalg.norm(eye) - d) < 1e-4
        v = eye[:, None] - g.pos
        cosi = (g.nrm * v).sum(0) / np.linalg.norm(v, axis=0)
        # texels facing the eye within 60 deg are visible; back faces are
        # not, except within a pixel of the silhouette, where the depth
        # map's sample may miss the surface
        assert (L[cov & (cosi > 0.5)] == 1).all()
        assert not L[cov & (cosi < -0.15)].any()
        if d == 4.0:
            a = orc.area(g, L)[1]
            assert abs(a / (2 * math.pi * (1 - 1 / d)) - 1) < 1e-2
        # no depth test passes when the depth map is at the near plane
        L0 = np.zeros_like(L)
        orc.lasso(g.pos32, L0, M, square, np.zeros_like(D), 0.0, 1)
        assert not L0.any()


def test_lasso_square_on_facing_plane(orc):
    # plane z = 0 seen head-on from distance 4: NDC (x, y) maps to world
    # (x, y) * 4 tan(30 deg); a square lasso [0.2,0.6] x [-0.4,0] cuts the
    # world rectangle of those bounds
    A = np.array([[8.0, 0.0], [0.0, 8.0], [0.0, 0.0]])
    b = np.array([-4.0, -4.0, 0.0])
    m = synth.plane_grid(9, 9, A=A, b=b)
    W = 512
    g = orc.geometry_image(m, W, W)
    M = look_at_perspective((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0))
    D = orc.depth_map(m, M, 256, 256)
    poly = np.array([[0.2, -0.4], [0.6, -0.4], [0.6, 0.0], [0.2, 0.0]], np.float32)
    L = np.zeros(W * W, np.uint8)
    orc.lasso(g.pos32, L, M, poly, D, 1e-4, 5)
    s = 4.0 * math.tan(math.radians(30))
    sel = L == 5
    x, y = g.pos[0, sel], g.pos[1, sel]
    texel = 8.0 / W
    assert x.min() > 0.2 * s - texel and x.max() < 0.6 * s + texel
    assert y.min() > -0.4 * s - texel and y.max() < 0.0 + texel
    area = orc.area(g, L)[5]
    assert abs(area / (0.4 * s * 0.4 * s) - 1) < 2e-2


def _tiling(rng):
    """Polygons that tile [-1, 1]^2 exactly: 8 x 8 cells of side 1/4, each a
    square, a square with a repeated collinear vertex, two triangles on a
    random diagonal, a fan of four triangles around its centre, or an L-shaped
    hexagon plus the square it leaves.  Every coordinate is a multiple of
    1/16, so every difference and product in the crossing test is exact in
    fp32.  Vertex order is reversed and rotated at random."""
    q = 0.25
    tiles = []
    for cy in range(8):
        for cx in range(8):
            x0, y0 = -1 + cx * q, -1 + cy * q
            x1, y1 = x0 + q, y0 + q
            xm, ym = x0 + q / 2, y0 + q / 2
            kind = rng.integers(5)
            if kind == 0:
                polys = [[(x0, y0), (x1, y0), (x1, y1), (x0, y1)]]
            elif kind == 1:
                polys = [[(x0, y0), (xm, y0), (x1, y0), (x1, y1), (x0, y1)]]
            elif kind == 2:
                if rng.integers(2):
                    polys = [[(x0, y0), (x1, y0), (x1, y1)], [(x0, y0), (x1, y1), (x0, y1)]]
                else:
                    polys = [[(x0, y0), (x1, y0), (x0, y1)], [(x1, y0), (x1, y1), (x0, y1)]]
            elif kind == 3:
                c = [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
                polys = [[c[k], c[(k + 1) % 4], (xm, ym)] for k in range(4)]
            else:
                polys = [[(x0, y0), (x1, y0), (x1, ym), (xm, ym), (xm, y1), (x0, y1)],
                         [(xm, ym), (x1, ym), (x1, y1), (xm, y1)]]
            for p in polys:
                if rng.integers(2):
                    p = p[::-1]
                r = int(rng.integers(len(p)))
                tiles.append(np.array(p[r:] + p[:r], np.float32))
    return tiles


def test_point_in_polygon_boundary_rule_tiles_exactly_once(orc):
    # The crossing rule is half-open: a point on an edge or vertex belongs to
    # the polygon reached by moving it right by e and up by d, with
    # 0 < d << e infinitesimal.  So where polygons tile a region, every point
    # of the region -- on shared edges, on horizontal edges, at shared
    # vertices, at T-junctions -- is inside exactly one of them.  A > slipped
    # to >= on one side of the straddle test, or a <= in the crossing test,
    # puts such points in zero or two tiles.
    rng = np.random.default_rng(2501)
    tiles = _tiling(rng)
    boxes = [(t[:, 0].min(), t[:, 0].max(), t[:, 1].min(), t[:, 1].max()) for t in tiles]
    g = np.arange(-16, 16, dtype=np.float64) / 16.0            # every vertex and edge point of the grid
    fine = rng.integers(-64, 64, size=(600, 2)) / 64.0        # points on diagonals and inside cells
    pts = [(x, y) for y in g for x in g] + [tuple(p) for p in fine]
    for x, y in pts:
        hits = 0
        for t, (bx0, bx1, by0, by1) in zip(tiles, boxes):
            if bx0 <= x <= bx1 and by0 <= y <= by1:
                hits += orc.point_in_polygon(x, y, t)
        assert hits == 1, (x, y, hits)


def test_point_in_polygon_boundary_convention(orc):
    # The edges that hold their points are the ones the rule above gives: for
    # an axis-aligned square the lower and left edges and the lower-left
    # corner belong to it, the upper and right ones and the other corners do
    # not (either winding).
    sq = np.array([[0.0, 0.0], [0.5, 0.0], [0.5, 0.5], [0.0, 0.5]], np.float32)
    for poly in (sq, sq[::-1].copy()):
        inside = [(0.0, 0.0), (0.25, 0.0), (0.0, 0.25), (0.25, 0.25)]
        outside = [(0.5, 0.0), (0.5, 0.5), (0.0, 0.5), (0.25, 0.5), (0.5, 0.25)]
        for x, y in inside:
            assert orc.point_in_polygon(x, y, poly), (x, y)
        for x, y in outside:
            assert not orc.point_in_polygon(x, y, poly), (x, y)
    # a point on a slanted edge belongs to the polygon on the edge's right
    lower = np.array([[0.0, 0.0], [0.5, 0.0], [0.5, 0.5]], np.float32)
    upper = np.array([[0.0, 0.0], [0.5, 0.5], [0.0, 0.5]], np.float32)
    assert orc.point_in_polygon(0.25, 0.25, lower) and not orc.point_in_polygon(0.25, 0.25, upper)
