"""The paper's screen-space tool in the oracle (§4.3.1), pinned: the tool
transform against window coordinates computed in fp64, a window-sized
all-ones tool against the lasso with a screen-covering polygon, the world
area a disk tool cuts from a facing plane (pi r^2), and the orientation of
the shape texture."""

import math

import numpy as np
import pytest

import synth
from synth.edits import look_at_perspective


def test_tool_transform_matches_window_coordinates(orc):
    rng = np.random.default_rng(5)
    for _ in range(50):
        Ww, Wh = rng.integers(64, 4096, 2).astype(float)
        Tw, Th = rng.uniform(4, 400, 2)
        Tpx, Tpy = rng.uniform(0, Ww), rng.uniform(0, Wh)
        a = orc.tool_coeffs([Ww, Wh, Tpx, Tpy, Tw, Th]).astype(np.float64)
        xn = rng.uniform(-1, 1, 200)
        yn = rng.uniform(-1, 1, 200)
        # window position from the lower-left corner; the tool square
        # centred on (Tpx, Tpy) spans [0, 1]
        s_ref = ((xn + 1) * Ww / 2 - Tpx) / Tw + 0.5
        t_ref = ((yn + 1) * Wh / 2 - Tpy) / Th + 0.5
        s = xn * a[0] + a[1]
        t = yn * a[2] + a[3]
        scale = 1 + np.abs(s_ref) + Ww / Tw
        assert np.all(np.abs(s - s_ref) <= 1e-6 * scale)
        assert np.all(np.abs(t - t_ref) <= 1e-6 * (1 + np.abs(t_ref) + Wh / Th))


def _facing_plane(orc, W=512):
    A = np.array([[8.0, 0.0], [0.0, 8.0], [0.0, 0.0]])
    b = np.array([-4.0, -4.0, 0.0])
    m = synth.plane_grid(9, 9, A=A, b=b)
    g = orc.geometry_image(m, W, W)
    M = look_at_perspective((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0))
    D = orc.depth_map(m, M, 256, 256)
    return m, g, M, D


def test_window_sized_tool_is_the_full_screen_lasso(orc):
    wl = synth.tiny_workload()
    g = orc.geometry_image(wl.mesh, 256, 256)
    for ci in (0, 3, 7):
        M = wl.cameras[ci]
        D = orc.depth_map(wl.mesh, M, 128, 128)
        a = np.zeros(256 * 256, np.uint8)
        b = np.zeros(256 * 256, np.uint8)
        orc.tool(g.pos32, a, M, [640, 480, 320, 240, 640, 480], np.ones((8, 8), np.uint8), D, 1e-4, 3)
        orc.lasso(g.pos32, b, M, np.array([[-3, -3], [3, -3], [3, 3], [-3, 3]], np.float32), D, 1e-4, 3)
        assert (b == 3).sum() > 1000
        # the same selection, up to texels whose NDC is within rounding of
        # the window border (s = fmaf(xn, 1, 0.5) is then exactly in [0, 1])
        assert np.array_equal(a, b)


def test_disk_tool_on_facing_plane(orc):
    # plane z = 0 seen head-on from distance 4, 60 degree fovy: a window of
    # Wh pixels spans 2 * 4 tan(30 deg) world units; a disk of diameter Tw
    # pixels cuts a world disk of radius (Tw / 2) * that / Wh
    m, g, M, D = _facing_plane(orc)
    n = 512
    yy, xx = np.mgrid[0:n, 0:n]
    disk = (((xx + 0.5) / n - 0.5) ** 2 + ((yy + 0.5) / n - 0.5) ** 2 <= 0.25).astype(np.uint8)
    Ww = Wh = 1024
    for (Tpx, Tpy, Tw) in ((512, 512, 200), (300, 700, 120)):
        L = np.zeros(512 * 512, np.uint8)
        orc.tool(g.pos32, L, M, [Ww, Wh, Tpx, Tpy, Tw, Tw], disk, D, 1e-4, 9)
        unit = 2 * 4 * math.tan(math.radians(30)) / Wh     # world units per pixel
        r = Tw / 2 * unit
        area = orc.area(g, L)[9]
        assert abs(area / (math.pi * r * r) - 1) < 2e-2
        # centred on the tool position
        sel = L == 9
        cx, cy = (Tpx - Ww / 2) * unit, (Tpy - Wh / 2) * unit
        assert abs(g.pos[0, sel].mean() - cx) < 0.02 * r and abs(g.pos[1, sel].mean() - cy) < 0.02 * r


def test_shape_texture_orientation(orc):
    m, g, M, D = _facing_plane(orc)
    quad = np.zeros((4, 4), np.uint8)
    quad[:2, :2] = 1                       # rows 0-1 are t < 1/2, columns 0-1 s < 1/2
    L = np.zeros(512 * 512, np.uint8)
    orc.tool(g.pos32, L, M, [1000, 1000, 500, 500, 400, 400], quad, D, 1e-4, 4)
    sel = L == 4
    assert sel.sum() > 1000
    # lower-left quadrant of the tool: world x < 0 and y < 0 (x and y grow
    # with window x and y for this camera)
    assert (g.pos[0, sel] < 1e-6).all() and (g.pos[1, sel] < 1e-6).all()
    assert g.pos[0, sel].min() < -0.5 and g.pos[1, sel].min() < -0.5
