"""Pins of the oracle's texture-space raster and geometry image (§4.3.1).

The paper delegates rasterisation to the GPU's fixed-function unit; the
oracle's reading is an 8-bit fixed-point snap, texel-centre samples and
half-open edge ownership.  These tests fix that reading from outside the
oracle: a partition of the atlas must be covered exactly once, a symbolic
perturbation (sample moved by (eta, eta^2)) must agree with the ownership
rule, positions of an affine chart must be the affine map of the texel
centre, and texel areas must integrate to the surface area.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import synth


def test_vessel_partition_exactly_once(orc):
    for amp in (0.0, 0.02):
        m = synth.vessel(noise_amp=amp)
        for (W, H) in ((512, 512), (37, 53), (300, 127)):
            g = orc.geometry_image(m, W, H, cover=True)
            assert (g.cover == 1).all(), (amp, W, H)
            assert (g.tri_id >= 0).all()


@pytest.mark.parametrize("mirror", [False, True])
def test_centre_lattice_box_is_half_open(orc, mirror):
    # vertices exactly on texel centres: boundary and interior edges pass
    # through rows and columns of centres; the box [a,c) x [b,d) results
    W, H = 64, 48
    a, b, c, d = 5, 7, 45, 39          # (c-a) % 4 == 0, (d-b) % 4 == 0
    m = synth.plane_grid(5, 5, uv0=((a + .5) / W, (b + .5) / H), uv1=((c + .5) / W, (d + .5) / H),
                         mirror=mirror)
    g = orc.geometry_image(m, W, H, cover=True)
    cov = g.cover.reshape(H, W)
    want = np.zeros((H, W), np.int32)
    want[b:d, a:c] = 1
    assert (cov == want).all()


def test_fan_centre_vertex_owned_once(orc):
    W = H = 32
    for k in (3, 5, 7, 8, 13):
        ang = np.arange(k) * 2 * math.pi / k + 0.1
        cx, cy = 16.5 / W, 16.5 / H
        pts = [(cx, cy)] + [(cx + 0.25 * math.cos(t), cy + 0.25 * math.sin(t)) for t in ang]
        uv = np.array(pts, np.float32)
        tri = np.array([[0, 1 + i, 1 + (i + 1) % k] for i in range(k)], np.int32)
        pos = np.concatenate([uv, np.zeros((k + 1, 1), np.float32)], axis=1)
        m = synth.Mesh(pos, np.tile([[0, 0, 1]], (k + 1, 1)).astype(np.float32), uv, tri)
        g = orc.geometry_image(m, W, H, cover=True)
        assert g.cover.reshape(H, W)[16, 16] == 1
        assert g.cover.max() == 1


def _perturbed_inside(P, V):
    """Exact inside test of sample P displaced by (eta, eta^2), eta -> 0+.

    The sample is inside the counter-clockwise triangle iff for every edge
    s->t the edge function at P + (eta, eta^2), a polynomial in eta, is
    positive, i.e. (e(P), -(ty-sy), (tx-sx)) > 0 lexicographically.
    """
    (x0, y0), (x1, y1), (x2, y2) = V
    area = (x1 - x0) * (y2 - y0) - (y1 - y0) * (x2 - x0)
    if area == 0:
        return False
    order = [0, 1, 2] if area > 0 else [0, 2, 1]
    for k in range(3):
        s, t = V[order[k]], V[order[(k + 1) % 3]]
        dx, dy = t[0] - s[0], t[1] - s[1]
        e = dx * (P[1] - s[1]) - dy * (P[0] - s[0])
        key = (e, -dy, dx)
        if not key > (0, 0, 0):
            return False
    return True


def test_ownership_matches_symbolic_perturbation(orc):
    rng = np.random.default_rng(7)
    W, H = 12, 10
    for trial in range(60):
        # vertices on the 1/256-texel grid, many of them on texel centres or
        # on lines through them
        q = rng.integers(0, 12 * 256, size=(3, 2))
        if trial % 2 == 0:
            q = (q // 128) * 128
        uv = np.stack([q[:, 0] / (256.0 * W), q[:, 1] / (256.0 * H)], axis=1).astype(np.float32)
        m = synth.Mesh(np.zeros((3, 3), np.float32), np.zeros((3, 3), np.float32), uv,
                       np.array([[0, 1, 2]], np.int32))
        g = orc.geometry_image(m, W, H, normals=False, cover=True)
        V = [(Fraction(int(x)), Fraction(int(y))) for x, y in q]
        for j in range(H):
            for i in range(W):
                P = (Fraction(256 * i + 128), Fraction(256 * j + 128))
                assert bool(g.cover[j * W + i]) == _perturbed_inside(P, V), (trial, i, j, q)


def test_lowest_index_wins_on_overlap(orc):
    W = H = 16
    m1 = synth.plane_grid(2, 2, uv0=(0.1, 0.1), uv1=(0.9, 0.9))
    m = synth.merge_meshes([m1, m1])         # same chart twice: tris 0,1 and 2,3
    g = orc.geometry_image(m, W, H, cover=True)
    cov = g.cover > 0
    assert (g.cover[cov] == 2).all()
    assert set(np.unique(g.tri_id[cov])) <= {0, 1}


def test_affine_chart_positions_and_bary(orc):
    # dyadic texture coordinates on the 1/(256 W) grid (snapping is exact)
    # and a dyadic map (vertex positions exact in fp32): the surface is then
    # exactly the affine image of texture space
    W, H = 96, 80
    A = np.array([[0.75, -0.25], [0.375, 1.125], [0.25, 0.5]])
    b = np.array([0.5, -1.0, 2.0])
    m = synth.plane_grid(7, 8, uv0=(3 / W, 5 / H), uv1=(93 / W, 75 / H), A=A, b=b)
    assert np.array_equal(m.pos.astype(np.float64), m.uv.astype(np.float64) @ A.T + b)
    g = orc.geometry_image(m, W, H)
    j, i = np.divmod(np.arange(W * H), W)
    cov = g.tri_id >= 0
    u = (i + 0.5) / W
    v = (j + 0.5) / H
    want = (np.stack([u, v], axis=1) @ A.T + b).T
    assert cov.sum() == (93 - 3) * (75 - 5)
    assert np.allclose(g.pos[:, cov], want[:, cov], rtol=0, atol=1e-12)
    assert np.isnan(g.pos[:, ~cov]).all()
    # barycentrics reproduce the texture coordinate of the centre
    t = m.tri[g.tri_id[cov]]
    b1, b2 = g.bary[0, cov], g.bary[1, cov]
    b0 = 1 - b1 - b2
    uvv = m.uv.astype(np.float64)
    rec_u = b0 * uvv[t[:, 0], 0] + b1 * uvv[t[:, 1], 0] + b2 * uvv[t[:, 2], 0]
    rec_v = b0 * uvv[t[:, 0], 1] + b1 * uvv[t[:, 1], 1] + b2 * uvv[t[:, 2], 1]
    assert np.allclose(rec_u, u[cov], atol=1e-12) and np.allclose(rec_v, v[cov], atol=1e-12)
    assert (b1 >= 0).all() and (b2 >= 0).all() and (b0 >= -1e-15).all()
    # normals: the plane's unit normal (vertex normals and face normals)
    n = np.cross(A[:, 0], A[:, 1])
    n /= np.linalg.norm(n)
    assert np.allclose(g.nrm[:, cov].T, n, atol=1e-7)
    g2 = orc.geometry_image(m, W, H, normals=False)
    assert np.allclose(g2.nrm[:, cov].T, n, atol=1e-12)
    # texel area of an affine chart: |A e_u x A e_v| / (W H), exactly
    jac = np.linalg.norm(np.cross(A[:, 0], A[:, 1]))
    assert np.allclose(g.w[cov], jac / (W * H), rtol=1e-12)
    assert (g.w[~cov] == 0).all()


def test_sphere_normals_radial(orc):
    m = synth.sphere(radius=2.0, n_theta=129, n_phi=65)
    g = orc.geometry_image(m, 256, 256)
    cov = g.tri_id >= 0
    p = g.pos[:, cov]
    nr = g.nrm[:, cov]
    radial = p / np.linalg.norm(p, axis=0)
    assert np.abs(nr - radial).max() < 5e-3
    assert np.allclose(np.linalg.norm(nr, axis=0), 1.0, atol=1e-12)


def _revolution_area(f, df, a, b):
    from scipy.integrate import quad
    return 2 * math.pi * quad(lambda z: f(z) * math.sqrt(1 + df(z) ** 2), a, b,
                              epsabs=1e-13, epsrel=1e-13, limit=200)[0]


def test_vessel_area_against_quadrature(orc):
    exact = _revolution_area(lambda z: 1 + 0.3 * math.sin(3 * z), lambda z: 0.9 * math.cos(3 * z),
                             0.0, math.pi)
    assert abs(exact - 24.683463437) < 1e-8
    m = synth.vessel(noise_amp=0.0)
    p = m.pos.astype(np.float64)
    t = m.tri.astype(np.int64)
    mesh_area = 0.5 * np.linalg.norm(np.cross(p[t[:, 1]] - p[t[:, 0]], p[t[:, 2]] - p[t[:, 0]]),
                                     axis=1).sum()
    assert abs(mesh_area / exact - 1) < 5e-4
    g = orc.geometry_image(m, 512, 512)
    tex = g.w.sum()
    assert abs(tex / mesh_area - 1) < 1e-3
    assert abs(tex / exact - 1) < 1e-3


def test_sphere_area(orc):
    R = 1.5
    m = synth.sphere(radius=R, n_theta=257, n_phi=129)
    g = orc.geometry_image(m, 1024, 1024)
    assert abs(g.w.sum() / (4 * math.pi * R * R) - 1) < 1e-3


def test_row_band_equals_full(orc):
    m = synth.vessel()
    full = orc.geometry_image(m, 200, 150)
    band = orc.geometry_image(m, 200, 150, rows=(40, 77))
    sl = slice(40 * 200, 77 * 200)
    assert (band.tri_id == full.tri_id[sl]).all()
    assert np.array_equal(band.pos, full.pos[:, sl], equal_nan=True)
    assert np.array_equal(band.w, full.w[sl])
