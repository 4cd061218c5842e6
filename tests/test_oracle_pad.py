"""Texture padding in the oracle (§4.3.2), pinned without the oracle's own
window loops: Chebyshev distances from scipy's chessboard distance
transform, closed-form rings around rectangular islands, and invariants
(padding writes only uncovered texels, so it never changes an area; it is
idempotent; radius 0 pads nothing)."""

import numpy as np
import pytest
from scipy import ndimage

import oracle
import synth


def _chessboard_to(mask):
    """Chebyshev distance of every texel to the nearest True texel."""
    if not mask.any():
        return np.full(mask.shape, np.inf)
    return ndimage.distance_transform_cdt(~mask, metric="chessboard").astype(np.float64)


def _random_cover(rng, H, W, p):
    # blobs: a coarse random field upsampled, thresholded
    c = rng.random((H // 4 + 1, W // 4 + 1)) < p
    return np.kron(c, np.ones((4, 4), bool))[:H, :W]


@pytest.mark.parametrize("k", [1, 2, 3])
def test_outline_is_chessboard_ring(k):
    rng = np.random.default_rng(k)
    for (H, W, p) in ((37, 53, 0.3), (64, 64, 0.6), (5, 90, 0.5)):
        cov = _random_cover(rng, H, W, p)
        tri = np.where(cov, 0, -1).astype(np.int32)
        got = oracle.outline(tri, W, H, k).reshape(H, W).astype(bool)
        want = ~cov & (_chessboard_to(cov) <= k)
        assert np.array_equal(got, want)


def test_outline_of_a_rectangle_closed_form():
    W, H = 40, 30
    tri = np.full((H, W), -1, np.int32)
    tri[10:20, 5:17] = 3                        # a 12 x 10 island
    o = oracle.outline(tri, W, H, 1)
    assert o.sum() == 2 * (12 + 10) + 4         # the one-texel ring
    o2 = oracle.outline(tri, W, H, 2).reshape(H, W)
    assert o2.sum() == (12 + 4) * (10 + 4) - 12 * 10
    # clipped at the atlas border: an island in the corner
    tri2 = np.full((H, W), -1, np.int32)
    tri2[:3, :4] = 0
    assert oracle.outline(tri2, W, H, 1).sum() == (4 + 1) * (3 + 1) - 4 * 3


@pytest.mark.parametrize("k", [1, 2])
def test_pad_is_chessboard_neighbourhood_of_the_edit(k):
    rng = np.random.default_rng(10 + k)
    H, W = 48, 61
    cov = _random_cover(rng, H, W, 0.5)
    tri = np.where(cov, 0, -1).astype(np.int32)
    o = oracle.outline(tri, W, H, k)
    for trial in range(5):
        edited = cov & (rng.random((H, W)) < 0.05)
        layer = rng.integers(0, 200, H * W).astype(np.uint8)
        before = layer.copy()
        n = oracle.pad(o, edited, W, H, k, layer, 250)
        want = o.reshape(H, W).astype(bool) & (_chessboard_to(edited) <= k)
        got = (layer != before).reshape(H, W) | (want & (before.reshape(H, W) == 250))
        assert np.array_equal(got, want)
        assert n == want.sum()
        assert (layer.reshape(H, W)[want] == 250).all()
        assert np.array_equal(layer.reshape(H, W)[~want], before.reshape(H, W)[~want])


def test_padding_never_changes_area_and_is_idempotent():
    wl = synth.scan_workload(n_brush=6, n_lasso=0, n_ops=0, W=256, n_charts=4, nx=32, ny=16, depth=64)
    W = H = 256
    g = oracle.geometry_image(wl.mesh, W, H)
    o = oracle.outline(g.tri_id, W, H, 1)
    assert o.sum() > 0 and not (o.astype(bool) & (g.tri_id >= 0)).any()
    layer = np.zeros(W * H, np.uint8)
    for e in wl.edits:
        sel = np.zeros(W * H, np.uint8)
        oracle.brush(g.pos32, sel, e.centre, e.radius * 3, 1)
        oracle.brush(g.pos32, layer, e.centre, e.radius * 3, e.label)
        a0 = oracle.area(g, layer)
        n = oracle.pad(o, sel, W, H, 1, layer, e.label)
        assert n >= 0
        assert np.array_equal(oracle.area(g, layer), a0)        # outline texels weigh nothing
        snap = layer.copy()
        oracle.pad(o, sel, W, H, 1, layer, e.label)
        assert np.array_equal(layer, snap)                       # idempotent
    z = layer.copy()
    everything = (g.tri_id >= 0).astype(np.uint8)               # edits select covered texels only
    oracle.pad(o, everything, W, H, 0, z, 9)
    assert np.array_equal(z, layer)                              # radius 0 reaches no other texel
    oracle.pad(o, everything, W, H, 1, z, 9)
    ob = o.astype(bool)
    assert (z[ob] == 9).all() and np.array_equal(z[~ob], layer[~ob])   # radius 1 reaches the whole outline
