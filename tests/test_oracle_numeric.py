"""Numeric layers in the oracle (§4.2: data texture of integers or floats
plus a mask texture), pinned against what the number formats and the
geometry fix:

  - binary16 bit patterns that follow from the IEEE 754 format (normals,
    subnormals, ties to even, the largest finite value, overflow), and
    numpy's own double-to-half conversion on random values;
  - a mask packed by hand;
  - zonal statistics on an 8 x 8 plane seen as a W x W atlas, whose texel
    centres sit at x_i = 8 (i + 1/2) / W - 4: the discrete moments
    mean(x^2) = 16/3 (1 - 1/W^2), min x^2 = (4/W)^2, max x^2 = (4 - 4/W)^2,
    per-quadrant means of x of -2 and +2, the plane's area 64;
  - two charts of equal texel count but areas 64 and 4 holding 1 and 3:
    the area-weighted mean is 76/68, not the texel mean 2;
  - a brush SET selects pi r^2 of the plane and ERASE takes it back;
  - a range selection |x| <= 1 labels a band of area 16.
"""

import math

import numpy as np
import pytest

import synth
from oracle import numeric as N


@pytest.mark.parametrize("x,bits", [
    (1.0, 0x3C00), (-2.5, 0xC100), (0.5, 0x3800), (65504.0, 0x7BFF), (65519.99, 0x7BFF),
    (2.0 ** -14, 0x0400), (2.0 ** -24, 0x0001), (2.0 ** -25, 0x0000), (3 * 2.0 ** -25, 0x0002),
    (1 + 2.0 ** -11, 0x3C00), (1 + 3 * 2.0 ** -11, 0x3C02), (1 + 2.0 ** -11 + 2.0 ** -40, 0x3C01),
    (-0.0, 0x8000), (0.1, 0x2E66), (1 / 3, 0x3555), (2.0 ** -14 - 2.0 ** -25, 0x0400),
])
def test_f16_bits_from_the_format(x, bits):
    assert N.f16_bits(x) == bits


def test_f16_overflow_and_numpy_agreement():
    for x in (65520.0, -65520.0, 1e9, math.inf):
        with pytest.raises(OverflowError):
            N.f16_bits(x)
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.normal(0, 1, 4000), rng.normal(0, 1e4, 2000) % 65500,
                         rng.uniform(-1, 1, 2000) * 2.0 ** -14, rng.uniform(-1, 1, 2000) * 2.0 ** -23])
    want = xs.astype(np.float16).view(np.uint16)
    got = np.array([N.f16_bits(float(x)) for x in xs], np.uint16)
    assert np.array_equal(got, want)


def test_encode_ranges():
    assert N.encode(255, N.U8) == 255 and N.encode(65535, N.U16) == 65535
    assert N.encode(-2 ** 31, N.I32) == -2 ** 31 and N.encode(2 ** 31 - 1, N.I32) == 2 ** 31 - 1
    for v, dt in ((256, N.U8), (-1, N.U8), (65536, N.U16), (1.5, N.I32), (2 ** 31, N.I32),
                  (float("nan"), N.F32), (1e39, N.F32), (7e4, N.F16)):
        with pytest.raises(ValueError):
            N.encode(v, dt)
    assert N.encode(0.1, N.F32) == np.float32(0.1)
    assert N.encode(3.4e38, N.F32) == np.float32(3.4e38)


def test_mask_packing_by_hand():
    v = np.zeros(71, bool)
    v[[0, 5, 31, 32, 70]] = True
    w = N.pack_mask(v)
    assert w.dtype == np.uint32 and list(w) == [0x80000021, 0x1, 0x40]
    assert np.array_equal(N.unpack_mask(w, 71), v)
    assert N.pack_mask(np.ones(64, bool)).tolist() == [0xFFFFFFFF, 0xFFFFFFFF]


def _plane(orc, W):
    A = np.array([[8.0, 0.0], [0.0, 8.0], [0.0, 0.0]])
    m = synth.plane_grid(5, 5, A=A, b=(-4.0, -4.0, 0.0))
    g = orc.geometry_image(m, W, W)
    assert (g.tri_id >= 0).all()
    return g


@pytest.mark.parametrize("W", [64, 96])
def test_stats_plane_moments(orc, W):
    g = _plane(orc, W)
    x = g.pos[0]
    L = N.NumericLayer(W * W, N.F32)
    L.data[:] = (x * x).astype(np.float32)
    L.valid[:] = True
    s = N.stats(g.tri_id, g.w, L)[0]
    assert s["count"] == W * W
    assert abs(s["area"] - 64.0) < 1e-9
    assert abs(s["wsum"] / s["area"] - 16 / 3 * (1 - 1 / W ** 2)) < 1e-6
    assert abs(s["vmin"] - (4 / W) ** 2) <= 2 ** -23 * (4 / W) ** 2
    assert abs(s["vmax"] - (4 - 4 / W) ** 2) <= 2 ** -23 * 16
    # quadrant labels 1..4; mean x of each is -2 or +2, area 16, count W^2/4
    y = g.pos[1]
    region = (1 + (x > 0) + 2 * (y > 0)).astype(np.uint8)
    X = N.NumericLayer(W * W, N.F32)
    X.data[:] = x.astype(np.float32)
    X.valid[:] = True
    q = N.stats(g.tri_id, g.w, X, region)
    for lab, sx in ((1, -2), (2, 2), (3, -2), (4, 2)):
        assert q[lab]["count"] == W * W // 4
        assert abs(q[lab]["area"] - 16.0) < 1e-9
        assert abs(q[lab]["wsum"] / q[lab]["area"] - sx) < 1e-6
    assert q[0]["count"] == 0 and q[0]["vmin"] == np.inf and q[0]["vmax"] == -np.inf
    # texels outside the mask are left out
    X.valid[region != 2] = False
    q2 = N.stats(g.tri_id, g.w, X, region)
    assert q2[2]["count"] == W * W // 4 and q2[1]["count"] == 0


def test_stats_are_area_weighted(orc):
    W = 64
    big = synth.plane_grid(5, 5, uv0=(0.0, 0.0), uv1=(0.5, 1.0), A=((16.0, 0.0), (0.0, 8.0), (0.0, 0.0)),
                           b=(-4.0, -4.0, 0.0))
    small = synth.plane_grid(5, 5, uv0=(0.5, 0.0), uv1=(1.0, 1.0), A=((4.0, 0.0), (0.0, 2.0), (0.0, 0.0)),
                             b=(8.0, 0.0, 0.0))
    g = orc.geometry_image(synth.merge_meshes([big, small]), W, W)
    assert (g.tri_id >= 0).all()
    L = N.NumericLayer(W * W, N.F16)
    L.data[:] = np.where(g.pos[0] < 6.0, 1.0, 3.0).astype(np.float16)
    L.valid[:] = True
    s = N.stats(g.tri_id, g.w, L)[0]
    assert s["count"] == W * W and abs(s["area"] - 68.0) < 1e-9
    assert abs(s["wsum"] / s["area"] - 76.0 / 68.0) < 1e-12
    assert s["vmin"] == 1.0 and s["vmax"] == 3.0


def test_brush_set_then_erase(orc):
    W = 256
    g = _plane(orc, W)
    for dt, val in ((N.F32, 2.75), (N.F16, -0.1), (N.I32, -7), (N.U16, 40000), (N.U8, 3)):
        L = N.NumericLayer(W * W, dt)
        n = N.brush(g.pos32, L, (0.5, -0.25, 0.0), 2.0, N.SET, val)
        s = N.stats(g.tri_id, g.w, L)[0]
        assert s["count"] == n and abs(s["area"] / (math.pi * 4.0) - 1) < 1e-2
        assert s["vmin"] == s["vmax"] == float(N.encode(val, dt))
        assert (L.data[L.valid] == N.encode(val, dt)).all() and not L.data[~L.valid].any()
        N.brush(g.pos32, L, (0.5, -0.25, 0.0), 2.0, N.ERASE)
        assert not L.valid.any() and N.stats(g.tri_id, g.w, L)[0]["count"] == 0
        assert (L.data != 0).sum() == n                # ERASE keeps the data


def test_padding_never_changes_statistics(orc):
    """Padding writes uncovered texels only, so a numeric layer's statistics
    are the same before and after it, while the padded texels hold the
    value and are valid."""
    W = 128
    m = synth.plane_grid(5, 5, uv0=(0.2, 0.25), uv1=(0.7, 0.8), A=((8.0, 0.0), (0.0, 8.0), (0.0, 0.0)))
    g = orc.geometry_image(m, W, W)
    L = N.NumericLayer(W * W, N.I32)
    sel = np.zeros(W * W, np.uint8)
    orc.brush(g.pos32, sel, (2.0, 2.0, 0.0), 1.5, 1)
    N.brush(g.pos32, L, (2.0, 2.0, 0.0), 1.5, N.SET, -9)
    before = N.stats(g.tri_id, g.w, L)
    out = orc.outline(g.tri_id, W, W, 2)
    n = N.pad(out, sel, W, W, 2, L, N.SET, -9)
    assert n > 0 and (g.tri_id[L.valid & (sel == 0)] < 0).all()
    after = N.stats(g.tri_id, g.w, L)
    assert before.tobytes() == after.tobytes()
    assert (L.valid.sum() == (sel == 1).sum() + n) and (L.data[L.valid] == -9).all()
    N.pad(out, sel, W, W, 2, L, N.ERASE)
    assert L.valid.sum() == (sel == 1).sum()


def test_range_selection_band(orc):
    W = 128
    g = _plane(orc, W)
    L = N.NumericLayer(W * W, N.F32)
    L.data[:] = (g.pos[0] * g.pos[0]).astype(np.float32)
    L.valid[:] = True
    dst = np.zeros(W * W, np.uint8)
    n = N.select(L, 0.0, 1.0, dst, 5)
    # |x| <= 1: the band -1 <= x <= 1 of height 8, discretised to whole
    # texel columns of width 8 / W
    area = orc.area(g, dst)[5]
    assert n > 0 and abs(area - 16.0) <= 2 * 8 * (8 / W) + 1e-9
    assert N.select(L, 2.0, 1.0, dst, 6) == 0
    L.valid[:W * W // 2] = False
    assert N.select(L, 0.0, 1.0, dst, 7) == n // 2


# ---------------------------------------------------------------------------
# operations between numeric layers


def _layer(dtype, data, valid):
    L = N.NumericLayer(len(data), dtype)
    L.data[:] = np.asarray(data).astype(N.NP_DTYPE[dtype])
    L.valid[:] = np.asarray(valid, bool)
    return L


def test_mask_operations_inclusion_exclusion_and_data_source():
    # validity is set algebra on the masks: |A or B| = |A| + |B| - |A and B|,
    # A xor B = (A or B) minus (A and B), A and A = A, A xor A = nothing; a
    # valid result holds a's value where a is valid and b's elsewhere, and
    # texels left invalid keep dst's data
    rng = np.random.default_rng(11)
    n = 4099
    va, vb = rng.random(n) < 0.4, rng.random(n) < 0.6
    a = _layer(N.I32, rng.integers(-1000, 1000, n), va)
    b = _layer(N.I32, rng.integers(-1000, 1000, n), vb)
    out = {}
    for op in (N.NUM_AND, N.NUM_OR, N.NUM_XOR):
        d = _layer(N.I32, np.full(n, 77), np.ones(n, bool))
        out[op] = (N.combine(op, d, a, b), d)
    n_and, n_or, n_xor = out[N.NUM_AND][0], out[N.NUM_OR][0], out[N.NUM_XOR][0]
    assert n_or == va.sum() + vb.sum() - n_and
    assert n_xor == n_or - n_and
    d_or = out[N.NUM_OR][1]
    assert (d_or.data[va] == a.data[va]).all()
    assert (d_or.data[vb & ~va] == b.data[vb & ~va]).all()
    assert (d_or.data[~(va | vb)] == 77).all() and not d_or.valid[~(va | vb)].any()
    same = _layer(N.I32, a.data, va)
    assert N.combine(N.NUM_AND, same, same, same) == va.sum() and (same.valid == va).all()
    assert N.combine(N.NUM_XOR, same, same, same) == 0 and not same.valid.any()


@pytest.mark.parametrize("dtype", [N.U8, N.U16, N.I32, N.F16, N.F32])
def test_min_max_sum_identity_and_idempotence(dtype):
    # min(a, b) + max(a, b) = a + b and min <= max, each one of the two;
    # MIN(A, A) = MAX(A, A) = A
    rng = np.random.default_rng(dtype)
    n = 3000
    if dtype in N.INT_RANGE:
        lo, hi = N.INT_RANGE[dtype]
        xa, xb = rng.integers(lo, hi, n, endpoint=True), rng.integers(lo, hi, n, endpoint=True)
    else:
        xa = rng.normal(0, 100, n).astype(N.NP_DTYPE[dtype])
        xb = rng.normal(0, 100, n).astype(N.NP_DTYPE[dtype])
    v = rng.random(n) < 0.8
    a, b = _layer(dtype, xa, v), _layer(dtype, xb, np.ones(n, bool))
    mn, mx = _layer(dtype, np.zeros(n), v), _layer(dtype, np.zeros(n), v)
    N.combine(N.NUM_MIN, mn, a, b)
    N.combine(N.NUM_MAX, mx, a, b)
    A, B = a.data.astype(np.float64)[v], b.data.astype(np.float64)[v]
    lo_, hi_ = mn.data.astype(np.float64)[v], mx.data.astype(np.float64)[v]
    assert (lo_ + hi_ == A + B).all() and (lo_ <= hi_).all()
    assert ((lo_ == A) | (lo_ == B)).all()
    assert (mn.valid == v).all() and (mx.valid == v).all()
    c = _layer(dtype, a.data, v)
    N.combine(N.NUM_MIN, c, c, c)
    assert np.array_equal(c.data, a.data) and (c.valid == v).all()


def test_integer_sums_saturate_at_the_range():
    # u8 over every pair: the sum where it fits, 255 exactly when a + b >= 255
    x = np.repeat(np.arange(256), 256)
    y = np.tile(np.arange(256), 256)
    a, b = _layer(N.U8, x, np.ones(x.size, bool)), _layer(N.U8, y, np.ones(x.size, bool))
    d = _layer(N.U8, np.zeros(x.size), np.zeros(x.size, bool))
    N.combine(N.NUM_ADD, d, a, b)
    fits = x + y <= 255
    assert (d.data[fits].astype(np.int64) == (x + y)[fits]).all()
    assert (d.data[~fits] == 255).all()
    # the adding order does not matter and 0 is neutral
    d2 = _layer(N.U8, np.zeros(x.size), np.zeros(x.size, bool))
    N.combine(N.NUM_ADD, d2, b, a)
    assert np.array_equal(d.data, d2.data)
    big = 2 ** 31 - 1
    a = _layer(N.I32, [big, -big - 1, 5, -7], np.ones(4, bool))
    b = _layer(N.I32, [5, -1, -big - 1, big], np.ones(4, bool))
    d = _layer(N.I32, np.zeros(4), np.zeros(4, bool))
    N.combine(N.NUM_ADD, d, a, b)
    assert d.data.tolist() == [big, -big - 1, 5 - big - 1, big - 7]


def test_float_sums_round_once():
    rng = np.random.default_rng(5)
    # binary16: the exact sum rounded by the format's own rule (f16_bits,
    # pinned above by IEEE bit patterns), ties and subnormals included
    raw = rng.integers(0, 0x7C00, (2, 20000)).astype(np.uint16)      # finite positives
    raw[:, ::2] |= 0x8000                                             # and negatives
    h = raw.view(np.float16)
    a, b = _layer(N.F16, h[0], np.ones(h.shape[1], bool)), _layer(N.F16, h[1], np.ones(h.shape[1], bool))
    d = _layer(N.F16, np.zeros(h.shape[1]), np.zeros(h.shape[1], bool))
    N.combine(N.NUM_ADD, d, a, b)
    for k in range(h.shape[1]):
        s = float(h[0, k]) + float(h[1, k])          # exact in fp64
        try:
            want = N.f16_bits(s)
        except OverflowError:
            want = 0x7BFF | (0x8000 if s < 0 else 0)  # saturates at the largest finite value
        assert d.data.view(np.uint16)[k] == want, (h[0, k], h[1, k])
    # binary32: operands in [1, 2^20] have an exact double sum, whose
    # nearest binary32 is the correctly rounded sum
    fa = rng.uniform(1, 2 ** 20, 20000).astype(np.float32)
    fb = rng.uniform(1, 2 ** 20, 20000).astype(np.float32)
    a, b = _layer(N.F32, fa, np.ones(fa.size, bool)), _layer(N.F32, fb, np.ones(fa.size, bool))
    d = _layer(N.F32, np.zeros(fa.size), np.zeros(fa.size, bool))
    N.combine(N.NUM_ADD, d, a, b)
    exact = fa.astype(np.float64) + fb.astype(np.float64)
    assert np.array_equal(d.data, exact.astype(np.float32))
    top = np.finfo(np.float32).max
    a, b = _layer(N.F32, [top, -top], [1, 1]), _layer(N.F32, [top, -top], [1, 1])
    d = _layer(N.F32, [0, 0], [0, 0])
    N.combine(N.NUM_ADD, d, a, b)
    assert d.data.tolist() == [top, -top]
