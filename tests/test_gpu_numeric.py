"""Numeric layers on the GPU (uvl_numeric_*) against the oracle's numeric
layers.

Bars: data bit patterns and mask words bit-exact after sequences of brush,
lasso and tool edits that SET and ERASE, in every dtype (including binary16
subnormal ties and rounding just above a tie, and the binary32 extremes),
on atlases whose width is a multiple of 32 (one mask word per 8 lanes), a
multiple of 4 only, and neither; range selections bit-exact; zonal
statistics with count, minimum and maximum exact, area within count times
the quantisation bound of one texel, and the weighted sum within the
rounding of fp64 sums in any order plus the area quantisation.  At the
benchmark's 8192^2 scan model: a numeric lasso selects exactly the texels
the label lasso selects, and statistics over sampled rows match the oracle
computed on those rows.
"""

import numpy as np
import pytest

import synth
from oracle import numeric as N

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_14807_amd import uvl
    uvl.device_check()
    return uvl


DTYPES = [N.U8, N.U16, N.I32, N.F16, N.F32]
VALUES = {N.U8: (200, 7), N.U16: (40000, 3), N.I32: (-123456, 2 ** 31 - 1),
          N.F16: (3 * 2.0 ** -25, 1 + 2.0 ** -11 + 2.0 ** -40), N.F32: (0.1, -3.4e38)}
UINT = {1: np.uint8, 2: np.uint16, 4: np.uint32}


def _bits(a):
    return np.ascontiguousarray(a).view(UINT[a.dtype.itemsize])


def _disk(n):
    yy, xx = np.mgrid[0:n, 0:n]
    return ((((xx + 0.5) / n - 0.5) ** 2 + ((yy + 0.5) / n - 0.5) ** 2) <= 0.25).astype(np.uint8)


def _scan_small():
    return synth.scan_workload(n_brush=12, n_lasso=12, n_ops=0, W=1024, n_charts=4, nx=64, ny=32, depth=512)


class _Scene:
    """A model at one atlas size on both sides, with depth maps per camera."""

    def __init__(self, gpu, orc, wl, W, H):
        import torch
        self.wl, self.W, self.H = wl, W, H
        self.dm = gpu.DeviceMesh.from_mesh(wl.mesh)
        self.g = gpu.GeometryImage(W, H, normals=False, bary=False)
        gpu.build_geometry_image(self.dm, self.g)
        self.og = orc.geometry_image(wl.mesh, W, H, normals=False)
        self.depth, self.odepth = {}, {}
        for e in wl.edits:
            if e.kind == "lasso" and e.camera not in self.depth:
                M = wl.cameras[e.camera]
                d = torch.empty((wl.depth_h, wl.depth_w), dtype=torch.float32, device="cuda")
                gpu.render_depth(self.dm, M, d)
                self.depth[e.camera] = d
                self.odepth[e.camera] = orc.depth_map(wl.mesh, M, wl.depth_w, wl.depth_h)


def _edit_both(gpu, sc, L, R, e, mode, value, shape, shape_np, tool):
    wl = sc.wl
    if e.kind == "brush":
        gpu.numeric_brush(sc.g, L, e.centre, e.radius, mode, value)
        N.brush(sc.og.pos32, R, e.centre, e.radius, mode, value)
    elif tool is None:
        M = wl.cameras[e.camera]
        gpu.numeric_lasso(sc.g, L, M, e.poly, sc.depth[e.camera], wl.bias, mode, value)
        N.lasso(sc.og.pos32, R, M, e.poly, sc.odepth[e.camera], wl.bias, mode, value)
    else:
        M = wl.cameras[e.camera]
        gpu.numeric_tool(sc.g, L, M, tool, shape, sc.depth[e.camera], wl.bias, mode, value)
        N.tool(sc.og.pos32, R, M, tool, shape_np, sc.odepth[e.camera], wl.bias, mode, value)


@pytest.mark.parametrize("W,H", [(1024, 1024), (256, 65), (132, 40), (37, 53)])
def test_numeric_edits_match_oracle(gpu, orc, W, H):
    import torch
    wl = _scan_small()
    sc = _Scene(gpu, orc, wl, W, H)
    shape_np = _disk(64)
    shape = torch.from_numpy(shape_np).cuda().contiguous()
    rng = np.random.default_rng(W * 7 + H)
    for dt in DTYPES:
        L = gpu.numeric_create(gpu.NumericLayer(W, H, dt))
        R = N.NumericLayer(W * H, dt)
        for i, e in enumerate(wl.edits):
            mode = N.ERASE if i % 4 == 3 else N.SET
            value = VALUES[dt][i % 2]
            tool = None
            if e.kind == "lasso" and i % 3 == 0:
                tool = (1024.0, 1024.0, float(rng.uniform(200, 800)), float(rng.uniform(200, 800)),
                        float(rng.uniform(100, 500)), float(rng.uniform(100, 500)))
            _edit_both(gpu, sc, L, R, e, mode, value, shape, shape_np, tool)
        if W >= 256:
            assert R.valid.any() and not R.valid.all(), dt
        assert np.array_equal(_bits(L.numpy()), _bits(R.data)), (W, H, dt)
        assert np.array_equal(L.mask_words(), R.words), (W, H, dt)


@pytest.mark.parametrize("W,H", [(1024, 1024), (37, 53)])
def test_range_selection_matches_oracle(gpu, orc, W, H):
    rng = np.random.default_rng(W + H)
    n = W * H
    vals = {N.U8: rng.integers(0, 256, n), N.U16: rng.integers(0, 65536, n),
            N.I32: rng.integers(-2 ** 31, 2 ** 31, n), N.F16: rng.normal(0, 100, n), N.F32: rng.normal(0, 1, n)}
    ranges = {N.U8: [(10, 200), (255, 255), (3, 2)], N.U16: [(1000, 1000), (0, 65535)],
              N.I32: [(-2 ** 31, 0), (-5.5, 1e9)], N.F16: [(-1.5, 1.5), (0.0, np.inf)],
              N.F32: [(-0.25, 0.5), (-np.inf, -1.0)]}
    for dt in DTYPES:
        R = N.NumericLayer(n, dt)
        R.data[:] = vals[dt].astype(N.NP_DTYPE[dt])
        R.valid[:] = rng.random(n) < 0.7
        L = gpu.NumericLayer(W, H, dt)
        L.copy_from(R.data, R.valid)
        assert np.array_equal(L.mask_words(), R.words)
        for ldt, npdt in ((gpu.U8, np.uint8), (gpu.U16, np.uint16)):
            base = rng.integers(0, 5, n).astype(npdt)
            ref = base.copy()
            dst = gpu.Layer(W, H, ldt)
            dst.copy_from(base)
            for k, (lo, hi) in enumerate(ranges[dt]):
                gpu.numeric_select(L, lo, hi, dst, 9 + k)
                N.select(R, lo, hi, ref, 9 + k)
            assert np.array_equal(dst.numpy(), ref), (W, H, dt, ldt)


def _check_stats(got, want, area_scale, abs_err, tag):
    nz = want["count"] > 0
    assert np.array_equal(got["count"], want["count"]), tag
    assert np.array_equal(got["vmin"][nz], want["vmin"][nz]) and np.array_equal(got["vmax"][nz], want["vmax"][nz]), tag
    assert (got["vmin"][~nz] == np.inf).all() and (got["vmax"][~nz] == -np.inf).all(), tag
    assert (got["area_w"][~nz] == 0).all() and (got["wsum"][~nz] == 0).all(), tag
    cnt = want["count"].astype(np.float64)
    area = got["area_w"].astype(np.float64) * area_scale
    assert (np.abs(area - want["area"]) <= cnt * abs_err + 1e-12 * want["area"]).all(), tag
    # each area quantised by at most abs_err; fp64 sums in any order
    # (the unquantised weights agree to 1e-12 relative)
    bound = want["abs_vsum"] * abs_err + ((cnt + 4) * 2.0 ** -51 + 1e-12) * want["abs_wsum"]
    assert (np.abs(got["wsum"] * area_scale - want["wsum"]) <= bound).all(), tag


@pytest.mark.parametrize("W,H", [(1024, 1024), (300, 200), (37, 53)])
def test_zonal_stats_match_oracle(gpu, orc, W, H):
    wl = _scan_small()
    sc = _Scene(gpu, orc, wl, W, H)
    n = W * H
    rng = np.random.default_rng(3 * W + H)
    jj, ii = np.divmod(np.arange(n), W)
    # coherent regions: blocks of 37 x 23 texels, labels 0..6 (u8) or up to
    # 3000 (u16)
    blk = (ii // 37) * 1000 + jj // 23
    reg8 = (blk % 7).astype(np.uint8)
    reg16 = (blk % 3001).astype(np.uint16)
    vals = {N.U8: rng.integers(0, 256, n), N.U16: rng.integers(0, 65536, n),
            N.I32: rng.integers(-2 ** 31, 2 ** 31, n), N.F16: rng.normal(0, 1000, n),
            N.F32: rng.normal(0, 1, n) * np.exp(rng.normal(0, 8, n))}
    regions = [None, (gpu.U8, reg8), (gpu.U16, reg16)]
    for dt in DTYPES:
        R = N.NumericLayer(n, dt)
        R.data[:] = vals[dt].astype(N.NP_DTYPE[dt])
        R.valid[:] = rng.random(n) < 0.8
        L = gpu.NumericLayer(W, H, dt)
        L.copy_from(R.data, R.valid)
        for reg in regions:
            if reg is None:
                got = gpu.numeric_stats(sc.g, L)
                want = N.stats(sc.og.tri_id, sc.og.w, R)
            else:
                lay = gpu.Layer(W, H, reg[0])
                lay.copy_from(reg[1])
                got = gpu.numeric_stats(sc.g, L, lay)
                want = N.stats(sc.og.tri_id, sc.og.w, R, reg[1])
            assert want["count"].sum() > 0
            _check_stats(got, want, sc.g.area_scale, sc.g.area_abs_err, (W, H, dt, reg and reg[0]))


def test_stats_empty_and_edited(gpu, orc):
    """No valid texel gives empty groups; after numeric edits the statistics
    match the oracle's over the same edits."""
    wl = _scan_small()
    W = H = 512
    sc = _Scene(gpu, orc, wl, W, H)
    L = gpu.numeric_create(gpu.NumericLayer(W, H, gpu.F32))
    s = gpu.numeric_stats(sc.g, L)[0]
    assert s["count"] == 0 and s["area_w"] == 0 and s["vmin"] == np.inf and s["vmax"] == -np.inf
    R = N.NumericLayer(W * H, N.F32)
    for i, e in enumerate(wl.edits):
        _edit_both(gpu, sc, L, R, e, N.SET, 0.5 + i, None, None, None)
    _check_stats(gpu.numeric_stats(sc.g, L), N.stats(sc.og.tri_id, sc.og.w, R), sc.g.area_scale,
                 sc.g.area_abs_err, "edited")


def test_scan_full_size_numeric(gpu, orc):
    """The 8192^2 scan model of the benchmark: a numeric lasso SET marks
    exactly the texels the label lasso selects, an ERASE by the same lasso
    clears them; statistics over six sampled rows (a region label on those
    rows) match the oracle computed on those rows."""
    import torch
    from paper_2501_14807_amd.model import Model
    wl = synth.scan_workload()
    m = Model.from_workload(wl).build()
    W, H, n = wl.W, wl.H, wl.W * wl.H
    L = gpu.numeric_create(gpu.NumericLayer(W, H, gpu.F32))
    lab = gpu.create_layer(gpu.Layer(W, H, gpu.U8))
    lassos = [e for e in wl.edits if e.kind == "lasso"][:3]
    for e in lassos:
        M = wl.cameras[e.camera]
        d = m.depth_for(e.camera, M)
        gpu.edit_lasso(m.geom, lab, M, e.poly, d, wl.bias, 1)
        gpu.numeric_lasso(m.geom, L, M, e.poly, d, wl.bias, gpu.SET, 2.5)
    sel = lab.data[:n] == 1
    valid = torch.from_numpy(L.valid()).cuda()
    assert int(sel.sum()) > 10000
    assert torch.equal(valid, sel)
    data = L.data[:n]
    assert bool((data[sel] == 2.5).all()) and not bool(data[~sel].any())
    e = lassos[0]
    gpu.numeric_lasso(m.geom, L, wl.cameras[e.camera], e.poly, m.depth_for(e.camera, wl.cameras[e.camera]),
                      wl.bias, gpu.ERASE)
    lab2 = gpu.create_layer(gpu.Layer(W, H, gpu.U8))
    gpu.edit_lasso(m.geom, lab2, wl.cameras[e.camera], e.poly, m.depth_for(e.camera, wl.cameras[e.camera]),
                   wl.bias, 1)
    valid = torch.from_numpy(L.valid()).cuda()
    assert torch.equal(valid, sel & (lab2.data[:n] != 1))
    del valid, sel, lab, lab2
    # statistics on sampled rows
    rng = np.random.default_rng(91)
    vals = rng.normal(0, 1, n).astype(np.float32)
    ok = rng.random(n) < 0.9
    L.copy_from(vals, ok)
    rows = sorted(rng.choice(H, size=6, replace=False).tolist())
    region = np.zeros(n, np.uint8)
    tri, w, v, val = [], [], [], []
    for r in rows:
        region[r * W:(r + 1) * W] = 1
        og = orc.geometry_image(wl.mesh, W, H, rows=(r, r + 1), normals=False)
        tri.append(og.tri_id)
        w.append(og.w)
        v.append(vals[r * W:(r + 1) * W])
        val.append(ok[r * W:(r + 1) * W])
    reg = gpu.Layer(W, H, gpu.U8)
    reg.copy_from(region)
    got = gpu.numeric_stats(m.geom, L, reg)
    R = N.NumericLayer(len(rows) * W, N.F32)
    R.data[:] = np.concatenate(v)
    R.valid[:] = np.concatenate(val)
    want = N.stats(np.concatenate(tri), np.concatenate(w), R)
    assert want["count"][0] > 0
    _check_stats(got[1:2], want, m.geom.area_scale, m.geom.area_abs_err, "full-size rows")


# ---------------------------------------------------------------------------
# operations between numeric layers


def _random_values(rng, dtype, n):
    """Values over the dtype's whole range, with its extremes and (floats)
    random bit patterns, so that sums saturate, round to ties and land on
    subnormals."""
    if dtype == N.U8:
        v = rng.integers(0, 256, n).astype(np.uint8)
        edge = [0, 1, 254, 255, 128]
    elif dtype == N.U16:
        v = rng.integers(0, 65536, n).astype(np.uint16)
        edge = [0, 1, 65534, 65535, 32768]
    elif dtype == N.I32:
        v = rng.integers(-2 ** 31, 2 ** 31, n, dtype=np.int64).astype(np.int32)
        edge = [-2 ** 31, 2 ** 31 - 1, -1, 0, 1]
    elif dtype == N.F16:
        b = rng.integers(0, 65536, n).astype(np.uint16)
        b[(b & 0x7c00) == 0x7c00] &= 0xbfff            # no inf / NaN
        v = b.view(np.float16)
        edge = [65504.0, -65504.0, 2.0 ** -24, -2.0 ** -24, 1.0, 2.0 ** -11, 0.0, -0.0, 65472.0]
    else:
        b = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
        b[(b & 0x7f800000) == 0x7f800000] &= 0xbfffffff
        v = b.view(np.float32)
        m = float(np.finfo(np.float32).max)
        edge = [m, -m, m / 2, 1.0, 2.0 ** -24, 2.0 ** -149, 0.0, -0.0]
    k = min(n, 4 * len(edge))
    v[:k] = np.resize(np.array(edge, dtype=v.dtype), k)
    return v


@pytest.mark.parametrize("dtype", DTYPES)
def test_numeric_ops_bit_exact(gpu, dtype):
    """AND / OR / XOR / MIN / MAX / ADD between numeric layers, into a third
    layer and in place (dst = a, dst = b), on sizes with and without whole
    mask words and 4-texel groups, against the oracle's numeric layers: data
    bits and mask words identical; the mask bits past the last texel stay."""
    rng = np.random.default_rng(4100 + dtype)
    for (W, H) in ((1024, 37), (37, 53), (300, 200), (1, 1), (4099, 3)):
        n = W * H
        print(f"case: dtype {dtype} size {W}x{H}", flush=True)
        for op in (N.NUM_AND, N.NUM_OR, N.NUM_XOR, N.NUM_MIN, N.NUM_MAX, N.NUM_ADD):
            for alias in (0, 1, 2):
                va, vb, vd = (rng.random(n) < p for p in (0.6, 0.5, 0.3))
                xa, xb, xd = (_random_values(rng, dtype, n) for _ in range(3))
                # the same pairs again with shuffled partners
                xb[n // 2:] = rng.permutation(xa[n // 2:])
                ra, rb, rd = N.NumericLayer(n, dtype), N.NumericLayer(n, dtype), N.NumericLayer(n, dtype)
                for r, x, v in ((ra, xa, va), (rb, xb, vb), (rd, xd, vd)):
                    r.data[:] = x
                    r.valid[:] = v
                A, B, D = (gpu.NumericLayer(W, H, dtype) for _ in range(3))
                A.copy_from(xa, va)
                B.copy_from(xb, vb)
                D.copy_from(xd, vd)
                nw = (n + 31) // 32
                if n % 32:
                    # bits past the last texel of dst's last word must stay
                    import torch
                    tail = np.array([np.uint32(0xffffffff) << np.uint32(n % 32)], np.uint32)
                    last = D.mask[nw - 1:nw].cpu().numpy().view(np.uint32) | tail
                    D.mask[nw - 1:nw].copy_(torch.from_numpy(last.view(np.int32)))
                gd, od = {0: (D, rd), 1: (A, ra), 2: (B, rb)}[alias]
                gpu.numeric_op(op, gd, A, B)
                N.combine(op, od, ra, rb)
                got_words = gd.mask_words()
                want_words = od.words
                if n % 32 and alias == 0:
                    want_words = want_words.copy()
                    want_words[-1] |= tail[0]
                tag = (W, H, op, alias)
                assert np.array_equal(_bits(gd.numpy()), _bits(od.data)), tag
                assert np.array_equal(got_words, want_words), tag


def test_numeric_ops_refuse_mismatches(gpu):
    A = gpu.NumericLayer(64, 8, N.F32)
    B = gpu.NumericLayer(64, 8, N.F16)
    C = gpu.NumericLayer(64, 9, N.F32)
    with pytest.raises(Exception):
        gpu.numeric_op(N.NUM_ADD, A, A, B)
    with pytest.raises(Exception):
        gpu.numeric_op(N.NUM_ADD, A, A, C)
    with pytest.raises(Exception):
        gpu.numeric_op(9, A, A, A)
