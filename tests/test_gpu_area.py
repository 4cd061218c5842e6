"""Per-label areas on the GPU against the oracle (Table 1: the surface area
one texel stands for, summed over a label's texels).

Bars: every non-zero bin within 1e-6 relative of the oracle's fp64 area,
empty bins exactly zero; the per-block area sums exact.  Cases: atlas widths above one 1024-column wave unit
and above 4096 columns, widths that are not multiples of 16 (the lanes' scalar
path), u8 and u16 layers in one fused query and one by one; a mesh whose
texel areas span a factor 1.6e5, which one 32-bit word per texel cannot hold
to 1e-6 (the build reports it and the binding rebuilds with two words), with
areas and zonal statistics held to the same bar.
"""

import ctypes

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


def _labels(rng, n, dt, top):
    """Blocky labels (runs of 64) with 10% scattered ones."""
    base = rng.integers(0, top, n // 64 + 1).repeat(64)[:n]
    noise = rng.integers(0, top, n)
    v = np.where(rng.uniform(size=n) < 0.1, noise, base)
    return v.astype(np.uint8 if dt == 1 else np.uint16)


def _dev_layer(gpu, arr, W, H, dt):
    lay = gpu.Layer(W, H, dt)
    lay.copy_from(arr)
    return lay


def _check_bins(got, ref, tag):
    nz = ref > 0
    assert nz.any(), tag
    assert np.allclose(got[nz], ref[nz], rtol=1e-6, atol=0), tag
    assert (got[~nz] == 0).all(), tag


@pytest.mark.parametrize("W,H", [(4100, 257), (8195, 40), (1030, 19), (4096, 64), (17, 300)])
def test_area_wide_and_ragged_atlases(gpu, orc, W, H):
    """The vessel at atlas widths over several wave units (4100, 8195), with
    ragged last units and widths that are not multiples of 16."""
    print(f"case: vessel areas at {W}x{H}", flush=True)
    wl = synth.tiny_workload()
    dm = gpu.DeviceMesh.from_mesh(wl.mesh)
    g = gpu.GeometryImage(W, H)
    gpu.build_geometry_image(dm, g)
    og = orc.geometry_image(wl.mesh, W, H)
    rng = np.random.default_rng(W * 7 + H)
    n = W * H
    specs = [(gpu.U8, 256), (gpu.U16, 65536), (gpu.U8, 5), (gpu.U16, 300)]
    arrs = [(_labels(rng, n, dt, top), dt) for dt, top in specs]
    layers = [_dev_layer(gpu, a, W, H, dt) for a, dt in arrs]
    fused = gpu.area_query(g, layers)
    for k, ((a, dt), got) in enumerate(zip(arrs, fused)):
        ref = orc.area(og, a)
        _check_bins(got, ref, (W, H, k))
        single = gpu.area_query(g, [layers[k]])[0]
        assert np.array_equal(single, got), (W, H, k)


@pytest.mark.parametrize("W,H", [(512, 512), (4100, 257), (1030, 19), (17, 300)])
def test_area_block_sums(gpu, W, H):
    """The geometry image's per-block area sums (blocks of 4 rows x 8
    columns, ragged at the right and bottom edges) equal the sums of the
    blocks' area words, exactly."""
    wl = synth.tiny_workload()
    dm = gpu.DeviceMesh.from_mesh(wl.mesh)
    g = gpu.GeometryImage(W, H)
    gpu.build_geometry_image(dm, g)
    h = g.host()
    aw = h["area_w"].astype(np.uint64).reshape(H, W)
    bw, bh = -(-W // 8), -(-H // 4)
    pad = np.zeros((bh * 4, bw * 8), np.uint64)
    pad[:H, :W] = aw
    want = pad.reshape(bh, 4, bw, 8).sum(axis=(1, 3)).reshape(-1)
    assert np.array_equal(h["area_blk"], want)
    assert want.sum() == aw.sum() > 0


def _two_scale_mesh():
    """Two planar charts side by side in texture space with equal UV areas:
    one a unit square in 3D, the other a 400 x 400 square, so texel areas
    differ by 1.6e5."""
    a = synth.mesh.plane_grid(17, 33, uv0=(0.0, 0.0), uv1=(0.5, 1.0), A=((2.0, 0.0), (0.0, 1.0), (0.0, 0.0)))
    b = synth.mesh.plane_grid(17, 33, uv0=(0.5, 0.0), uv1=(1.0, 1.0), A=((800.0, 0.0), (0.0, 400.0), (0.0, 0.0)),
                              b=(-400.0, 0.0, 5.0))
    return synth.mesh.merge_meshes([a, b])


def test_two_word_texel_areas(gpu, orc):
    """Texel areas 1.6e5 apart: one word per texel is refused with
    UVL_E_RANGE, the binding's retry gives two words, and every texel, bin and
    statistics group is within 1e-6 of the oracle."""
    import torch
    mesh = _two_scale_mesh()
    W, H = 1000, 300
    print(f"case: two-scale mesh {W}x{H}", flush=True)
    dm = gpu.DeviceMesh.from_mesh(mesh)
    og = orc.geometry_image(mesh, W, H)
    cov = og.w > 0
    assert og.w[cov].max() / og.w[cov].min() > 1e5
    # one word: refused (the planes are still written)
    g1 = gpu.GeometryImage(W, H)
    ws = torch.empty(gpu.lib().uvl_build_workspace_bytes(dm.nt, W, H), dtype=torch.uint8, device="cuda")
    st = gpu.lib().uvl_build_geometry_image(ctypes.byref(dm.c), ctypes.byref(g1.c), ws.data_ptr(), ws.numel(), None)
    assert st == gpu.E_RANGE
    # the binding rebuilds with two words
    g = gpu.GeometryImage(W, H)
    gpu.build_geometry_image(dm, g)
    assert g.wide and g.area_blk is None and g.c.area_blk is None
    h = g.host()
    assert np.array_equal(h["tri_id"], og.tri_id)
    a = (h["area_w_hi"].astype(np.float64) * 2.0 ** 32 + h["area_w"].astype(np.float64)) * g.area_scale
    assert (a[~cov] == 0).all()
    assert (np.abs(a[cov] - og.w[cov]) <= 2.0 ** -20 * og.w[cov]).all()
    assert g.area_abs_err == 0.5 * g.area_scale
    # areas: u8 and u16 layers, more u8 layers than one two-word launch holds
    rng = np.random.default_rng(5)
    n = W * H
    arrs = [(_labels(rng, n, gpu.U8, 256 if k % 2 else 9), gpu.U8) for k in range(18)]
    arrs.append((_labels(rng, n, gpu.U16, 65536), gpu.U16))
    layers = [_dev_layer(gpu, x, W, H, dt) for x, dt in arrs]
    fused = gpu.area_query(g, layers)
    for k, ((x, dt), got) in enumerate(zip(arrs, fused)):
        _check_bins(got, orc.area(og, x), ("two-word", k))
    assert gpu.lib().uvl_area_bin_count(ctypes.byref(g.c), (gpu.CLayer * 1)(layers[0].c), 1) == 512
    # zonal statistics of a binary32 layer over a u8 region
    R = N.NumericLayer(n, N.F32)
    R.data[:] = rng.uniform(-3, 7, n).astype(np.float32)
    R.valid[:] = rng.uniform(size=n) < 0.7
    L = gpu.NumericLayer(W, H, gpu.F32)
    L.copy_from(R.data, R.valid)
    reg = arrs[1][0]
    got = gpu.numeric_stats(g, L, layers[1])
    want = N.stats(og.tri_id, og.w, R, reg)
    nz = want["count"] > 0
    assert np.array_equal(got["count"], want["count"])
    assert np.array_equal(got["vmin"][nz], want["vmin"][nz]) and np.array_equal(got["vmax"][nz], want["vmax"][nz])
    area = (got["area_w_hi"].astype(np.float64) * 2.0 ** 32 + got["area_w"].astype(np.float64)) * g.area_scale
    assert np.allclose(area[nz], want["area"][nz], rtol=1e-6, atol=0)
    # each product w v off by 2^-20 relative at most, fp64 sums in any order
    bound = 2.0 ** -20 * want["abs_wsum"] + (want["count"] + 4) * 2.0 ** -51 * want["abs_wsum"]
    assert (np.abs(got["wsum"] * g.area_scale - want["wsum"]) <= bound).all()
