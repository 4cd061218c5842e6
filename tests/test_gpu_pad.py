"""Texture padding on the GPU (uvl_build_outline, uvl_pad_brush,
uvl_pad_lasso, uvl_numeric_pad_brush/lasso) against the oracle's padding,
bit for bit: the outline list equals the oracle's outline mask, and label
and numeric layers after edits each followed by its padding equal the
oracle's (edit, selection mask, padding)."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_14807_amd import uvl
    uvl.device_check()
    return uvl


def _scan_small():
    return synth.scan_workload(n_brush=24, n_lasso=24, n_ops=0, W=1024, n_charts=4, nx=64, ny=32, depth=512)


def test_outline_matches_oracle(gpu, orc):
    wl = _scan_small()
    dm = gpu.DeviceMesh.from_mesh(wl.mesh)
    for (W, H) in ((1024, 1024), (300, 200), (37, 53), (1, 1)):
        g = gpu.GeometryImage(W, H, normals=False, bary=False)
        gpu.build_geometry_image(dm, g)
        tri = g.host()["tri_id"]
        for k in (0, 1, 2):
            o = gpu.Outline(g, k)
            want = np.nonzero(orc.outline(tri, W, H, k))[0]
            assert o.n == want.size, (W, H, k)
            assert np.array_equal(o.numpy(), want), (W, H, k)
    # an outline list longer than the first guess of its capacity
    g = gpu.GeometryImage(37, 53, normals=False, bary=False)
    gpu.build_geometry_image(gpu.DeviceMesh.from_mesh(synth.plane_grid(3, 3, uv0=(0.45, 0.45), uv1=(0.55, 0.55))), g)
    o = gpu.Outline(g, 8)
    assert np.array_equal(o.numpy(), np.nonzero(orc.outline(g.host()["tri_id"], 37, 53, 8))[0])


@pytest.mark.parametrize("k", [1, 2])
def test_padding_matches_oracle(gpu, orc, k):
    from paper_2501_14807_amd.model import Model
    wl = _scan_small()
    W = H = wl.W
    m = Model.from_workload(wl).build()
    og = orc.geometry_image(wl.mesh, W, H)
    ol = orc.outline(og.tri_id, W, H, k)
    o = gpu.Outline(m.geom, k)
    assert np.array_equal(o.numpy(), np.nonzero(ol)[0])
    refs = [np.zeros(W * H, np.uint8 if dt == gpu.U8 else np.uint16) for dt in wl.layer_dtypes]
    depth_o = {}
    m.clear_layers()
    padded = 0
    for e in wl.edits:
        lay, ref = m.layers[e.layer], refs[e.layer]
        sel = np.zeros(W * H, np.uint8)
        if e.kind == "brush":
            gpu.edit_brush(m.geom, lay, e.centre, e.radius, e.label)
            gpu.pad_brush(m.geom, lay, o, e.centre, e.radius, e.label)
            orc.brush(og.pos32, sel, e.centre, e.radius, 1)
            orc.brush(og.pos32, ref, e.centre, e.radius, e.label)
        else:
            M = wl.cameras[e.camera]
            d = m.depth_for(e.camera, M)
            gpu.edit_lasso(m.geom, lay, M, e.poly, d, m.bias, e.label)
            gpu.pad_lasso(m.geom, lay, o, M, e.poly, d, m.bias, e.label)
            if e.camera not in depth_o:
                depth_o[e.camera] = orc.depth_map(wl.mesh, M, wl.depth_w, wl.depth_h)
            orc.lasso(og.pos32, sel, M, e.poly, depth_o[e.camera], m.bias, 1)
            orc.lasso(og.pos32, ref, M, e.poly, depth_o[e.camera], m.bias, e.label)
        padded += orc.pad(ol, sel, W, H, k, ref, e.label)
    assert padded > 0
    for L, ref in zip(m.layers, refs):
        assert np.array_equal(L.numpy(), ref)


def test_padding_writes_only_the_outline(gpu):
    """Radius 0 reaches no outline texel (they are all uncovered), and
    padding never touches covered texels."""
    import torch
    from paper_2501_14807_amd.model import Model
    wl = _scan_small()
    m = Model.from_workload(wl).build()
    o1 = gpu.Outline(m.geom, 1)
    lay = m.layers[0]
    m.clear_layers()
    e = [x for x in wl.edits if x.kind == "brush"][0]
    gpu.pad_brush(m.geom, lay, gpu.Outline(m.geom, 0), e.centre, 1e30, 7)
    assert not lay.numpy().any()
    gpu.pad_brush(m.geom, lay, o1, e.centre, 1e30, 7)
    got = lay.numpy()
    mask = np.zeros(got.size, bool)
    mask[o1.numpy()] = True
    assert (got[mask] == 7).all() and not got[~mask].any()


@pytest.mark.parametrize("k,dt", [(1, 4), (2, 3)])
def test_numeric_padding_matches_oracle(gpu, orc, k, dt):
    """Numeric layers (binary16, int32): each edit (every fifth an ERASE)
    followed by its padding, data bits and mask words against the oracle."""
    from oracle import numeric as N
    from paper_2501_14807_amd.model import Model
    wl = _scan_small()
    W = H = wl.W
    m = Model.from_workload(wl).build()
    og = orc.geometry_image(wl.mesh, W, H)
    ol = orc.outline(og.tri_id, W, H, k)
    o = gpu.Outline(m.geom, k)
    L = gpu.numeric_create(gpu.NumericLayer(W, H, dt))
    R = N.NumericLayer(W * H, dt)
    depth_o = {}
    padded = 0
    for i, e in enumerate(wl.edits):
        mode = N.ERASE if i % 5 == 4 else N.SET
        value = (i + 1) * (0.375 if dt == N.F16 else -3)
        sel = np.zeros(W * H, np.uint8)
        if e.kind == "brush":
            gpu.numeric_brush(m.geom, L, e.centre, e.radius, mode, value)
            gpu.numeric_pad_brush(m.geom, L, o, e.centre, e.radius, mode, value)
            orc.brush(og.pos32, sel, e.centre, e.radius, 1)
            N.brush(og.pos32, R, e.centre, e.radius, mode, value)
        else:
            M = wl.cameras[e.camera]
            d = m.depth_for(e.camera, M)
            gpu.numeric_lasso(m.geom, L, M, e.poly, d, m.bias, mode, value)
            gpu.numeric_pad_lasso(m.geom, L, o, M, e.poly, d, m.bias, mode, value)
            if e.camera not in depth_o:
                depth_o[e.camera] = orc.depth_map(wl.mesh, M, wl.depth_w, wl.depth_h)
            orc.lasso(og.pos32, sel, M, e.poly, depth_o[e.camera], m.bias, 1)
            N.lasso(og.pos32, R, M, e.poly, depth_o[e.camera], m.bias, mode, value)
        padded += N.pad(ol, sel, W, H, k, R, mode, value)
    assert padded > 0
    ut = np.uint16 if dt == N.F16 else np.uint32
    assert np.array_equal(L.numpy().view(ut), R.data.view(ut))
    assert np.array_equal(L.mask_words(), R.words)


def test_padded_waves_equal_edit_then_pad(gpu, orc):
    """Waves with padding: label and numeric layers end as after each edit
    followed by its padding, one launch each, in order (k = 1 and 2, tile
    culling on and off); tools pad by the same rule (checked against the
    oracle's padding of the tool's selection)."""
    import torch
    from oracle import numeric as N
    from paper_2501_14807_amd.model import Model
    wl = _scan_small()
    W = H = wl.W
    m = Model.from_workload(wl).build()
    maps = {}

    def depth(cam):
        if cam not in maps:
            d = torch.empty((m.depth_h, m.depth_w), dtype=torch.float32, device="cuda")
            gpu.render_depth(m.mesh, wl.cameras[cam], d, m.depth_ws)
            maps[cam] = d
        return maps[cam]

    edits = wl.edits[:40]
    for k in (1, 2):
        o = gpu.Outline(m.geom, k)
        lab = m.layers[0]
        num = gpu.NumericLayer(W, H, gpu.I32)
        # reference: edit, then its padding, one by one
        gpu.create_layer(lab)
        gpu.numeric_create(num)
        for i, e in enumerate(edits):
            mode = gpu.ERASE if i % 5 == 4 else gpu.SET
            label = 1 + i % 200
            if e.kind == "brush":
                gpu.edit_brush(m.geom, lab, e.centre, e.radius, label)
                gpu.pad_brush(m.geom, lab, o, e.centre, e.radius, label)
                gpu.numeric_brush(m.geom, num, e.centre, e.radius, mode, -i)
                gpu.numeric_pad_brush(m.geom, num, o, e.centre, e.radius, mode, -i)
            else:
                M = wl.cameras[e.camera]
                gpu.edit_lasso(m.geom, lab, M, e.poly, depth(e.camera), m.bias, label)
                gpu.pad_lasso(m.geom, lab, o, M, e.poly, depth(e.camera), m.bias, label)
                gpu.numeric_lasso(m.geom, num, M, e.poly, depth(e.camera), m.bias, mode, -i)
                gpu.numeric_pad_lasso(m.geom, num, o, M, e.poly, depth(e.camera), m.bias, mode, -i)
        torch.cuda.synchronize()
        ref = (lab.numpy().copy(), num.numpy().copy(), num.mask_words().copy())
        assert ref[0].any()
        for words in (1 << 20, 0):
            wave = gpu.Wave(max_edits=2 * len(edits), max_lassos=2 * len(edits), max_cull_words=words)
            gpu.create_layer(lab)
            gpu.numeric_create(num)
            batch = gpu.EditBatch()
            for i, e in enumerate(edits):
                mode = gpu.ERASE if i % 5 == 4 else gpu.SET
                label = 1 + i % 200
                if e.kind == "brush":
                    batch.brush(m.geom, lab, e.centre, e.radius, label)
                    batch.numeric_brush(m.geom, num, e.centre, e.radius, mode, -i)
                else:
                    M = wl.cameras[e.camera]
                    batch.lasso(m.geom, lab, M, e.poly, depth(e.camera), m.bias, label)
                    batch.numeric_lasso(m.geom, num, M, e.poly, depth(e.camera), m.bias, mode, -i)
            wave.submit(batch, outlines=[(m.geom, o)])
            torch.cuda.synchronize()
            assert np.array_equal(lab.numpy(), ref[0]), (k, words)
            assert np.array_equal(num.numpy(), ref[1]), (k, words)
            assert np.array_equal(num.mask_words(), ref[2]), (k, words)
            wave.close()
    # tools: one padded wave of three tools against the oracle
    og = orc.geometry_image(wl.mesh, W, H)
    ol = orc.outline(og.tri_id, W, H, 1)
    o = gpu.Outline(m.geom, 1)
    n = 64
    yy, xx = np.mgrid[0:n, 0:n]
    disk_np = ((((xx + 0.5) / n - 0.5) ** 2 + ((yy + 0.5) / n - 0.5) ** 2) <= 0.25).astype(np.uint8)
    disk = torch.from_numpy(disk_np).cuda().contiguous()
    cam = [e for e in wl.edits if e.kind == "lasso"][0].camera
    M = wl.cameras[cam]
    od = orc.depth_map(wl.mesh, M, wl.depth_w, wl.depth_h)
    tools = [(1024.0, 1024.0, 300.0, 500.0, 400.0, 300.0), (1024.0, 1024.0, 700.0, 450.0, 250.0, 250.0),
             (1024.0, 1024.0, 512.0, 512.0, 1024.0, 1024.0)]
    lab = m.layers[0]
    gpu.create_layer(lab)
    ref = np.zeros(W * H, np.uint8)
    batch = gpu.EditBatch()
    for q, t in enumerate(tools):
        batch.tool(m.geom, lab, M, t, disk, depth(cam), m.bias, 10 + q)
        sel = np.zeros(W * H, np.uint8)
        orc.tool(og.pos32, sel, M, t, disk_np, od, m.bias, 1)
        orc.tool(og.pos32, ref, M, t, disk_np, od, m.bias, 10 + q)
        orc.pad(ol, sel, W, H, 1, ref, 10 + q)
    wave = gpu.Wave(max_edits=8, max_lassos=8)
    wave.submit(batch, outlines=[(m.geom, o)])
    torch.cuda.synchronize()
    assert (ref[ol == 1] != 0).any()
    assert np.array_equal(lab.numpy(), ref)
    wave.close()


def test_padded_wave_rejects_bad_outlines(gpu):
    import ctypes
    from paper_2501_14807_amd.model import Model
    wl = _scan_small()
    m = Model.from_workload(wl).build()
    o = gpu.Outline(m.geom, 1)
    wave = gpu.Wave(max_edits=4, max_lassos=4)
    batch = gpu.EditBatch()
    e = [x for x in wl.edits if x.kind == "brush"][0]
    batch.brush(m.geom, m.layers[0], e.centre, e.radius, 3)
    L = gpu.lib()
    for idx, n, k in ((o.idx.data_ptr(), o.n, 9), (o.idx.data_ptr(), -1, 1), (None, 5, 1),
                      (o.idx.data_ptr(), m.geom.n + 1, 1)):
        ol = gpu.CWaveOutline(ctypes.addressof(m.geom.c), idx, n, k, 0)
        rc = L.uvl_wave_submit_padded(wave.h, batch.array(), len(batch), 0, ctypes.byref(ol), 1, None)
        assert rc == -1, (n, k)
    assert L.uvl_wave_submit_padded(wave.h, batch.array(), len(batch), 0, None, 1, None) == -1
    wave.close()
