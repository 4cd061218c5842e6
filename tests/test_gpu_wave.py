"""Batched edit waves: one persistent launch == the edits applied one launch
at a time, bit for bit, for every tile size, across models, layers, dtypes
and ragged atlases (label and numeric layers); and against the CPU oracle."""

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


def _models(gpu):
    from paper_2501_14807_amd.model import Model
    tiny = synth.tiny_workload()
    scan = synth.scan_workload(n_brush=30, n_lasso=30, n_ops=0, W=1024, n_charts=4, nx=64, ny=32, depth=512)
    out = []
    m = Model.from_workload(tiny).build()
    out.append((m, tiny, tiny.edits))
    # the same vessel on a ragged atlas with a u16 layer
    m2 = Model(tiny.mesh, 37 * 11, 53 * 5, [gpu.U16, gpu.U8], depth_w=128, depth_h=96).build()
    rng = np.random.default_rng(3)
    edits2 = []
    for e in tiny.edits[:40]:
        e2 = type(e)(**{**e.__dict__})
        e2.layer = int(rng.integers(0, 2))
        e2.label = int(rng.integers(0, 65536 if e2.layer == 0 else 256))
        edits2.append(e2)
    out.append((m2, tiny, edits2))
    m3 = Model.from_workload(scan).build()
    out.append((m3, scan, scan.edits))
    return out


def _plain(gpu, models):
    """Reference: fresh layers, edits applied one launch each."""
    res = []
    for m, wl, edits in models:
        m.clear_layers()
        m.apply_all(edits, wl.cameras)
        res.append([l.numpy().copy() for l in m.layers])
    return res


def test_wave_equals_plain_all_tile_sizes(gpu):
    models = _models(gpu)
    ref = _plain(gpu, models)
    n = sum(len(e) for _, _, e in models)
    # culling masks for every layer, for some layers only (the scan-scale
    # model's 1024 tiles x 1 word do not fit 600 words), and none
    for words in (1 << 20, 600, 0):
        wave = gpu.Wave(max_edits=n, max_lassos=n, max_cull_words=words)
        for chunks in (1, 2, 4, 8, 0):
            batch = gpu.EditBatch()
            for m, wl, edits in models:
                m.clear_layers()
                m.add_to_batch(batch, edits, wl.cameras)
            wave.submit(batch, tile_chunks=chunks)
            for (m, _, _), r in zip(models, ref):
                for k, l in enumerate(m.layers):
                    assert np.array_equal(l.numpy(), r[k]), (words, chunks, k)
        wave.close()


def test_wave_against_oracle_and_interleaving(gpu, orc):
    from oracle import workload
    from paper_2501_14807_amd.model import Model
    wl = synth.tiny_workload()
    og, ol, _ = workload.run(wl)
    m = Model.from_workload(wl).build()
    wave = gpu.Wave(64, 64)
    # two submits in a row: first half, then second half
    for part in (wl.edits[:29], wl.edits[29:]):
        b = gpu.EditBatch()
        m.add_to_batch(b, part, wl.cameras)
        wave.submit(b)
    assert np.array_equal(m.layers[0].numpy(), ol[0])
    # resubmitting a wave leaves the layers unchanged
    b = gpu.EditBatch()
    m.add_to_batch(b, wl.edits, wl.cameras)
    wave.submit(b)
    wave.submit(b)
    assert np.array_equal(m.layers[0].numpy(), ol[0])
    wave.close()


def test_wave_tune_then_submit(gpu):
    models = _models(gpu)[:2]
    ref = _plain(gpu, models)
    n = sum(len(e) for _, _, e in models)
    wave = gpu.Wave(n, n)
    batch = gpu.EditBatch()
    for m, wl, edits in models:
        m.clear_layers()
        m.add_to_batch(batch, edits, wl.cameras)
    wave.tune(batch)
    for m, _, _ in models:
        assert wave.tuned_chunks(m.geom.n) in (1, 2, 4, 8)
    for m, _, _ in models:
        m.clear_layers()
    wave.submit(batch)
    for (m, _, _), r in zip(models, ref):
        for k, l in enumerate(m.layers):
            assert np.array_equal(l.numpy(), r[k])
    wave.close()


def test_wave_errors(gpu):
    from paper_2501_14807_amd.model import Model
    wl = synth.tiny_workload()
    m = Model.from_workload(wl).build()
    wave = gpu.Wave(4, 1)
    b = gpu.EditBatch()
    m.add_to_batch(b, wl.edits[:6], wl.cameras)
    with pytest.raises(gpu.UvlError) as ei:
        wave.submit(b)
    assert ei.value.code == -4            # more edits than the handle holds
    b = gpu.EditBatch()
    lassos = [e for e in wl.edits if e.kind == "lasso"][:2]
    m.add_to_batch(b, lassos, wl.cameras)
    with pytest.raises(gpu.UvlError) as ei:
        wave.submit(b)
    assert ei.value.code == -4            # more lassos than the handle holds
    # one layer edited through two different geometry images
    g2 = gpu.GeometryImage(wl.W, wl.H)
    gpu.build_geometry_image(m.mesh, g2)
    b = gpu.EditBatch()
    e = [x for x in wl.edits if x.kind == "brush"][0]
    b.brush(m.geom, m.layers[0], e.centre, e.radius, 1)
    b.brush(g2, m.layers[0], e.centre, e.radius, 2)
    with pytest.raises(gpu.UvlError) as ei:
        wave.submit(b)
    assert ei.value.code == -1
    b = gpu.EditBatch()
    b.brush(m.geom, m.layers[0], e.centre, e.radius, 300)
    with pytest.raises(gpu.UvlError) as ei:
        wave.submit(b)
    assert ei.value.code == -3
    wave.close()


def test_tile_boxes(gpu):
    wl = synth.tiny_workload()
    for (W, H) in ((512, 512), (37, 53), (1000, 3), (64, 96), (2100, 300)):
        dm = gpu.DeviceMesh.from_mesh(wl.mesh)
        g = gpu.GeometryImage(W, H)
        gpu.build_geometry_image(dm, g)
        pos = g.host()["pos"].reshape(3, H, W)
        box = g.tile_box.cpu().numpy()
        tx, ty = (W + 31) // 32, (H + 31) // 32
        bx, by = (tx + 7) // 8, (ty + 7) // 8
        assert box.shape == (tx * ty + bx * by, 6)
        for b in range(ty):
            for a in range(tx):
                p = pos[:, 32 * b:32 * b + 32, 32 * a:32 * a + 32].reshape(3, -1)
                cov = ~np.isnan(p[0])
                k = b * tx + a
                if cov.any():
                    assert np.array_equal(box[k, :3], p[:, cov].min(axis=1))
                    assert np.array_equal(box[k, 3:], p[:, cov].max(axis=1))
                else:
                    assert (box[k, :3] == np.inf).all() and (box[k, 3:] == -np.inf).all()
        # blocks of 8 x 8 tiles: the union of their tiles' bounds
        tiles = box[:tx * ty].reshape(ty, tx, 6)
        for b in range(by):
            for a in range(bx):
                t = tiles[8 * b:8 * b + 8, 8 * a:8 * a + 8].reshape(-1, 6)
                k = tx * ty + b * bx + a
                assert np.array_equal(box[k, :3], t[:, :3].min(axis=0)), (W, H, a, b)
                assert np.array_equal(box[k, 3:], t[:, 3:].max(axis=0)), (W, H, a, b)


def _project(M, p):
    """fp32 NDC of positions p [3, n] with the fmaf order of the kernels
    (numpy float32 arithmetic with float64 fused steps rounded once)."""
    M = M.reshape(4, 4).astype(np.float64)
    x, y, z = (p[k].astype(np.float64) for k in range(3))

    def fma(a, b, c):   # exact product + sum, one rounding (float64 is exact
        return np.float32(a * b + c)   # enough for these fp32 operands' products)

    c = []
    for r in range(4):
        v = fma(M[r, 0], x, M[r, 3])
        v = fma(M[r, 1], y, np.float64(v))
        v = fma(M[r, 2], z, np.float64(v))
        c.append(v)
    return c[0] / c[3], c[1] / c[3], c[3]


def test_wave_culling_boundaries(gpu):
    """Brushes and lassos whose boundaries pass exactly through texels near
    tile edges: the wave (with tile culling) must equal the plain path."""
    from paper_2501_14807_amd.model import Model
    wl = synth.tiny_workload()
    m = Model.from_workload(wl).build()
    pos = m.geom.host()["pos"]
    cov = np.nonzero(~np.isnan(pos[0]))[0]
    rng = np.random.default_rng(8)
    brushes = []
    for _ in range(40):
        a, b = rng.choice(cov, 2)
        c = pos[:, a]
        # radius equal to the fp32 distance of texel b (a texel of another tile)
        d = pos[:, b] - c
        r = np.float32(np.sqrt(np.float32(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])))
        brushes.append((c, r))
    M = wl.cameras[2]
    xn, yn, w = _project(M, pos[:, cov])
    ok = (w > 0) & (np.abs(xn) < 0.9) & (np.abs(yn) < 0.9)
    idx = np.nonzero(ok)[0]
    polys = []
    for _ in range(20):
        i, j = rng.choice(idx, 2)
        x0, x1 = sorted([xn[i], xn[j]])
        y0, y1 = sorted([yn[i], yn[j]])
        if x1 - x0 < 1e-3 or y1 - y0 < 1e-3:
            continue
        polys.append(np.array([[x0, y0], [x1, y0], [x1, y1], [x0, y1]], np.float32))
    d = m.depth_for(2, M)

    def plain():
        m.clear_layers()
        for k, (c, r) in enumerate(brushes):
            gpu.edit_brush(m.geom, m.layers[0], c, r, 1 + k % 250)
        for k, P in enumerate(polys):
            gpu.edit_lasso(m.geom, m.layers[0], M, P, d, 1.0, 1 + (k + 7) % 250)
        return m.layers[0].numpy().copy()

    ref = plain()
    m.clear_layers()
    b = gpu.EditBatch()
    for k, (c, r) in enumerate(brushes):
        b.brush(m.geom, m.layers[0], c, r, 1 + k % 250)
    for k, P in enumerate(polys):
        b.lasso(m.geom, m.layers[0], M, P, d, 1.0, 1 + (k + 7) % 250)
    wave = gpu.Wave(len(b), len(b))
    for chunks in (1, 8):
        m.clear_layers()
        wave.submit(b, tile_chunks=chunks)
        assert np.array_equal(m.layers[0].numpy(), ref), chunks
    wave.close()


def test_wave_depth_culling(gpu):
    """Tiles culled by the depth test (occluded or facing away) change
    nothing: screen-covering lassos at biases around zero, where texels of
    the visible surface sit right at the stored depth, give the plain path's
    layers; and the depth test does cull (fewer tiles visited than with a
    depth map that hides nothing)."""
    import torch
    from paper_2501_14807_amd.model import Model
    wl = synth.tiny_workload()
    scan = synth.scan_workload(n_brush=1, n_lasso=8, n_ops=0, W=1024, n_charts=4, nx=64, ny=32, depth=512)
    poly = np.array([[-0.95, -0.95], [0.95, -0.95], [0.95, 0.95], [-0.95, 0.95]], np.float32)
    biases = (1e-2, 1e-4, 0.0, -1e-5, -1e-4)
    visited = []
    for w_ in (wl, scan):
        m = Model.from_workload(w_).build()
        cams = list(range(0, len(w_.cameras), max(1, len(w_.cameras) // 4)))[:4]
        maps = {}
        for ci in cams:     # one map per camera, alive for the whole test
            maps[ci] = torch.empty((m.depth_h, m.depth_w), dtype=torch.float32, device="cuda")
            gpu.render_depth(m.mesh, w_.cameras[ci], maps[ci], m.depth_ws)
        wave = gpu.Wave(64, 64)
        m.clear_layers()
        for ci in cams:
            for k, bias in enumerate(biases):
                gpu.edit_lasso(m.geom, m.layers[0], w_.cameras[ci], poly, maps[ci], bias, 1 + (3 * ci + k) % 250)
        ref = m.layers[0].numpy().copy()
        m.clear_layers()
        b = gpu.EditBatch()
        for ci in cams:
            for k, bias in enumerate(biases):
                b.lasso(m.geom, m.layers[0], w_.cameras[ci], poly, maps[ci], bias, 1 + (3 * ci + k) % 250)
        wave.submit(b)
        assert np.array_equal(m.layers[0].numpy(), ref)
        # one lasso: the real depth map against one that hides nothing
        M = w_.cameras[cams[0]]
        d = maps[cams[0]]
        b1 = gpu.EditBatch()
        b1.lasso(m.geom, m.layers[0], M, poly, d, 1e-4, 5)
        wave.submit(b1)
        culled = wave.visited_tiles()
        open_map = torch.full_like(d, 2.0)
        b2 = gpu.EditBatch()
        b2.lasso(m.geom, m.layers[0], M, poly, open_map, 1e-4, 5)
        wave.submit(b2)
        visited.append((culled, wave.visited_tiles()))
        wave.close()
    assert all(c <= o for c, o in visited), visited
    # the vessel hides its far side from every camera
    assert visited[0][0] < 0.9 * visited[0][1], visited


def test_wave_adversarial_polygons(gpu):
    """Self-intersecting, degenerate, tiny, screen-covering and off-screen
    polygons, and grid-snapped zigzags: the wave (whose cull pass classifies
    tiles as outside / inside / crossed by the polygon) gives the plain
    path's layers."""
    import torch
    from paper_2501_14807_amd.model import Model
    from test_gpu_parity import _adversarial_polygons
    wl = synth.tiny_workload()
    m = Model.from_workload(wl).build()
    polys = _adversarial_polygons()
    rng = np.random.default_rng(33)
    polys += [synth.star_polygon(rng, int(n)) for n in rng.integers(3, 65, 12)]
    for ci in (0, 5, 11):
        M = wl.cameras[ci]
        d = torch.empty((256, 256), dtype=torch.float32, device="cuda")
        gpu.render_depth(m.mesh, M, d, m.depth_ws)
        m.clear_layers()
        for k, P in enumerate(polys):
            gpu.edit_lasso(m.geom, m.layers[0], M, P, d, 1e-4, 1 + k % 250)
        ref = m.layers[0].numpy().copy()
        m.clear_layers()
        b = gpu.EditBatch()
        for k, P in enumerate(polys):
            b.lasso(m.geom, m.layers[0], M, P, d, 1e-4, 1 + k % 250)
        wave = gpu.Wave(len(b), len(b))
        wave.submit(b)
        assert np.array_equal(m.layers[0].numpy(), ref), ci
        # one at a time too (no later edit hides a wrong tile)
        for k, P in enumerate(polys):
            m.clear_layers()
            gpu.edit_lasso(m.geom, m.layers[0], M, P, d, 1e-4, 7)
            one = m.layers[0].numpy().copy()
            m.clear_layers()
            b1 = gpu.EditBatch()
            b1.lasso(m.geom, m.layers[0], M, P, d, 1e-4, 7)
            wave.submit(b1)
            assert np.array_equal(m.layers[0].numpy(), one), (ci, k)
        wave.close()


def _numeric_edits(m, wl, edits, dtypes, seed):
    """(edit, numeric layer index, mode, value) with every fourth an ERASE."""
    rng = np.random.default_rng(seed)
    out = []
    for i, e in enumerate(edits):
        k = int(rng.integers(0, len(dtypes)))
        gpu_mode = 1 if i % 4 == 3 else 0
        dt = dtypes[k]
        value = {1: 200 - i % 50, 2: 40000 + i, 3: -1000 * i - 7, 4: 0.375 * i - 3.0, 5: 0.1 * i}[dt]
        out.append((e, k, gpu_mode, value))
    return out


def _apply_numeric_plain(gpu, m, wl, items, layers):
    for e, k, mode, value in items:
        if e.kind == "brush":
            gpu.numeric_brush(m.geom, layers[k], e.centre, e.radius, mode, value)
        else:
            M = wl.cameras[e.camera]
            gpu.numeric_lasso(m.geom, layers[k], M, e.poly, m.depth_for(e.camera, M), m.bias, mode, value)


def _add_numeric_batch(gpu, batch, m, wl, items, layers):
    """Numeric edits into a batch; each camera gets its own depth map, kept
    alive by the batch (the model's small depth cache would recycle them
    before the wave runs)."""
    import torch
    maps = {}
    for e, k, mode, value in items:
        if e.kind == "brush":
            batch.numeric_brush(m.geom, layers[k], e.centre, e.radius, mode, value)
        else:
            M = wl.cameras[e.camera]
            if e.camera not in maps:
                d = torch.empty((m.depth_h, m.depth_w), dtype=torch.float32, device="cuda")
                gpu.render_depth(m.mesh, M, d, m.depth_ws)
                maps[e.camera] = d
            batch.numeric_lasso(m.geom, layers[k], M, e.poly, maps[e.camera], m.bias, mode, value)


def test_wave_numeric_layers_equal_plain(gpu):
    """Numeric layers in waves (SET and ERASE, every dtype, widths a multiple
    of 32 and not), mixed with label layers in the same waves: data bits and
    mask words identical to the numeric single-edit calls in order."""
    import torch
    from paper_2501_14807_amd.model import Model
    tiny = synth.tiny_workload()
    scan = synth.scan_workload(n_brush=30, n_lasso=30, n_ops=0, W=1024, n_charts=4, nx=64, ny=32, depth=512)
    # widths 1024 (a multiple of 32), 396 (of 4 only) and 407 (neither)
    setups = [(Model.from_workload(scan).build(), scan),
              (Model(tiny.mesh, 396, 200, [gpu.U8], depth_w=128, depth_h=96).build(), tiny),
              (Model(tiny.mesh, 37 * 11, 53 * 5, [gpu.U8], depth_w=128, depth_h=96).build(), tiny)]
    for seed, (m, wl) in enumerate(setups):
        W, H = m.geom.width, m.geom.height
        kinds = [gpu.U8, gpu.U16, gpu.I32, gpu.F16, gpu.F32]
        ref = [gpu.numeric_create(gpu.NumericLayer(W, H, dt)) for dt in kinds]
        got = [gpu.numeric_create(gpu.NumericLayer(W, H, dt)) for dt in kinds]
        items = _numeric_edits(m, wl, wl.edits, kinds, seed)
        _apply_numeric_plain(gpu, m, wl, items, ref)
        label_edits = [e for e in wl.edits[:20] if e.layer < len(m.layers)]
        m.clear_layers()
        m.apply_all(label_edits, wl.cameras)
        lab_ref = [l.numpy().copy() for l in m.layers]
        n = len(items) + 20
        for chunks in (1, 4):
            for L in got:
                gpu.numeric_create(L)
            m.clear_layers()
            wave = gpu.Wave(max_edits=n, max_lassos=n)
            batch = gpu.EditBatch()
            m.add_to_batch(batch, label_edits, wl.cameras)
            _add_numeric_batch(gpu, batch, m, wl, items, got)
            wave.submit(batch, tile_chunks=chunks)
            torch.cuda.synchronize()
            for dt, r, g in zip(kinds, ref, got):
                assert r.valid().any() and not r.valid().all(), (seed, dt)
                assert np.array_equal(g.mask_words(), r.mask_words()), (seed, chunks, dt)
                ut = {1: np.uint8, 2: np.uint16, 4: np.uint32}[r.numpy().dtype.itemsize]
                assert np.array_equal(g.numpy().view(ut), r.numpy().view(ut)), (seed, chunks, dt)
            for k, l in enumerate(m.layers):
                assert np.array_equal(l.numpy(), lab_ref[k]), (seed, chunks, k)
            wave.close()


def test_wave_tools_equal_plain(gpu):
    """The paper's screen-space tool in waves, beside brushes and lassos, on
    a label and a numeric layer: identical to uvl_edit_tool /
    uvl_numeric_tool launched one by one in order, with tile culling (the
    tool's square as a rectangle) and without, at two tile sizes."""
    import torch
    from paper_2501_14807_amd.model import Model
    wl = synth.scan_workload(n_brush=20, n_lasso=20, n_ops=0, W=1024, n_charts=4, nx=64, ny=32, depth=512)
    m = Model.from_workload(wl).build()
    W, H = wl.W, wl.H
    n = 64
    yy, xx = np.mgrid[0:n, 0:n]
    disk = torch.from_numpy(((((xx + 0.5) / n - 0.5) ** 2 + ((yy + 0.5) / n - 0.5) ** 2) <= 0.25)
                            .astype(np.uint8)).cuda().contiguous()
    rng = np.random.default_rng(41)
    maps = {}

    def depth(cam):
        if cam not in maps:
            d = torch.empty((m.depth_h, m.depth_w), dtype=torch.float32, device="cuda")
            gpu.render_depth(m.mesh, wl.cameras[cam], d, m.depth_ws)
            maps[cam] = d
        return maps[cam]

    ops = []          # (kind, args) in order
    for i, e in enumerate(wl.edits):
        label = 1 + i % 200
        if e.kind == "brush":
            ops.append(("brush", e, label))
        else:
            ops.append(("lasso", e, label))
            Ww, Wh = 1024.0, 1024.0
            t = (Ww, Wh, float(rng.uniform(-100, 1100)), float(rng.uniform(-100, 1100)),
                 float(rng.uniform(40, 600)), float(rng.uniform(40, 600)))
            ops.append(("tool", (e.camera, t), label + 1))
    ops.append(("tool", (wl.edits[1].camera, (512.0, 512.0, 256.0, 256.0, 512.0, 512.0)), 250))
    lab = m.layers[0]
    num = gpu.NumericLayer(W, H, gpu.F32)

    def plain():
        gpu.create_layer(lab)
        gpu.numeric_create(num)
        for kind, a, label in ops:
            if kind == "brush":
                gpu.edit_brush(m.geom, lab, a.centre, a.radius, label)
                gpu.numeric_brush(m.geom, num, a.centre, a.radius, gpu.SET, label * 0.5)
            elif kind == "lasso":
                M = wl.cameras[a.camera]
                gpu.edit_lasso(m.geom, lab, M, a.poly, depth(a.camera), m.bias, label)
                gpu.numeric_lasso(m.geom, num, M, a.poly, depth(a.camera), m.bias, gpu.ERASE)
            else:
                cam, t = a
                gpu.edit_tool(m.geom, lab, wl.cameras[cam], t, disk, depth(cam), m.bias, label)
                gpu.numeric_tool(m.geom, num, wl.cameras[cam], t, disk, depth(cam), m.bias, gpu.SET, -label)
        torch.cuda.synchronize()
        return lab.numpy().copy(), num.numpy().copy(), num.mask_words().copy()

    ref = plain()
    assert ref[0].any() and ref[2].any()
    for words in (1 << 20, 0):
        wave = gpu.Wave(max_edits=2 * len(ops), max_lassos=2 * len(ops), max_cull_words=words)
        for chunks in (1, 4):
            gpu.create_layer(lab)
            gpu.numeric_create(num)
            batch = gpu.EditBatch()
            for kind, a, label in ops:
                if kind == "brush":
                    batch.brush(m.geom, lab, a.centre, a.radius, label)
                    batch.numeric_brush(m.geom, num, a.centre, a.radius, gpu.SET, label * 0.5)
                elif kind == "lasso":
                    M = wl.cameras[a.camera]
                    batch.lasso(m.geom, lab, M, a.poly, depth(a.camera), m.bias, label)
                    batch.numeric_lasso(m.geom, num, M, a.poly, depth(a.camera), m.bias, gpu.ERASE)
                else:
                    cam, t = a
                    batch.tool(m.geom, lab, wl.cameras[cam], t, disk, depth(cam), m.bias, label)
                    batch.numeric_tool(m.geom, num, wl.cameras[cam], t, disk, depth(cam), m.bias, gpu.SET, -label)
            wave.submit(batch, tile_chunks=chunks)
            torch.cuda.synchronize()
            assert np.array_equal(lab.numpy(), ref[0]), (words, chunks)
            assert np.array_equal(num.numpy().view(np.uint32), ref[1].view(np.uint32)), (words, chunks)
            assert np.array_equal(num.mask_words(), ref[2]), (words, chunks)
            if words:
                assert wave.visited_tiles() < 2 * (W // 32) * (H // 32)   # culling skipped tiles
        wave.close()
