"""Serving on the GPU: each request's result is the same alone and in the
mix (continuous batching vs plain one-launch-per-request vs each model's
requests applied on their own), bit for bit, with and without texture
padding."""

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


def _setup(gpu):
    from paper_2501_14807_amd.model import Model
    scan = synth.scan_workload(n_brush=0, n_lasso=0, n_ops=0, W=1024, n_charts=4, nx=64, ny=32, depth=512)
    meshes = [synth.vessel(seed=s) for s in range(3)] + [scan.mesh]
    sizes = [(512, 512), (300, 200), (256, 384), (1024, 1024)]
    dtypes = [[gpu.U8, gpu.U16]] * 4
    models = [Model(m, w, h, dt, depth_w=256, depth_h=256) for m, (w, h), dt in zip(meshes, sizes, dtypes)]
    for m in models:
        m.build()
    cams, stream = synth.serve_stream(meshes, dtypes, 700, 30000.0, seed=11)
    return models, cams, stream


def _requests(stream, only=None):
    from paper_2501_14807_amd.serve import Request
    out = []
    for i, d in enumerate(stream):
        if only is not None and d["model"] != only:
            continue
        out.append(Request(i, d["t"], d["model"], d["kind"], edit=d.get("edit"), op=d.get("op"),
                           layer=d.get("layer", 0)))
    return out


def _run(gpu, models, cams, reqs, mode, pad_k=None):
    import torch
    from paper_2501_14807_amd.serve import GpuExecutor, Server
    for m in models:
        m.clear_layers()
    ex = GpuExecutor(models, cams, max_wave_edits=1024, pad_k=pad_k)
    st = Server(ex, len(models), 1 << 40).run(reqs, mode)
    torch.cuda.synchronize()
    layers = [[l.numpy().copy() for l in m.layers] for m in models]
    areas = {r.rid: r.result for r in reqs if r.kind == "area"}
    ex.wave.close()
    return st, layers, areas


def test_alone_equals_mix(gpu):
    models, cams, stream = _setup(gpu)
    st_b, lay_b, area_b = _run(gpu, models, cams, _requests(stream), "batched")
    st_p, lay_p, area_p = _run(gpu, models, cams, _requests(stream), "plain")
    assert st_b.failed == st_p.failed == 0
    assert st_b.rounds < st_b.n                  # requests were batched
    for a, b in zip(lay_b, lay_p):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    assert area_b.keys() == area_p.keys() and len(area_b) > 10
    for k in area_b:
        assert np.array_equal(area_b[k], area_p[k]), k
    # each model's requests on their own
    for mi in range(len(models)):
        st, lay, areas = _run(gpu, models, cams, _requests(stream, only=mi), "plain")
        for x, y in zip(lay[mi], lay_b[mi]):
            assert np.array_equal(x, y)
        for k, v in areas.items():
            assert np.array_equal(v, area_b[k])


def test_padded_serving_batched_equals_plain(gpu):
    """With texture padding after every edit: continuous batching (padding
    inside the waves) gives the layers of plain serving (an edit launch and
    its padding launch per request), and the areas of unpadded serving
    (padding writes uncovered texels only)."""
    models, cams, stream = _setup(gpu)
    st_b, lay_b, area_b = _run(gpu, models, cams, _requests(stream), "batched", pad_k=1)
    st_p, lay_p, area_p = _run(gpu, models, cams, _requests(stream), "plain", pad_k=1)
    _, lay_u, area_u = _run(gpu, models, cams, _requests(stream), "plain")
    assert st_b.failed == st_p.failed == 0 and st_b.rounds < st_b.n
    padded_somewhere = False
    for a, b, u in zip(lay_b, lay_p, lay_u):
        for x, y, z in zip(a, b, u):
            assert np.array_equal(x, y)
            padded_somewhere = padded_somewhere or not np.array_equal(x, z)
    assert padded_somewhere
    for k in area_b:
        assert np.array_equal(area_b[k], area_p[k]) and np.array_equal(area_b[k], area_u[k]), k
