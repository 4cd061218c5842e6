"""Seeded generators: determinism, recorded hashes, and the workload shapes."""

import hashlib
import json
import os

import numpy as np

import synth
from synth.mesh import grid_triangles, shelf_pack

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_tiny_workload_hashes_recorded():
    with open(os.path.join(GOLDEN, "synth_sha256.json")) as f:
        want = json.load(f)
    wl = synth.tiny_workload()
    assert _sha(wl.mesh.pos) == want["vessel_pos"]
    assert _sha(wl.mesh.uv) == want["vessel_uv"]
    assert _sha(wl.mesh.tri) == want["vessel_tri"]
    assert _sha(wl.mesh.nrm) == want["vessel_nrm"]
    assert _sha(np.stack(wl.cameras)) == want["tiny_cameras"]
    assert _sha(np.stack([e.centre for e in wl.edits if e.kind == "brush"])) == want["tiny_brush_centres"]
    assert _sha(np.concatenate([e.poly for e in wl.edits if e.kind == "lasso"])) == want["tiny_polys"]
    assert "".join("b" if e.kind == "brush" else "l" for e in wl.edits) == want["tiny_kinds"]


def test_tiny_workload_shape():
    wl = synth.tiny_workload()
    assert wl.mesh.nt == 32258 and wl.mesh.nv == 128 * 128
    assert (wl.W, wl.H, wl.depth_w, wl.depth_h) == (512, 512, 256, 256)
    kinds = [e.kind for e in wl.edits]
    assert kinds.count("brush") == 32 and kinds.count("lasso") == 32
    for e in wl.edits:
        assert 1 <= e.label <= 7
        if e.kind == "brush":
            assert 0.05 <= e.radius <= 0.3
        else:
            assert e.poly.shape == (8, 2)
    assert len(wl.cameras) == 32


def test_triangle_counts_of_the_workloads():
    # scan-scale: 64 charts of 256 x 128 vertices; largest: 256 of 128 x 128
    assert 64 * grid_triangles(256, 128).shape[0] == 4145280
    assert 256 * grid_triangles(128, 128).shape[0] == 8258048


def test_grid_triangles_ccw_in_uv():
    m = synth.plane_grid(6, 4)
    uv = m.uv.astype(np.float64)
    t = m.tri
    e = ((uv[t[:, 1], 0] - uv[t[:, 0], 0]) * (uv[t[:, 2], 1] - uv[t[:, 0], 1])
         - (uv[t[:, 1], 1] - uv[t[:, 0], 1]) * (uv[t[:, 2], 0] - uv[t[:, 0], 0]))
    assert (e > 0).all()


def test_shelf_pack_gutters_and_bounds():
    rects = [(50, 20)] * 7 + [(30, 40)] * 3
    pl = shelf_pack(rects, 200, 200, 2)
    boxes = [(x, y, x + w, y + h) for (x, y), (w, h) in zip(pl, rects)]
    for a in range(len(boxes)):
        x0, y0, x1, y1 = boxes[a]
        assert x0 >= 2 and y0 >= 2 and x1 <= 198 and y1 <= 198
        for b in range(a):
            X0, Y0, X1, Y1 = boxes[b]
            # at least a 2-texel gutter between any two rectangles
            assert x1 + 2 <= X0 or X1 + 2 <= x0 or y1 + 2 <= Y0 or Y1 + 2 <= y0
    assert shelf_pack([(300, 10)], 200, 200, 2) is None


def test_small_scan_workload_structure():
    wl = synth.scan_workload(n_brush=20, n_lasso=24, n_ops=16, W=1024, n_charts=4, nx=32, ny=16,
                             depth=256)
    assert wl.mesh.nt == 4 * 31 * 15 * 2
    assert len(wl.layer_dtypes) == 9 and wl.layer_dtypes[8] == 2
    assert len(wl.cameras) == 3                  # one per 8 lassos
    uv = wl.mesh.uv
    assert uv.min() >= 2 / 1024 and uv.max() <= 1 - 2 / 1024
    for o in wl.ops:
        if o.op == 3:
            assert o.lut[0] == 0
    wl2 = synth.scan_workload(n_brush=20, n_lasso=24, n_ops=16, W=1024, n_charts=4, nx=32, ny=16,
                              depth=256)
    assert np.array_equal(wl.mesh.pos, wl2.mesh.pos)
    assert all(np.array_equal(a.poly, b.poly) for a, b in zip(wl.edits, wl2.edits)
               if a.kind == "lasso")
