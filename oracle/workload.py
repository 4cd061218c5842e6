"""Run a whole seeded workload through the oracle (test infrastructure only).

Applies the workload's edits in submission order to zeroed layers: brushes
directly, lassos after rendering (and caching) the depth map of their camera;
then the layer operations in order; then per-label areas of every layer.
"""

from __future__ import annotations

import numpy as np

from . import geometry_image, depth_map, brush, lasso, layer_op, area, U8


def new_layers(wl, n=None):
    n = wl.W * wl.H if n is None else n
    return [np.zeros(n, np.uint8 if dt == U8 else np.uint16) for dt in wl.layer_dtypes]


def apply_edits(wl, geom, layers, edits=None, depth_cache=None):
    """Apply edits to layers over the texels of ``geom`` (all rows or a band)."""
    pos32 = geom.pos32
    cache = {} if depth_cache is None else depth_cache
    for e in (wl.edits if edits is None else edits):
        if e.kind == "brush":
            brush(pos32, layers[e.layer], e.centre, e.radius, e.label)
        else:
            if e.camera not in cache:
                cache[e.camera] = depth_map(wl.mesh, wl.cameras[e.camera], wl.depth_w, wl.depth_h)
            lasso(pos32, layers[e.layer], wl.cameras[e.camera], e.poly, cache[e.camera],
                  wl.bias, e.label)
    return layers


def apply_ops(wl, layers, ops=None):
    for o in (wl.ops if ops is None else ops):
        layer_op(o.op, layers[o.dst], layers[o.a], layers[o.b], o.sel_a, o.sel_b, o.out_label,
                 o.lut)
    return layers


def run(wl, rows=None):
    """Full pass: geometry image, edits, layer operations, areas."""
    geom = geometry_image(wl.mesh, wl.W, wl.H, rows=rows)
    n = geom.tri_id.size
    layers = new_layers(wl, n)
    apply_edits(wl, geom, layers)
    apply_ops(wl, layers)
    areas = [area(geom, L) for L in layers]
    return geom, layers, areas
