"""A model resident on the device: mesh, geometry image, layers, depth maps.

This is the plain path (one launch per edit), driving the C entry points in
the order the paper's system uses them (§4: structures live on the GPU; the
host only issues commands): build the geometry image once, then for each edit
render the depth texture if the camera changed (§4.3.1) and launch the edit;
layer operations and per-label areas run on the same stream.

Edits are duck-typed: ``kind`` ('brush' | 'lasso'), ``layer``, ``label``,
and ``centre``/``radius`` (brush) or ``camera``/``poly`` (lasso).
"""

from __future__ import annotations

from collections import OrderedDict
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import uvl


class Model:
    def __init__(self, mesh, width: int, height: int, layer_dtypes: Sequence[int], depth_w: int = 256,
                 depth_h: int = 256, bias: float = 1e-4, normals: bool = True, bary: bool = True,
                 device="cuda", depth_cache: int = 2, pool: Optional["uvl.LayerPool"] = None):
        """pool: commit the layers in a LayerPool (§4.2's texture arrays per
        (width, height, dtype)) instead of torch tensors; release() returns
        them."""
        self.mesh = uvl.DeviceMesh.from_mesh(mesh, device=device)
        self.geom = uvl.GeometryImage(width, height, normals=normals, bary=bary, device=device)
        self.pool = pool
        if pool is None:
            self.layers = [uvl.Layer(width, height, dt, device=device) for dt in layer_dtypes]
        else:
            self.layers = [pool.alloc(width, height, dt) for dt in layer_dtypes]
        self.depth_w, self.depth_h, self.bias = int(depth_w), int(depth_h), float(bias)
        self.device = device
        self.build_ws = torch.empty(uvl.lib().uvl_build_workspace_bytes(self.mesh.nt, width, height), dtype=torch.uint8,
                                    device=device)
        self.depth_ws = uvl.depth_workspace(self.mesh)
        self._depth: "OrderedDict[int, torch.Tensor]" = OrderedDict()
        self._depth_cap = max(1, depth_cache)
        self.bins = torch.empty(uvl.nbins(self.layers), dtype=torch.int64, device=device)

    def release(self):
        """Return pool-committed layers to their pool (waits for the device)."""
        if self.pool is not None:
            for l in self.layers:
                self.pool.free(l)
            self.layers = []

    @classmethod
    def from_workload(cls, wl, **kw):
        return cls(wl.mesh, wl.W, wl.H, wl.layer_dtypes, wl.depth_w, wl.depth_h, wl.bias, **kw)

    # -- set-up -----------------------------------------------------------
    def build(self):
        uvl.build_geometry_image(self.mesh, self.geom, self.build_ws)
        self.clear_layers()
        return self

    def clear_layers(self):
        for l in self.layers:
            uvl.create_layer(l)
        self._depth.clear()

    # -- depth textures -----------------------------------------------------
    def depth_for(self, cam_id: int, view_proj) -> torch.Tensor:
        d = self._depth.get(cam_id)
        if d is not None:
            self._depth.move_to_end(cam_id)
            return d
        if len(self._depth) >= self._depth_cap:
            _, d = self._depth.popitem(last=False)
        else:
            d = torch.empty((self.depth_h, self.depth_w), dtype=torch.float32, device=self.device)
        uvl.render_depth(self.mesh, view_proj, d, self.depth_ws)
        self._depth[cam_id] = d
        return d

    # -- edits ----------------------------------------------------------------
    def apply(self, e, cameras):
        layer = self.layers[e.layer]
        if e.kind == "brush":
            uvl.edit_brush(self.geom, layer, e.centre, e.radius, e.label)
        else:
            M = cameras[e.camera]
            d = self.depth_for(e.camera, M)
            uvl.edit_lasso(self.geom, layer, M, e.poly, d, self.bias, e.label)

    def apply_all(self, edits, cameras):
        for e in edits:
            self.apply(e, cameras)

    def add_to_batch(self, batch: "uvl.EditBatch", edits, cameras, render: bool = True):
        """Append edits to a wave batch.  Each lasso camera gets one depth map
        owned by the batch (alive until the batch is dropped), rendered now
        unless render=False; returns {camera: depth map} so that the caller
        can render them later with render_maps()."""
        maps = {}
        for e in edits:
            layer = self.layers[e.layer]
            if e.kind == "brush":
                batch.brush(self.geom, layer, e.centre, e.radius, e.label)
            else:
                M = cameras[e.camera]
                d = maps.get(e.camera)
                if d is None:
                    d = torch.empty((self.depth_h, self.depth_w), dtype=torch.float32, device=self.device)
                    if render:
                        uvl.render_depth(self.mesh, M, d, self.depth_ws)
                    maps[e.camera] = d
                batch.lasso(self.geom, layer, M, e.poly, d, self.bias, e.label)
        return maps

    def render_maps(self, maps, cameras):
        for cam, d in maps.items():
            uvl.render_depth(self.mesh, cameras[cam], d, self.depth_ws)

    # -- layer algebra ---------------------------------------------------------
    def apply_op(self, o):
        b = None if o.op == uvl.REMAP else self.layers[o.b]
        uvl.layer_op(o.op, self.layers[o.dst], self.layers[o.a], b, o.sel_a, o.sel_b, o.out_label, o.lut)

    # -- queries -------------------------------------------------------------
    def areas(self, sync: bool = True, layers: Optional[Sequence[int]] = None):
        ls = self.layers if layers is None else [self.layers[k] for k in layers]
        bins = None
        if layers is None:
            need = uvl.nbins(self.layers) * (2 if self.geom.wide else 1)
            if self.bins.numel() < need:
                self.bins = torch.empty(need, dtype=torch.int64, device=self.device)
            bins = self.bins
        return uvl.area_query(self.geom, ls, bins=bins, sync=sync)

    def run(self, wl):
        """One full pass of a workload: geometry image, edits, operations, areas."""
        self.build()
        self.apply_all(wl.edits, wl.cameras)
        for o in wl.ops:
            self.apply_op(o)
        return self.areas()
