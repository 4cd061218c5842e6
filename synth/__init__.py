"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package only draws inputs: meshes (positions, normals, texture coordinates,
triangles), edit streams (brush spheres, lasso polygons, cameras), layer-algebra
operations and request arrivals.  It holds none of the layer method's own
arithmetic (rasterisation, selection, algebra, area), so the GPU library and the
CPU oracle can both consume it without sharing code with each other.

Seeds follow one convention: ``numpy.random.default_rng(1000 * workload + k)``
with k = 0 mesh, 1 edits, 2 cameras, 3 layer operations, 4 arrivals.
"""

from .mesh import (Mesh, vessel, sphere, plane_grid, displaced_chart,
                   shelf_pack, atlas_mesh, scan_mesh, batch_model_mesh,
                   max_model_mesh, merge_meshes)
from .edits import (look_at_perspective, random_camera, star_polygon,
                    surface_points, BrushEdit, LassoEdit, LayerOp,
                    tiny_workload, scan_workload, batch_workload,
                    serve_workload, serve_stream, max_workload)

__all__ = [
    "Mesh", "vessel", "sphere", "plane_grid", "displaced_chart", "shelf_pack",
    "atlas_mesh", "scan_mesh", "batch_model_mesh", "max_model_mesh",
    "merge_meshes", "look_at_perspective", "random_camera", "star_polygon",
    "surface_points", "BrushEdit", "LassoEdit", "LayerOp", "tiny_workload",
    "scan_workload", "batch_workload", "serve_workload", "serve_stream", "max_workload",
]
