"""CPU oracle for the texture-layer method (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and it
shares no code with it.  The arithmetic lives in ``uvl_oracle.c`` (plain C,
fp64 geometry, canonical fp32 predicates); this module builds it with gcc and
wraps it for numpy arrays.

Pins (tests/test_oracle_*.py): raster partition and half-open ownership on
meshes whose vertices and edges hit texel centres; affine position maps;
plane and sphere depth in closed form; spherical-cap and visible-cap areas;
total area of a surface of revolution against quadrature; crossing-number
point-in-polygon against a winding-number brute force; layer algebra against
numpy truth tables; inclusion-exclusion of areas.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "uvl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

U8, U16 = 1, 2
AND, OR, XOR, REMAP = 0, 1, 2, 3

GCC_FLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, u32, f32 = ctypes.c_int64, ctypes.c_int, ctypes.c_uint32, ctypes.c_float
        L.orc_geometry_image.argtypes = [P, P, P, P, i64, i64, i32, i32, i32, i32, P, P, P, P, P, P]
        L.orc_geometry_image.restype = i32
        L.orc_depth_map.argtypes = [P, P, i64, i64, P, i32, i32, i32, i32, P]
        L.orc_depth_map.restype = i32
        L.orc_brush.argtypes = [P, P, P, i64, P, f32, u32, P, i32]
        L.orc_brush.restype = i64
        L.orc_point_in_polygon.argtypes = [f32, f32, P, i32]
        L.orc_point_in_polygon.restype = i32
        L.orc_lasso.argtypes = [P, P, P, i64, P, P, i32, P, i32, i32, f32, u32, P, i32]
        L.orc_lasso.restype = i64
        L.orc_layer_op.argtypes = [i32, P, i32, P, i32, P, i32, i64, u32, u32, u32, P]
        L.orc_layer_op.restype = i32
        L.orc_area.argtypes = [P, P, P, i32, i64, P, i32]
        L.orc_tool_coeffs.argtypes = [P, P]
        L.orc_tool_coeffs.restype = None
        L.orc_tool.argtypes = [P, P, P, i64, P, P, P, i32, i32, P, i32, i32, f32, u32, P, i32]
        L.orc_tool.restype = i64
        L.orc_outline.argtypes = [P, i32, i32, i32, P]
        L.orc_outline.restype = i64
        L.orc_pad.argtypes = [P, P, i32, i32, i32, u32, P, i32]
        L.orc_pad.restype = i64
        L.orc_area.restype = i32
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _dtype_code(arr: np.ndarray) -> int:
    if arr.dtype == np.uint8:
        return U8
    if arr.dtype == np.uint16:
        return U16
    raise TypeError("layers are uint8 or uint16")


class GeomImage:
    """Oracle geometry image for rows [j0, j1): planes of (j1 - j0) * W values."""

    def __init__(self, W, j0, j1, tri_id, bary, pos, nrm, w, cover=None):
        self.W, self.j0, self.j1 = W, j0, j1
        self.tri_id, self.bary, self.pos, self.nrm, self.w = tri_id, bary, pos, nrm, w
        self.cover = cover

    @property
    def pos32(self):
        """Positions rounded once to fp32 (the plane the predicates read)."""
        return self.pos.astype(np.float32)


def geometry_image(mesh, W: int, H: int, rows=None, normals: bool = True,
                   cover: bool = False) -> GeomImage:
    j0, j1 = (0, H) if rows is None else rows
    n = (j1 - j0) * W
    pos = _c(mesh.pos, np.float32)
    nrm = _c(mesh.nrm, np.float32) if normals else None
    uv = _c(mesh.uv, np.float32)
    tri = _c(mesh.tri, np.int32)
    tri_id = np.empty(n, np.int32)
    bary = np.empty((2, n), np.float64)
    p = np.empty((3, n), np.float64)
    nm = np.empty((3, n), np.float64)
    w = np.empty(n, np.float64)
    cc = np.empty(n, np.int32) if cover else None
    rc = lib().orc_geometry_image(_p(pos), _p(nrm), _p(uv), _p(tri), pos.shape[0], tri.shape[0],
                                  W, H, j0, j1, _p(tri_id), _p(bary), _p(p), _p(nm), _p(w), _p(cc))
    if rc != 0:
        raise ValueError(f"orc_geometry_image failed: {rc}")
    return GeomImage(W, j0, j1, tri_id, bary, p, nm, w, cc)


def depth_map(mesh, M, Wd: int, Hd: int, rows=None) -> np.ndarray:
    r0, r1 = (0, Hd) if rows is None else rows
    pos = _c(mesh.pos, np.float32)
    tri = _c(mesh.tri, np.int32)
    Mf = _c(M, np.float32).reshape(16)
    out = np.empty((r1 - r0) * Wd, np.float32)
    rc = lib().orc_depth_map(_p(pos), _p(tri), pos.shape[0], tri.shape[0], _p(Mf), Wd, Hd, r0, r1,
                             _p(out))
    if rc != 0:
        raise ValueError(f"orc_depth_map failed: {rc}")
    return out.reshape(r1 - r0, Wd)


def brush(pos32: np.ndarray, layer: np.ndarray, centre, radius, label: int) -> int:
    """Apply one brush edit in place; pos32 is float32 [3, n]."""
    pos32 = _c(pos32, np.float32)
    c = _c(centre, np.float32)
    assert layer.flags.c_contiguous
    return int(lib().orc_brush(_p(pos32[0]), _p(pos32[1]), _p(pos32[2]), pos32.shape[1], _p(c),
                               float(np.float32(radius)), int(label), _p(layer), _dtype_code(layer)))


def point_in_polygon(x: float, y: float, poly) -> bool:
    poly = _c(poly, np.float32)
    return bool(lib().orc_point_in_polygon(float(np.float32(x)), float(np.float32(y)), _p(poly),
                                           poly.shape[0]))


def lasso(pos32: np.ndarray, layer: np.ndarray, M, poly, depth: np.ndarray, bias: float,
          label: int) -> int:
    pos32 = _c(pos32, np.float32)
    Mf = _c(M, np.float32).reshape(16)
    poly = _c(poly, np.float32)
    depth = _c(depth, np.float32)
    Hd, Wd = depth.shape
    assert layer.flags.c_contiguous
    return int(lib().orc_lasso(_p(pos32[0]), _p(pos32[1]), _p(pos32[2]), pos32.shape[1], _p(Mf),
                               _p(poly), poly.shape[0], _p(depth), Wd, Hd,
                               float(np.float32(bias)), int(label), _p(layer), _dtype_code(layer)))


def layer_op(op: int, dst: np.ndarray, a: np.ndarray, b=None, sel_a: int = 0, sel_b: int = 0,
             out_label: int = 0, lut=None) -> None:
    if b is None:
        b = a
    lutc = None if lut is None else _c(lut, np.uint16)
    if op == REMAP:
        if lutc is None or lutc.shape[0] != (256 if a.dtype == np.uint8 else 65536) or lutc[0] != 0:
            raise ValueError("REMAP needs a lut of 256 / 65536 entries with lut[0] == 0")
        if dst.dtype == np.uint8 and int(lutc.max()) > 255:
            raise ValueError("REMAP table entries must fit the destination")
    rc = lib().orc_layer_op(op, _p(dst), _dtype_code(dst), _p(a), _dtype_code(a), _p(b),
                            _dtype_code(b), dst.size, sel_a, sel_b, out_label, _p(lutc))
    if rc != 0:
        raise ValueError("orc_layer_op failed")


def area(geom: GeomImage, layer: np.ndarray, nbins=None) -> np.ndarray:
    if nbins is None:
        nbins = 256 if layer.dtype == np.uint8 else 65536
    out = np.empty(nbins, np.float64)
    rc = lib().orc_area(_p(geom.w), _p(geom.tri_id), _p(np.ascontiguousarray(layer)),
                        _dtype_code(layer), layer.size, _p(out), nbins)
    if rc != 0:
        raise ValueError("orc_area failed")
    return out


def outline(tri_id: np.ndarray, W: int, H: int, k: int = 1) -> np.ndarray:
    """Outline mask of texture padding (uint8 [H*W]): uncovered texels within
    Chebyshev distance k of a covered one (§4.3.2)."""
    tri = _c(tri_id, np.int32).reshape(-1)
    assert tri.size == W * H
    out = np.zeros(W * H, np.uint8)
    lib().orc_outline(_p(tri), int(W), int(H), int(k), _p(out))
    return out


def pad(outline_mask: np.ndarray, edited: np.ndarray, W: int, H: int, k: int, layer: np.ndarray,
        label: int) -> int:
    """Texture padding after one edit, in place: outline texels within
    Chebyshev distance k of an edited texel take `label` (§4.3.2)."""
    o = _c(outline_mask, np.uint8).reshape(-1)
    e = _c(edited, np.uint8).reshape(-1)
    assert o.size == W * H and e.size == W * H and layer.flags.c_contiguous
    return int(lib().orc_pad(_p(o), _p(e), int(W), int(H), int(k), int(label), _p(layer), _dtype_code(layer)))


def tool_coeffs(tool) -> np.ndarray:
    """fp32 (a_x, b_x, a_y, b_y) of the tool transform for tool = (Ww, Wh,
    Tpx, Tpy, Tw, Th): s = fmaf(xn, a_x, b_x), t = fmaf(yn, a_y, b_y)."""
    t = _c(tool, np.float64)
    out = np.zeros(4, np.float32)
    lib().orc_tool_coeffs(_p(t), _p(out))
    return out


def tool(pos32: np.ndarray, layer: np.ndarray, M, tool_params, shape: np.ndarray, depth: np.ndarray,
         bias: float, label: int) -> int:
    """The paper's screen-space tool (§4.3.1) in place; shape is u8 [sh, sw]."""
    pos32 = _c(pos32, np.float32)
    Mf = _c(M, np.float32).reshape(16)
    tp = _c(tool_params, np.float64)
    sh_ = _c(shape, np.uint8)
    depth = _c(depth, np.float32)
    Hd, Wd = depth.shape
    assert layer.flags.c_contiguous and tp.size == 6
    return int(lib().orc_tool(_p(pos32[0]), _p(pos32[1]), _p(pos32[2]), pos32.shape[1], _p(Mf), _p(tp), _p(sh_),
                              sh_.shape[1], sh_.shape[0], _p(depth), Wd, Hd, float(np.float32(bias)), int(label),
                              _p(layer), _dtype_code(layer)))
