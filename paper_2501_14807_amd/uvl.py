"""Python binding of libuvl.so (argument marshalling only).

Every step of the layer method runs in the HIP kernels behind the C ABI
declared in include/uvl.h; this module passes torch device pointers, host
parameter arrays and the current HIP stream through ctypes, and turns status
codes into exceptions.  PyTorch provides device memory and streams only.
There is no CPU fallback: if libuvl.so is missing the import fails.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libuvl.so")

U8, U16, I32, F16, F32 = 1, 2, 3, 4, 5
AND, OR, XOR, REMAP = 0, 1, 2, 3
SET, ERASE = 0, 1

STATUS = {0: "UVL_OK", -1: "UVL_E_INVAL", -2: "UVL_E_SHAPE", -3: "UVL_E_DTYPE",
          -4: "UVL_E_NOMEM", -5: "UVL_E_DEVICE", -6: "UVL_E_UNSUPPORTED"}


class UvlError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)} ({_lib().uvl_status_str(code).decode()})")


class CMesh(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("nrm", ctypes.c_void_p), ("uv", ctypes.c_void_p),
                ("tri", ctypes.c_void_p), ("nv", ctypes.c_int64), ("nt", ctypes.c_int64)]


class CGeom(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("tri_id", ctypes.c_void_p),
                ("pos_x", ctypes.c_void_p), ("pos_y", ctypes.c_void_p), ("pos_z", ctypes.c_void_p),
                ("nrm_x", ctypes.c_void_p), ("nrm_y", ctypes.c_void_p), ("nrm_z", ctypes.c_void_p),
                ("bary1", ctypes.c_void_p), ("bary2", ctypes.c_void_p),
                ("area_w", ctypes.c_void_p),
                ("area_scale", ctypes.c_double), ("area_abs_err", ctypes.c_double),
                ("tile_box", ctypes.c_void_p), ("area_w_hi", ctypes.c_void_p), ("area_blk", ctypes.c_void_p)]

TILE_SIDE = 32
TILE_BLOCK = 8
AREA_BLK_ROWS, AREA_BLK_COLS = 4, 8


class CLayer(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("dtype", ctypes.c_int32)]


class CNumeric(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("dtype", ctypes.c_int32)]


# uvl_numstat
NUMSTAT = np.dtype([("count", np.uint64), ("area_w", np.uint64), ("wsum", np.float64), ("vmin", np.float64),
                    ("vmax", np.float64), ("area_w_hi", np.uint64)])
E_RANGE = -7

_L = None

# exported names and ctypes signatures; the CPU tests check that include/uvl.h
# declares exactly these
_P, _I32, _I64, _U32, _F32, _SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                   ctypes.c_float, ctypes.c_size_t)
_F64 = ctypes.c_double
SIGNATURES = {
    "uvl_status_str": ([_I32], ctypes.c_char_p),
    "uvl_device_check": ([], _I32),
    "uvl_build_workspace_bytes": ([_I64, _I32, _I32], _SZ),
    "uvl_geom_bytes": ([_I32, _I32, _U32], _SZ),
    "uvl_build_geometry_image": ([_P, _P, _P, _SZ, _P], _I32),
    "uvl_create_layer": ([_P, _P], _I32),
    "uvl_depth_workspace_bytes": ([_I64], _SZ),
    "uvl_render_depth": ([_P, _P, _P, _I32, _I32, _P, _SZ, _P], _I32),
    "uvl_render_depth_noalloc": ([_P, _P, _P, _I32, _I32, _P], _I32),
    "uvl_edit_brush": ([_P, _P, _P, _F32, _U32, _P], _I32),
    "uvl_edit_lasso": ([_P, _P, _P, _P, _I32, _P, _I32, _I32, _F32, _U32, _P], _I32),
    "uvl_layer_op": ([_I32, _P, _P, _P, _U32, _U32, _U32, _P, _P], _I32),
    "uvl_area_bin_count": ([_P, _P, _I32], _I64),
    "uvl_area_query": ([_P, _P, _I32, _P, _P, _P], _I32),
    "uvl_wave_workspace_bytes": ([_I32, _I32, _I64], _SZ),
    "uvl_wave_create": ([_I32, _I32, _I64, _P, _SZ, _P], _I32),
    "uvl_wave_submit": ([_P, _P, _I32, _I32, _P], _I32),
    "uvl_wave_submit_padded": ([_P, _P, _I32, _I32, _P, _I32, _P], _I32),
    "uvl_wave_tune": ([_P, _P, _I32, _P], _I32),
    "uvl_wave_tuned_chunks": ([_P, _I64], _I32),
    "uvl_wave_visited_tiles": ([_P, _P, _P], _I32),
    "uvl_wave_destroy": ([_P], _I32),
    "uvl_edit_tool": ([_P, _P, _P, _P, _P, _I32, _I32, _P, _I32, _I32, _F32, _U32, _P], _I32),
    "uvl_outline_workspace_bytes": ([_I32, _I32], _SZ),
    "uvl_build_outline": ([_P, _I32, _P, _I64, _P, _P, _SZ, _P], _I32),
    "uvl_pad_brush": ([_P, _P, _P, _I64, _I32, _P, _F32, _U32, _P], _I32),
    "uvl_pad_lasso": ([_P, _P, _P, _I64, _I32, _P, _P, _I32, _P, _I32, _I32, _F32, _U32, _P], _I32),
    "uvl_numeric_create": ([_P, _P], _I32),
    "uvl_numeric_brush": ([_P, _P, _P, _F32, _I32, _F64, _P], _I32),
    "uvl_numeric_lasso": ([_P, _P, _P, _P, _I32, _P, _I32, _I32, _F32, _I32, _F64, _P], _I32),
    "uvl_numeric_tool": ([_P, _P, _P, _P, _P, _I32, _I32, _P, _I32, _I32, _F32, _I32, _F64, _P], _I32),
    "uvl_numeric_op": ([_I32, _P, _P, _P, _P], _I32),
    "uvl_numeric_select": ([_P, _F64, _F64, _P, _U32, _P], _I32),
    "uvl_numeric_pad_brush": ([_P, _P, _P, _I64, _I32, _P, _F32, _I32, _F64, _P], _I32),
    "uvl_numeric_pad_lasso": ([_P, _P, _P, _I64, _I32, _P, _P, _I32, _P, _I32, _I32, _F32, _I32, _F64, _P], _I32),
    "uvl_numeric_stats": ([_P, _P, _P, _P, _P, _P], _I32),
    "uvl_pool_create": ([_I32, _P], _I32),
    "uvl_pool_alloc": ([_P, _I32, _I32, _I32, _P, _P], _I32),
    "uvl_pool_free": ([_P, _P], _I32),
    "uvl_pool_array": ([_P, _I32, _I32, _I32, _P, _P, _P], _I32),
    "uvl_pool_stats": ([_P, _P, _P, _P], _I32),
    "uvl_pool_destroy": ([_P], _I32),
}

EDIT_BRUSH, EDIT_LASSO, EDIT_TOOL = 0, 1, 2


class CWaveOutline(ctypes.Structure):
    _fields_ = [("geom", ctypes.c_void_p), ("outline", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("k", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class CEdit(ctypes.Structure):
    _fields_ = [("geom", ctypes.c_void_p), ("layer", ctypes.c_void_p), ("kind", ctypes.c_int32),
                ("label", ctypes.c_uint32), ("center", ctypes.c_float * 3), ("radius", ctypes.c_float),
                ("view_proj", ctypes.c_void_p), ("poly_xy", ctypes.c_void_p), ("npoly", ctypes.c_int32),
                ("dw", ctypes.c_int32), ("dh", ctypes.c_int32), ("bias", ctypes.c_float),
                ("depth", ctypes.c_void_p), ("numeric", ctypes.c_void_p), ("mode", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("value", ctypes.c_double), ("tool", ctypes.c_void_p),
                ("shape", ctypes.c_void_p), ("sw", ctypes.c_int32), ("sh", ctypes.c_int32),
                ("bins", ctypes.c_void_p)]


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2501_14807_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        # the HIP runtime libuvl links, for host copies of pool layers
        L.hipMemcpy.argtypes = [_P, _P, _SZ, ctypes.c_int]
        L.hipMemcpy.restype = ctypes.c_int
        _L = L
    return _L


def lib():
    """The loaded libuvl.so (ctypes.CDLL)."""
    return _lib()


def _check(code: int, where: str):
    if code != 0:
        raise UvlError(code, where)


def _stream(stream=None):
    """The HIP stream handle: `stream`, or torch's current stream (read
    through torch's C binding: torch.cuda.current_stream() costs ~10 us)."""
    if stream is None:
        return ctypes.c_void_p(torch._C._cuda_getCurrentRawStream(torch._C._cuda_getDevice()))
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _f32(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} floats, got {a.size}")
    return a


def _pad(n: int, q: int = 64) -> int:
    return (n + q - 1) // q * q


def device_check():
    _check(_lib().uvl_device_check(), "uvl_device_check")


# ---------------------------------------------------------------------------
# device objects


class DeviceMesh:
    """A triangle mesh resident in device memory (fp32 pos/nrm/uv, int32 tri)."""

    def __init__(self, pos, uv, tri, nrm=None, device="cuda"):
        def dev(a, dt):
            if isinstance(a, torch.Tensor):
                return a.to(device=device, dtype=dt).contiguous()
            return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt).contiguous()
        self.pos = dev(pos, torch.float32).reshape(-1, 3)
        self.uv = dev(uv, torch.float32).reshape(-1, 2)
        self.tri = dev(tri, torch.int32).reshape(-1, 3)
        self.nrm = None if nrm is None else dev(nrm, torch.float32).reshape(-1, 3)
        self.c = CMesh(self.pos.data_ptr(), None if self.nrm is None else self.nrm.data_ptr(),
                       self.uv.data_ptr(), self.tri.data_ptr(), self.pos.shape[0], self.tri.shape[0])

    @classmethod
    def from_mesh(cls, m, device="cuda", normals=True):
        return cls(m.pos, m.uv, m.tri, m.nrm if normals else None, device)

    @property
    def nt(self) -> int:
        return int(self.tri.shape[0])


class GeometryImage:
    """Per-texel triangle id, position, normal, barycentrics and area weight.

    Planes are rows of padded tensors so that each starts 16-byte aligned.
    """

    def __init__(self, width: int, height: int, normals: bool = True, bary: bool = True,
                 device="cuda", tile_box: bool = True, wide: bool = False, area_blk: bool = True):
        self.width, self.height = int(width), int(height)
        n = self.width * self.height
        self.n = n
        p = _pad(n)
        self.tri_id = torch.empty(p, dtype=torch.int32, device=device)
        self.pos = torch.empty((3, p), dtype=torch.float32, device=device)
        self.nrm = torch.empty((3, p), dtype=torch.float32, device=device) if normals else None
        self.bary = torch.empty((2, p), dtype=torch.float32, device=device) if bary else None
        self.area_w = torch.empty(p, dtype=torch.int32, device=device)   # uint32 bits
        self.area_w_hi = None
        self._device = device
        self.tiles_x = (self.width + TILE_SIDE - 1) // TILE_SIDE
        self.tiles_y = (self.height + TILE_SIDE - 1) // TILE_SIDE
        self.ntiles = self.tiles_x * self.tiles_y
        # tile bounds, then the bounds of the blocks of TILE_BLOCK x TILE_BLOCK tiles
        self.nblocks = (-(-self.tiles_x // TILE_BLOCK)) * (-(-self.tiles_y // TILE_BLOCK))
        self.tile_box = (torch.empty((self.ntiles + self.nblocks, 6), dtype=torch.float32, device=device)
                         if tile_box else None)
        self.c = CGeom()
        self.c.width, self.c.height = self.width, self.height
        self.c.tri_id = self.tri_id.data_ptr()
        self.c.pos_x, self.c.pos_y, self.c.pos_z = (self.pos[k].data_ptr() for k in range(3))
        if normals:
            self.c.nrm_x, self.c.nrm_y, self.c.nrm_z = (self.nrm[k].data_ptr() for k in range(3))
        if bary:
            self.c.bary1, self.c.bary2 = self.bary[0].data_ptr(), self.bary[1].data_ptr()
        self.c.area_w = self.area_w.data_ptr()
        self.c.tile_box = None if self.tile_box is None else self.tile_box.data_ptr()
        # per-block sums of the one-word texel areas (4 rows x 8 columns)
        self.area_blk = None
        if area_blk and not wide:
            nb = (-(-self.width // AREA_BLK_COLS)) * (-(-self.height // AREA_BLK_ROWS))
            self.area_blk = torch.empty(nb, dtype=torch.int64, device=device)
            self.c.area_blk = self.area_blk.data_ptr()
        if wide:
            self.make_wide()
        self.c.area_scale = 0.0
        self.c.area_abs_err = 0.0
        self.addr = ctypes.addressof(self.c)     # the uvl_geom the library reads

    def make_wide(self):
        """Give the image a plane of high words: two-word texel areas (for
        meshes whose texel areas span more than 2^11)."""
        if self.area_w_hi is None:
            self.area_w_hi = torch.empty(self.area_w.numel(), dtype=torch.int32, device=self._device)
            self.c.area_w_hi = self.area_w_hi.data_ptr()
            self.area_blk = None                  # block sums are for one-word areas only
            self.c.area_blk = None

    @property
    def wide(self) -> bool:
        return self.area_w_hi is not None

    @property
    def area_scale(self) -> float:
        return float(self.c.area_scale)

    @property
    def area_abs_err(self) -> float:
        return float(self.c.area_abs_err)

    def nbytes(self) -> int:
        ts = [self.tri_id, self.pos, self.nrm, self.bary, self.area_w, self.tile_box, self.area_w_hi, self.area_blk]
        return sum(t.numel() * t.element_size() for t in ts if t is not None)

    # host copies of the first n elements of each plane
    def host(self):
        n = self.n
        out = {"tri_id": self.tri_id[:n].cpu().numpy(), "pos": self.pos[:, :n].cpu().numpy(),
               "area_w": self.area_w[:n].cpu().numpy().view(np.uint32)}
        if self.area_w_hi is not None:
            out["area_w_hi"] = self.area_w_hi[:n].cpu().numpy().view(np.uint32)
        if self.area_blk is not None:
            out["area_blk"] = self.area_blk.cpu().numpy().view(np.uint64)
        if self.nrm is not None:
            out["nrm"] = self.nrm[:, :n].cpu().numpy()
        if self.bary is not None:
            out["bary"] = self.bary[:, :n].cpu().numpy()
        return out


class Layer:
    """A layer's data texture: width*height uint8 or uint16 labels on the device."""

    def __init__(self, width: int, height: int, dtype: int = U8, device="cuda", data=None):
        self.width, self.height, self.dtype = int(width), int(height), int(dtype)
        n = self.width * self.height
        if data is None:
            tdt = torch.uint8 if dtype == U8 else torch.uint16
            data = torch.empty(_pad(n), dtype=tdt, device=device)
        self.data = data
        self.c = CLayer(data.data_ptr(), self.width, self.height, self.dtype)
        self.addr = ctypes.addressof(self.c)

    @property
    def n(self) -> int:
        return self.width * self.height

    def numpy(self) -> np.ndarray:
        return self.data[:self.n].cpu().numpy()

    def copy_from(self, arr: np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(arr))
        self.data[:self.n].copy_(t.to(self.data.dtype))


_TORCH_DTYPE = {U8: torch.uint8, U16: torch.uint16, I32: torch.int32, F16: torch.float16, F32: torch.float32}
_NP_DTYPE = {U8: np.uint8, U16: np.uint16, I32: np.int32, F16: np.float16, F32: np.float32}


class NumericLayer:
    """A numeric layer: width*height values of dtype (U8, U16, I32, F16,
    F32) and a mask of one validity bit per texel (bit t % 32 of word t / 32)."""

    def __init__(self, width: int, height: int, dtype: int = F32, device="cuda"):
        self.width, self.height, self.dtype = int(width), int(height), int(dtype)
        if self.dtype not in _TORCH_DTYPE:
            raise ValueError(f"dtype {dtype}")
        n = self.width * self.height
        self.data = torch.empty(_pad(n), dtype=_TORCH_DTYPE[self.dtype], device=device)
        self.mask = torch.empty(_pad((n + 31) // 32), dtype=torch.int32, device=device)
        self.c = CNumeric(self.data.data_ptr(), self.mask.data_ptr(), self.width, self.height, self.dtype)

    @property
    def n(self) -> int:
        return self.width * self.height

    def numpy(self) -> np.ndarray:
        return self.data[:self.n].cpu().numpy()

    def mask_words(self) -> np.ndarray:
        return self.mask[:(self.n + 31) // 32].cpu().numpy().view(np.uint32)

    def valid(self) -> np.ndarray:
        w = self.mask_words().astype(np.uint64)
        bits = (w[:, None] >> np.arange(32, dtype=np.uint64)) & np.uint64(1)
        return bits.reshape(-1)[:self.n].astype(bool)

    def copy_from(self, data: np.ndarray, valid: np.ndarray):
        """Upload values and validity flags (one per texel)."""
        self.data[:self.n].copy_(torch.from_numpy(np.ascontiguousarray(data, _NP_DTYPE[self.dtype])))
        v = np.zeros(((self.n + 31) // 32) * 32, np.uint64)
        v[:self.n] = np.asarray(valid, bool)
        words = (v.reshape(-1, 32) << np.arange(32, dtype=np.uint64)).sum(axis=1).astype(np.uint32)
        self.mask[:words.size].copy_(torch.from_numpy(words.view(np.int32)))


# ---------------------------------------------------------------------------
# the C entry points, one function each


def build_geometry_image(mesh: DeviceMesh, geom: GeometryImage, workspace: Optional[torch.Tensor] = None,
                         stream=None) -> GeometryImage:
    L = _lib()
    need = L.uvl_build_workspace_bytes(mesh.nt, geom.width, geom.height)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=mesh.pos.device)
    st = L.uvl_build_geometry_image(ctypes.byref(mesh.c), ctypes.byref(geom.c), _ptr(workspace),
                                    workspace.numel(), _stream(stream))
    if st == E_RANGE and not geom.wide:
        # texel areas too spread out for one word per texel: two words
        geom.make_wide()
        st = L.uvl_build_geometry_image(ctypes.byref(mesh.c), ctypes.byref(geom.c), _ptr(workspace),
                                        workspace.numel(), _stream(stream))
    _check(st, "uvl_build_geometry_image")
    return geom


def create_layer(layer: Layer, stream=None) -> Layer:
    _check(_lib().uvl_create_layer(ctypes.byref(layer.c), _stream(stream)), "uvl_create_layer")
    return layer


def depth_workspace(mesh: DeviceMesh) -> torch.Tensor:
    return torch.empty(_lib().uvl_depth_workspace_bytes(mesh.nt), dtype=torch.uint8, device=mesh.pos.device)


def render_depth(mesh: DeviceMesh, view_proj, depth: torch.Tensor, workspace: Optional[torch.Tensor] = None,
                 stream=None) -> torch.Tensor:
    M = _f32(view_proj, 16)
    dh, dw = depth.shape
    if workspace is None:
        workspace = depth_workspace(mesh)
    _check(_lib().uvl_render_depth(ctypes.byref(mesh.c), M.ctypes.data_as(ctypes.c_void_p), _ptr(depth),
                                   dw, dh, _ptr(workspace), workspace.numel(), _stream(stream)),
           "uvl_render_depth")
    return depth


def render_depth_noalloc(mesh: DeviceMesh, view_proj, depth: torch.Tensor, stream=None) -> torch.Tensor:
    """uvl_render_depth on the library's static scratch (no workspace, no
    allocation); calls that overlap on one device race."""
    M = _f32(view_proj, 16)
    dh, dw = depth.shape
    _check(_lib().uvl_render_depth_noalloc(ctypes.byref(mesh.c), M.ctypes.data_as(ctypes.c_void_p), _ptr(depth),
                                           dw, dh, _stream(stream)), "uvl_render_depth_noalloc")
    return depth


def edit_brush(geom: GeometryImage, layer: Layer, center, radius: float, label: int, stream=None):
    c = _f32(center, 3)
    _check(_lib().uvl_edit_brush(ctypes.byref(geom.c), ctypes.byref(layer.c), c.ctypes.data_as(ctypes.c_void_p),
                                 float(np.float32(radius)), int(label), _stream(stream)), "uvl_edit_brush")


def edit_lasso(geom: GeometryImage, layer: Layer, view_proj, poly, depth: torch.Tensor, bias: float, label: int,
               stream=None):
    M = _f32(view_proj, 16)
    P = _f32(poly).reshape(-1)
    dh, dw = depth.shape
    _check(_lib().uvl_edit_lasso(ctypes.byref(geom.c), ctypes.byref(layer.c), M.ctypes.data_as(ctypes.c_void_p),
                                 P.ctypes.data_as(ctypes.c_void_p), P.size // 2, _ptr(depth), dw, dh,
                                 float(np.float32(bias)), int(label), _stream(stream)), "uvl_edit_lasso")


def edit_tool(geom: GeometryImage, layer: Layer, view_proj, tool, shape: torch.Tensor, depth: torch.Tensor,
              bias: float, label: int, stream=None):
    """The paper's screen-space tool: tool = (Ww, Wh, Tpx, Tpy, Tw, Th),
    shape a device uint8 [sh, sw] tensor."""
    M = _f32(view_proj, 16)
    tp = np.ascontiguousarray(np.asarray(tool, dtype=np.float64))
    if tp.size != 6:
        raise ValueError("tool needs 6 numbers (Ww, Wh, Tpx, Tpy, Tw, Th)")
    if shape.dtype != torch.uint8 or shape.dim() != 2 or not shape.is_contiguous():
        raise ValueError("shape must be a contiguous uint8 [sh, sw] tensor")
    sh, sw = shape.shape
    dh, dw = depth.shape
    _check(_lib().uvl_edit_tool(ctypes.byref(geom.c), ctypes.byref(layer.c), M.ctypes.data_as(ctypes.c_void_p),
                                tp.ctypes.data_as(ctypes.c_void_p), _ptr(shape), sw, sh, _ptr(depth), dw, dh,
                                float(np.float32(bias)), int(label), _stream(stream)), "uvl_edit_tool")


class PoolLayer:
    """A layer committed by a LayerPool: the same descriptor as Layer (so
    every call that takes a Layer takes it), on pool memory instead of a
    torch tensor.  Host copies go through the HIP runtime."""

    def __init__(self, pool: "LayerPool", ptr: int, slot: int, width: int, height: int, dtype: int):
        self.pool, self.ptr, self.slot = pool, ptr, slot
        self.width, self.height, self.dtype = int(width), int(height), int(dtype)
        self.c = CLayer(ptr, self.width, self.height, self.dtype)
        self.addr = ctypes.addressof(self.c)

    @property
    def n(self) -> int:
        return self.width * self.height

    def numpy(self) -> np.ndarray:
        out = np.empty(self.n, _NP_DTYPE[self.dtype])
        torch.cuda.synchronize()
        _check_hip(_lib().hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(self.ptr), out.nbytes,
                                    _HIP_D2H), "hipMemcpy")
        return out

    def copy_from(self, arr: np.ndarray):
        a = np.ascontiguousarray(arr, _NP_DTYPE[self.dtype]).reshape(-1)
        if a.size != self.n:
            raise ValueError("size")
        torch.cuda.synchronize()
        _check_hip(_lib().hipMemcpy(ctypes.c_void_p(self.ptr), a.ctypes.data_as(ctypes.c_void_p), a.nbytes,
                                    _HIP_H2D), "hipMemcpy")


_HIP_H2D, _HIP_D2H = 1, 2


def _check_hip(code: int, where: str):
    if code != 0:
        raise RuntimeError(f"{where}: hipError {code}")


class LayerPool:
    """Layers committed on demand into per-(width, height, dtype) reserved
    address ranges (uvl_pool_*): the layers of one key form an array at
    base + slot * stride."""

    def __init__(self, slots_per_key: int = 64):
        h = ctypes.c_void_p()
        _check(_lib().uvl_pool_create(int(slots_per_key), ctypes.byref(h)), "uvl_pool_create")
        self.h = h

    def alloc(self, width: int, height: int, dtype: int = U8) -> PoolLayer:
        ptr, slot = ctypes.c_void_p(), ctypes.c_int32()
        _check(_lib().uvl_pool_alloc(self.h, int(width), int(height), int(dtype), ctypes.byref(ptr),
                                     ctypes.byref(slot)), "uvl_pool_alloc")
        return PoolLayer(self, ptr.value, slot.value, width, height, dtype)

    def free(self, layer: PoolLayer):
        _check(_lib().uvl_pool_free(self.h, ctypes.c_void_p(layer.ptr)), "uvl_pool_free")

    def array(self, width: int, height: int, dtype: int):
        """(base address, slot stride in bytes, slots) of a key."""
        base, stride, slots = ctypes.c_void_p(), ctypes.c_size_t(), ctypes.c_int32()
        _check(_lib().uvl_pool_array(self.h, int(width), int(height), int(dtype), ctypes.byref(base),
                                     ctypes.byref(stride), ctypes.byref(slots)), "uvl_pool_array")
        return base.value, stride.value, slots.value

    def stats(self):
        """(reserved bytes, committed bytes, keys)."""
        r, c, k = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_int32()
        _check(_lib().uvl_pool_stats(self.h, ctypes.byref(r), ctypes.byref(c), ctypes.byref(k)), "uvl_pool_stats")
        return r.value, c.value, k.value

    def close(self):
        if self.h:
            torch.cuda.synchronize()
            _check(_lib().uvl_pool_destroy(self.h), "uvl_pool_destroy")
            self.h = None


def numeric_create(layer: NumericLayer, stream=None) -> NumericLayer:
    _check(_lib().uvl_numeric_create(ctypes.byref(layer.c), _stream(stream)), "uvl_numeric_create")
    return layer


NUM_AND, NUM_OR, NUM_XOR, NUM_MIN, NUM_MAX, NUM_ADD = 0, 1, 2, 3, 4, 5


def numeric_op(op: int, dst: NumericLayer, a: NumericLayer, b: NumericLayer, stream=None) -> NumericLayer:
    """dst = a op b texel by texel (uvl_numeric_op); dst may be a or b."""
    _check(_lib().uvl_numeric_op(int(op), ctypes.byref(dst.c), ctypes.byref(a.c), ctypes.byref(b.c),
                                 _stream(stream)), "uvl_numeric_op")
    return dst


def numeric_brush(geom: GeometryImage, layer: NumericLayer, center, radius: float, mode: int, value: float = 0.0,
                  stream=None):
    c = _f32(center, 3)
    _check(_lib().uvl_numeric_brush(ctypes.byref(geom.c), ctypes.byref(layer.c), c.ctypes.data_as(ctypes.c_void_p),
                                    float(np.float32(radius)), int(mode), float(value), _stream(stream)),
           "uvl_numeric_brush")


def numeric_lasso(geom: GeometryImage, layer: NumericLayer, view_proj, poly, depth: torch.Tensor, bias: float,
                  mode: int, value: float = 0.0, stream=None):
    M = _f32(view_proj, 16)
    P = _f32(poly).reshape(-1)
    dh, dw = depth.shape
    _check(_lib().uvl_numeric_lasso(ctypes.byref(geom.c), ctypes.byref(layer.c), M.ctypes.data_as(ctypes.c_void_p),
                                    P.ctypes.data_as(ctypes.c_void_p), P.size // 2, _ptr(depth), dw, dh,
                                    float(np.float32(bias)), int(mode), float(value), _stream(stream)),
           "uvl_numeric_lasso")


def numeric_tool(geom: GeometryImage, layer: NumericLayer, view_proj, tool, shape: torch.Tensor, depth: torch.Tensor,
                 bias: float, mode: int, value: float = 0.0, stream=None):
    M = _f32(view_proj, 16)
    tp = np.ascontiguousarray(np.asarray(tool, dtype=np.float64))
    if tp.size != 6 or shape.dtype != torch.uint8 or shape.dim() != 2 or not shape.is_contiguous():
        raise ValueError("tool needs 6 numbers and a contiguous uint8 [sh, sw] shape")
    sh, sw = shape.shape
    dh, dw = depth.shape
    _check(_lib().uvl_numeric_tool(ctypes.byref(geom.c), ctypes.byref(layer.c), M.ctypes.data_as(ctypes.c_void_p),
                                   tp.ctypes.data_as(ctypes.c_void_p), _ptr(shape), sw, sh, _ptr(depth), dw, dh,
                                   float(np.float32(bias)), int(mode), float(value), _stream(stream)),
           "uvl_numeric_tool")


def numeric_select(src: NumericLayer, lo: float, hi: float, dst: Layer, label: int, stream=None):
    _check(_lib().uvl_numeric_select(ctypes.byref(src.c), float(lo), float(hi), ctypes.byref(dst.c), int(label),
                                     _stream(stream)), "uvl_numeric_select")


def numeric_stats(geom: GeometryImage, layer: NumericLayer, region: Optional[Layer] = None,
                  bins: Optional[torch.Tensor] = None, host: bool = True, stream=None):
    """Zonal statistics: a NUMSTAT record per value of `region` (one when
    None).  host=True returns them as a numpy array (synchronous); host=False
    leaves them in `bins` (a device tensor of >= 48 bytes per group) and
    returns that tensor."""
    groups = 1 if region is None else (256 if region.dtype == U8 else 65536)
    assert NUMSTAT.itemsize == 48
    if bins is None:
        bins = torch.empty(groups * NUMSTAT.itemsize, dtype=torch.uint8, device=layer.data.device)
    if bins.numel() * bins.element_size() < groups * NUMSTAT.itemsize:
        raise ValueError("bins too small")
    out = np.empty(groups, NUMSTAT) if host else None
    _check(_lib().uvl_numeric_stats(ctypes.byref(geom.c), ctypes.byref(layer.c),
                                    None if region is None else ctypes.byref(region.c), _ptr(bins),
                                    None if out is None else out.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
           "uvl_numeric_stats")
    return out if host else bins


def disk_shape(n: int = 256, device="cuda") -> torch.Tensor:
    """The default tool shape: a disk inscribed in an n x n texture (texel
    centres within radius 1/2 of the centre)."""
    c = (torch.arange(n, dtype=torch.float64) + 0.5) / n - 0.5
    return ((c[:, None] ** 2 + c[None, :] ** 2) <= 0.25).to(torch.uint8).to(device).contiguous()


class Outline:
    """Outline texels of a geometry image for texture padding (§4.3.2)."""

    def __init__(self, geom: GeometryImage, k: int = 1, stream=None):
        L = _lib()
        need = L.uvl_outline_workspace_bytes(geom.width, geom.height)
        if need == 0:
            raise ValueError("bad atlas size")
        ws = torch.empty(need, dtype=torch.uint8, device=geom.tri_id.device)
        cap = max(1, geom.n // 8)
        while True:
            idx = torch.empty(cap, dtype=torch.int32, device=geom.tri_id.device)
            n = ctypes.c_int64()
            rc = L.uvl_build_outline(ctypes.byref(geom.c), int(k), _ptr(idx), cap, ctypes.byref(n), _ptr(ws), need,
                                     _stream(stream))
            if rc == -4 and n.value > cap:          # UVL_E_NOMEM: room for all of them, then again
                cap = int(n.value)
                continue
            _check(rc, "uvl_build_outline")
            break
        self.k = int(k)
        self.n = int(n.value)
        self.idx = idx[:max(self.n, 1)]

    def numpy(self) -> np.ndarray:
        return self.idx[:self.n].cpu().numpy()


def pad_brush(geom: GeometryImage, layer: Layer, outline: Outline, center, radius: float, label: int, stream=None):
    c = _f32(center, 3)
    _check(_lib().uvl_pad_brush(ctypes.byref(geom.c), ctypes.byref(layer.c), _ptr(outline.idx), outline.n, outline.k,
                                c.ctypes.data_as(ctypes.c_void_p), float(np.float32(radius)), int(label),
                                _stream(stream)), "uvl_pad_brush")


def pad_lasso(geom: GeometryImage, layer: Layer, outline: Outline, view_proj, poly, depth: torch.Tensor, bias: float,
              label: int, stream=None):
    M = _f32(view_proj, 16)
    P = _f32(poly).reshape(-1)
    dh, dw = depth.shape
    _check(_lib().uvl_pad_lasso(ctypes.byref(geom.c), ctypes.byref(layer.c), _ptr(outline.idx), outline.n, outline.k,
                                M.ctypes.data_as(ctypes.c_void_p), P.ctypes.data_as(ctypes.c_void_p), P.size // 2,
                                _ptr(depth), dw, dh, float(np.float32(bias)), int(label), _stream(stream)),
           "uvl_pad_lasso")


def numeric_pad_brush(geom: GeometryImage, layer: NumericLayer, outline: Outline, center, radius: float, mode: int,
                      value: float = 0.0, stream=None):
    c = _f32(center, 3)
    _check(_lib().uvl_numeric_pad_brush(ctypes.byref(geom.c), ctypes.byref(layer.c), _ptr(outline.idx), outline.n,
                                        outline.k, c.ctypes.data_as(ctypes.c_void_p), float(np.float32(radius)),
                                        int(mode), float(value), _stream(stream)), "uvl_numeric_pad_brush")


def numeric_pad_lasso(geom: GeometryImage, layer: NumericLayer, outline: Outline, view_proj, poly,
                      depth: torch.Tensor, bias: float, mode: int, value: float = 0.0, stream=None):
    M = _f32(view_proj, 16)
    P = _f32(poly).reshape(-1)
    dh, dw = depth.shape
    _check(_lib().uvl_numeric_pad_lasso(ctypes.byref(geom.c), ctypes.byref(layer.c), _ptr(outline.idx), outline.n,
                                        outline.k, M.ctypes.data_as(ctypes.c_void_p),
                                        P.ctypes.data_as(ctypes.c_void_p), P.size // 2, _ptr(depth), dw, dh,
                                        float(np.float32(bias)), int(mode), float(value), _stream(stream)),
           "uvl_numeric_pad_lasso")


def layer_op(op: int, dst: Layer, a: Layer, b: Optional[Layer] = None, sel_a: int = 0, sel_b: int = 0,
             out_label: int = 0, lut=None, stream=None):
    """lut: host table of 256 / 65536 uint16 entries (REMAP only; the
    library checks lut[0] == 0 and that every entry fits dst)."""
    host = None
    if op == REMAP:
        need = 256 if a.dtype == U8 else 65536
        if lut is None:
            raise ValueError(f"REMAP needs a host uint16 lut of {need} entries")
        if isinstance(lut, torch.Tensor):
            if lut.is_cuda:
                raise ValueError("REMAP tables are host arrays")
            lut = lut.numpy()
        host = np.ascontiguousarray(lut, dtype=np.uint16).reshape(-1)
        if host.size != need:
            raise ValueError(f"REMAP needs a host uint16 lut of {need} entries")
    _check(_lib().uvl_layer_op(int(op), ctypes.byref(dst.c), ctypes.byref(a.c),
                               None if b is None else ctypes.byref(b.c), int(sel_a), int(sel_b),
                               int(out_label), None if host is None else host.ctypes.data_as(ctypes.c_void_p),
                               _stream(stream)), "uvl_layer_op")


def nbins(layers: Sequence[Layer]) -> int:
    return sum(256 if l.dtype == U8 else 65536 for l in layers)


def bins_to_areas(bins: np.ndarray, nb: int, scale: float, wide: bool) -> np.ndarray:
    """fp64 areas of nb bins read back from the device (uint64 words; with
    two-word weights the low sums, then the high sums)."""
    b = np.asarray(bins).view(np.uint64)
    if not wide:
        return b[:nb].astype(np.float64) * scale
    lo, hi = b[:nb], b[nb:2 * nb]
    return np.array([float((int(h) << 32) + int(l)) * scale for l, h in zip(lo, hi)], np.float64)


def area_query(geom: GeometryImage, layers: Sequence[Layer], bins: Optional[torch.Tensor] = None,
               sync: bool = True, stream=None):
    """Per-label areas of each layer.

    sync=True: returns a list of fp64 numpy arrays (256 or 65536 bins each).
    sync=False: returns the device uint64 bins tensor (asynchronous; with
    two-word weights the low-word sums, then the high-word sums).
    """
    arr = (CLayer * len(layers))(*[l.c for l in layers])
    nb = nbins(layers)
    words = nb * (2 if geom.wide else 1)
    if bins is None:
        bins = torch.empty(words, dtype=torch.int64, device=geom.area_w.device)
    if bins.numel() < words:
        raise ValueError(f"bins needs {words} entries")
    host = np.empty(nb, np.float64) if sync else None
    _check(_lib().uvl_area_query(ctypes.byref(geom.c), arr, len(layers), _ptr(bins),
                                 None if host is None else host.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
           "uvl_area_query")
    if not sync:
        return bins
    out, off = [], 0
    for l in layers:
        k = 256 if l.dtype == U8 else 65536
        out.append(host[off:off + k])
        off += k
    return out


# ---------------------------------------------------------------------------
# batched edit waves


# uvl_edit as a numpy record (same offsets and size as CEdit), so a batch is
# filled one tuple per edit and handed to the library without a copy
EDIT_DTYPE = np.dtype({"names": [f[0] for f in CEdit._fields_],
                       "formats": ["<u8", "<u8", "<i4", "<u4", ("<f4", (3,)), "<f4", "<u8", "<u8", "<i4", "<i4",
                                   "<i4", "<f4", "<u8", "<u8", "<i4", "<i4", "<f8", "<u8", "<u8", "<i4", "<i4",
                                   "<u8"],
                       "offsets": [getattr(CEdit, f[0]).offset for f in CEdit._fields_],
                       "itemsize": ctypes.sizeof(CEdit)})


def _addr(a: np.ndarray) -> int:
    return a.__array_interface__["data"][0]


class EditBatch:
    """A packed array of uvl_edit records plus the host arrays they point to."""

    def __init__(self, capacity: int = 64):
        self._a = np.zeros(max(1, int(capacity)), EDIT_DTYPE)
        self._n = 0
        self._nl = 0
        self._keep = []

    def _slot(self) -> int:
        if self._n == self._a.shape[0]:
            a = np.zeros(2 * self._n, EDIT_DTYPE)
            a[:self._n] = self._a
            self._a = a
        self._n += 1
        return self._n - 1

    def brush(self, geom: GeometryImage, layer: Layer, center, radius: float, label: int,
              bins: Optional[torch.Tensor] = None):
        """bins: optional device uint64 area bins of the layer, kept up to
        date by the wave (uvl_edit.bins)."""
        c = _f32(center, 3)
        i = self._slot()
        self._a[i] = (geom.addr, layer.addr, EDIT_BRUSH, int(label), c, np.float32(radius), 0, 0, 0, 0, 0, 0.0, 0,
                      0, 0, 0, 0.0, 0, 0, 0, 0, 0 if bins is None else bins.data_ptr())
        self._keep.append((geom, layer, bins))

    def lasso(self, geom: GeometryImage, layer: Layer, view_proj, poly, depth: torch.Tensor, bias: float,
              label: int, bins: Optional[torch.Tensor] = None):
        M = _f32(view_proj, 16)
        P = _f32(poly).reshape(-1)
        dh, dw = depth.shape
        i = self._slot()
        self._a[i] = (geom.addr, layer.addr, EDIT_LASSO, int(label), (0.0, 0.0, 0.0), 0.0, _addr(M), _addr(P),
                      P.size // 2, dw, dh, np.float32(bias), depth.data_ptr(), 0, 0, 0, 0.0, 0, 0, 0, 0,
                      0 if bins is None else bins.data_ptr())
        self._nl += 1
        self._keep.append((geom, layer, M, P, depth, bins))

    def numeric_brush(self, geom: GeometryImage, layer: "NumericLayer", center, radius: float, mode: int,
                      value: float = 0.0):
        c = _f32(center, 3)
        i = self._slot()
        self._a[i] = (geom.addr, 0, EDIT_BRUSH, 0, c, np.float32(radius), 0, 0, 0, 0, 0, 0.0, 0,
                      ctypes.addressof(layer.c), int(mode), 0, float(value), 0, 0, 0, 0, 0)
        self._keep.append((geom, layer))

    def numeric_lasso(self, geom: GeometryImage, layer: "NumericLayer", view_proj, poly, depth: torch.Tensor,
                      bias: float, mode: int, value: float = 0.0):
        M = _f32(view_proj, 16)
        P = _f32(poly).reshape(-1)
        dh, dw = depth.shape
        i = self._slot()
        self._a[i] = (geom.addr, 0, EDIT_LASSO, 0, (0.0, 0.0, 0.0), 0.0, _addr(M), _addr(P), P.size // 2, dw, dh,
                      np.float32(bias), depth.data_ptr(), ctypes.addressof(layer.c), int(mode), 0, float(value),
                      0, 0, 0, 0, 0)
        self._nl += 1
        self._keep.append((geom, layer, M, P, depth))

    def _tool(self, geom, layer_addr, numeric_addr, label, mode, value, view_proj, tool, shape, depth, bias, keep):
        M = _f32(view_proj, 16)
        tp = np.ascontiguousarray(np.asarray(tool, dtype=np.float64))
        if tp.size != 6 or shape.dtype != torch.uint8 or shape.dim() != 2 or not shape.is_contiguous():
            raise ValueError("tool needs 6 numbers and a contiguous uint8 [sh, sw] shape")
        sh, sw = shape.shape
        dh, dw = depth.shape
        i = self._slot()
        self._a[i] = (geom.addr, layer_addr, EDIT_TOOL, int(label), (0.0, 0.0, 0.0), 0.0, _addr(M), 0, 0, dw, dh,
                      np.float32(bias), depth.data_ptr(), numeric_addr, int(mode), 0, float(value), _addr(tp),
                      shape.data_ptr(), sw, sh, 0)
        self._nl += 1
        self._keep.append((geom, keep, M, tp, shape, depth))

    def tool(self, geom: GeometryImage, layer: Layer, view_proj, tool, shape: torch.Tensor, depth: torch.Tensor,
             bias: float, label: int):
        """The paper's screen-space tool (as edit_tool) in the batch."""
        self._tool(geom, layer.addr, 0, label, 0, 0.0, view_proj, tool, shape, depth, bias, layer)

    def numeric_tool(self, geom: GeometryImage, layer: "NumericLayer", view_proj, tool, shape: torch.Tensor,
                     depth: torch.Tensor, bias: float, mode: int, value: float = 0.0):
        self._tool(geom, 0, ctypes.addressof(layer.c), 0, mode, value, view_proj, tool, shape, depth, bias, layer)

    def __len__(self):
        return self._n

    @property
    def n_lassos(self) -> int:
        return self._nl

    def array(self):
        """Pointer to the records (valid while the batch lives)."""
        return _addr(self._a)


class Wave:
    """Handle for batched edit waves (uvl_wave_*), workspace owned here."""

    def __init__(self, max_edits: int, max_lassos: int, max_cull_words: int = 1 << 22, device="cuda"):
        L = _lib()
        need = L.uvl_wave_workspace_bytes(int(max_edits), int(max_lassos), int(max_cull_words))
        if need == 0:
            raise ValueError("bad wave capacity")
        self.ws = torch.empty(need, dtype=torch.uint8, device=device)
        self.h = ctypes.c_void_p()
        _check(L.uvl_wave_create(int(max_edits), int(max_lassos), int(max_cull_words), _ptr(self.ws), need,
                                 ctypes.byref(self.h)), "uvl_wave_create")
        self.max_edits, self.max_lassos = int(max_edits), int(max_lassos)

    def submit(self, batch: EditBatch, tile_chunks: int = 0, stream=None, outlines=None):
        """Apply the batch; outlines = [(GeometryImage, Outline), ...] also pads
        the layers of those geometry images (uvl_wave_submit_padded)."""
        arr = batch.array()
        if not outlines:
            _check(_lib().uvl_wave_submit(self.h, arr, len(batch), int(tile_chunks), _stream(stream)),
                   "uvl_wave_submit")
            return
        ol = (CWaveOutline * len(outlines))(*[CWaveOutline(ctypes.addressof(g.c), o.idx.data_ptr(), o.n, o.k, 0)
                                               for g, o in outlines])
        _check(_lib().uvl_wave_submit_padded(self.h, arr, len(batch), int(tile_chunks), ol, len(outlines),
                                             _stream(stream)), "uvl_wave_submit_padded")

    def tune(self, batch: EditBatch, stream=None):
        arr = batch.array()
        _check(_lib().uvl_wave_tune(self.h, arr, len(batch), _stream(stream)), "uvl_wave_tune")

    def visited_tiles(self, stream=None) -> int:
        """Tiles the last submit visited (synchronous)."""
        v = ctypes.c_int64()
        _check(_lib().uvl_wave_visited_tiles(self.h, ctypes.byref(v), _stream(stream)), "uvl_wave_visited_tiles")
        return int(v.value)

    def tuned_chunks(self, texels: int) -> int:
        return int(_lib().uvl_wave_tuned_chunks(self.h, int(texels)))

    def close(self):
        if self.h:
            _lib().uvl_wave_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
