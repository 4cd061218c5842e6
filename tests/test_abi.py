"""The C ABI loads and exports every symbol include/uvl.h declares (no GPU).

Only validation paths that return before any HIP call are exercised here:
null pointers, sizes out of range, dtype and shape mismatches.  Fake device
addresses are never dereferenced on these paths.
"""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "uvl.h")


def _declared():
    hdr = open(HEADER).read()
    return re.findall(r"^\w[\w\s\*]*?\b(uvl_\w+)\s*\(", hdr, re.M)


@pytest.fixture(scope="module")
def uvl():
    from paper_2501_14807_amd import uvl as U
    if not os.path.exists(U.LIB_PATH):
        from paper_2501_14807_amd import build
        build.build()
    return U


def test_header_and_binding_agree(uvl):
    assert sorted(_declared()) == sorted(uvl.SIGNATURES)


def test_library_exports_every_declared_symbol(uvl):
    L = uvl.lib()
    for name in _declared():
        assert hasattr(L, name), name
    # and with C linkage (plain names in the dynamic symbol table)
    out = os.popen(f"nm -D --defined-only {uvl.LIB_PATH}").read()
    for name in _declared():
        assert re.search(rf"\bT {name}$", out, re.M), name


def test_status_strings(uvl):
    L = uvl.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert L.uvl_status_str(code)
    assert L.uvl_status_str(-99) == b"unknown status"


FAKE = 0x100000        # a 16-byte aligned address that is never dereferenced


def _geom(uvl, w=64, h=32):
    g = uvl.CGeom()
    g.width, g.height = w, h
    g.tri_id = g.area_w = FAKE
    g.pos_x = g.pos_y = g.pos_z = FAKE
    return g


def _layer(uvl, w=64, h=32, dt=1):
    return uvl.CLayer(FAKE, w, h, dt)


def test_brush_validation(uvl):
    L = uvl.lib()
    g, l = _geom(uvl), _layer(uvl)
    c = (ctypes.c_float * 3)(0, 0, 0)
    s = None
    assert L.uvl_edit_brush(None, ctypes.byref(l), c, 1.0, 1, s) == -1
    assert L.uvl_edit_brush(ctypes.byref(g), ctypes.byref(l), None, 1.0, 1, s) == -1
    assert L.uvl_edit_brush(ctypes.byref(g), ctypes.byref(l), c, -1.0, 1, s) == -1
    assert L.uvl_edit_brush(ctypes.byref(g), ctypes.byref(l), c, float("nan"), 1, s) == -1
    assert L.uvl_edit_brush(ctypes.byref(g), ctypes.byref(l), c, float("inf"), 1, s) == -1
    assert L.uvl_edit_brush(ctypes.byref(g), ctypes.byref(l), c, 1.0, 256, s) == -3
    l16 = _layer(uvl, dt=2)
    assert L.uvl_edit_brush(ctypes.byref(g), ctypes.byref(l16), c, 1.0, 65536, s) == -3
    lbad = _layer(uvl, dt=7)
    assert L.uvl_edit_brush(ctypes.byref(g), ctypes.byref(lbad), c, 1.0, 1, s) == -3
    lsz = _layer(uvl, w=63)
    assert L.uvl_edit_brush(ctypes.byref(g), ctypes.byref(lsz), c, 1.0, 1, s) == -2
    unaligned = uvl.CLayer(FAKE + 4, 64, 32, 1)
    assert L.uvl_edit_brush(ctypes.byref(g), ctypes.byref(unaligned), c, 1.0, 1, s) == -1
    g.pos_y = FAKE + 8
    assert L.uvl_edit_brush(ctypes.byref(g), ctypes.byref(l), c, 1.0, 1, s) == -1


def test_lasso_validation(uvl):
    L = uvl.lib()
    g, l = _geom(uvl), _layer(uvl)
    M = (ctypes.c_float * 16)(*([1.0] * 16))
    poly = (ctypes.c_float * 200)(*([0.5] * 200))
    s = None
    call = lambda n, dw=32, dh=32, bias=1e-4, depth=FAKE, label=1: L.uvl_edit_lasso(
        ctypes.byref(g), ctypes.byref(l), M, poly, n, depth, dw, dh, bias, label, s)
    assert call(2) == -1
    assert call(65) == -1
    assert call(8, depth=None) == -1
    assert call(8, dw=0) == -1
    assert call(8, dh=20000) == -1
    assert call(8, bias=float("nan")) == -1
    assert call(8, label=300) == -3
    poly[3] = float("nan")
    assert call(8) == -1


def test_layer_op_and_area_validation(uvl):
    L = uvl.lib()
    a, b = _layer(uvl), _layer(uvl)
    d16 = _layer(uvl, dt=2)
    s = None
    assert L.uvl_layer_op(9, ctypes.byref(a), ctypes.byref(a), ctypes.byref(b), 0, 0, 1, None, s) == -1
    assert L.uvl_layer_op(0, ctypes.byref(a), ctypes.byref(a), None, 0, 0, 1, None, s) == -1
    assert L.uvl_layer_op(0, ctypes.byref(a), ctypes.byref(a), ctypes.byref(b), 0, 0, 256, None, s) == -3
    assert L.uvl_layer_op(0, ctypes.byref(d16), ctypes.byref(a), ctypes.byref(_layer(uvl, h=31)), 0, 0, 1, None,
                          s) == -2
    assert L.uvl_layer_op(3, ctypes.byref(a), ctypes.byref(a), None, 0, 0, 0, None, s) == -1
    g = _geom(uvl)
    arr = (uvl.CLayer * 2)(a, _layer(uvl, w=8))
    assert L.uvl_area_query(ctypes.byref(g), arr, 2, FAKE, None, s) == -2
    assert L.uvl_area_query(ctypes.byref(g), arr, 0, FAKE, None, s) == -1
    assert L.uvl_area_query(ctypes.byref(g), arr, 33, FAKE, None, s) == -1
    assert L.uvl_area_query(ctypes.byref(g), arr, 1, None, None, s) == -1


def test_remap_tables_are_checked_on_the_host(uvl):
    """REMAP tables: the null key must map to itself (UVL_E_INVAL) and every
    entry must fit the destination's dtype (UVL_E_DTYPE); both are refused
    before anything is enqueued (fake device addresses, no GPU)."""
    L = uvl.lib()
    a8, a16, d8, d16 = _layer(uvl), _layer(uvl, dt=2), _layer(uvl), _layer(uvl, dt=2)
    s = None

    def remap(dst, a, lut):
        return L.uvl_layer_op(3, ctypes.byref(dst), ctypes.byref(a), None, 0, 0, 0,
                              lut.ctypes.data_as(ctypes.c_void_p), s)

    for a, n in ((a8, 256), (a16, 65536)):
        for dst in (d8, d16):
            lut = np.arange(n, dtype=np.uint16) % 200
            lut[0] = 7
            assert remap(dst, a, lut) == -1
        lut = np.zeros(n, np.uint16)
        lut[n - 1] = 256                    # does not fit a u8 destination
        assert remap(d8, a, lut) == -3
        lut[n - 1] = 65535
        assert remap(d8, a, lut) == -3
    lut = np.zeros(256, np.uint16)
    lut[255] = 256
    assert remap(d8, a8, lut) == -3


def test_geom_bytes(uvl):
    """uvl_geom_bytes: each 4-byte plane rounded to 256 bytes, optional
    planes by flag, the tile bounds of ceil(W/32) x ceil(H/32) tiles and of
    their blocks of 8 x 8 tiles, the area sums of 4 x 8 texel blocks."""
    L = uvl.lib()

    def plane(w, h):
        return -(-w * h * 4 // 256) * 256

    for w, h in ((1, 1), (37, 53), (512, 512), (8192, 8192), (32768, 3)):
        tx, ty = -(-w // 32), -(-h // 32)
        blocks = -(-tx // 8) * -(-ty // 8)
        box = -(-(tx * ty + blocks) * 24 // 256) * 256
        assert L.uvl_geom_bytes(w, h, 0) == 5 * plane(w, h)
        assert L.uvl_geom_bytes(w, h, 1) == 8 * plane(w, h)
        assert L.uvl_geom_bytes(w, h, 2) == 7 * plane(w, h)
        assert L.uvl_geom_bytes(w, h, 7) == 10 * plane(w, h) + box
        blk = -(-(-(-w // 8) * -(-h // 4) * 8) // 256) * 256
        assert L.uvl_geom_bytes(w, h, 16) == 5 * plane(w, h) + blk
    assert L.uvl_geom_bytes(0, 5, 0) == 0
    assert L.uvl_geom_bytes(5, 32769, 0) == 0
    assert L.uvl_geom_bytes(5, 5, 64) == 0
    # the binding's geometry image allocates what the library states (CPU tensors)
    g = uvl.GeometryImage(300, 173, device="cpu")
    assert g.nbytes() <= L.uvl_geom_bytes(300, 173, 7 | 16) < g.nbytes() + 2 * 256


def test_build_and_depth_validation(uvl):
    L = uvl.lib()
    m = uvl.CMesh(FAKE, None, FAKE, FAKE, 10, 4)
    g = _geom(uvl)
    ws_need = L.uvl_build_workspace_bytes(4, 64, 32)
    assert L.uvl_build_workspace_bytes(4, 0, 32) == 0 and L.uvl_build_workspace_bytes(-1, 64, 32) == 0
    assert ws_need >= 4 * 12
    assert L.uvl_build_geometry_image(ctypes.byref(m), ctypes.byref(g), FAKE, ws_need - 1, None) == -4
    g.width = 40000
    assert L.uvl_build_geometry_image(ctypes.byref(m), ctypes.byref(g), FAKE, ws_need, None) == -1
    g.width = 64
    g.nrm_x = FAKE
    assert L.uvl_build_geometry_image(ctypes.byref(m), ctypes.byref(g), FAKE, ws_need, None) == -1
    M = (ctypes.c_float * 16)()
    dws = L.uvl_depth_workspace_bytes(4)
    assert L.uvl_render_depth(ctypes.byref(m), M, FAKE, 0, 16, FAKE, dws, None) == -1
    assert L.uvl_render_depth(ctypes.byref(m), M, FAKE, 16, 16, FAKE, dws - 1, None) == -4
    big = uvl.CMesh(FAKE, None, FAKE, FAKE, 10, 4194305)     # above the scratch's limit
    assert L.uvl_render_depth_noalloc(ctypes.byref(big), M, FAKE, 16, 16, None) == -4
    assert L.uvl_render_depth_noalloc(ctypes.byref(m), M, FAKE, 16, 0, None) == -1
    assert L.uvl_render_depth_noalloc(None, M, FAKE, 16, 16, None) == -1
    assert L.uvl_create_layer(ctypes.byref(_layer(uvl, dt=5)), None) == -3
    assert L.uvl_create_layer(None, None) == -1


def test_edit_records_match_the_c_struct():
    """EditBatch fills numpy records that the library reads as uvl_edit."""
    import ctypes
    import torch
    from paper_2501_14807_amd import uvl

    class Fake:
        def __init__(self, addr):
            self.addr = addr

    g, lay = Fake(0x1000), Fake(0x2000)
    b = uvl.EditBatch(capacity=1)              # also exercises growth
    b.brush(g, lay, (0.25, -1.5, 3.0), 0.125, 7)
    M = np.arange(16, dtype=np.float32)
    poly = np.array([[0, 0], [1, 0], [0, 1]], np.float32)
    d = torch.zeros((48, 64), dtype=torch.float32)
    b.lasso(g, lay, M, poly, d, 1e-4, 9)
    assert len(b) == 2 and b.n_lassos == 1
    raw = ctypes.string_at(b.array(), 2 * ctypes.sizeof(uvl.CEdit))
    r0 = uvl.CEdit()
    r0.geom, r0.layer, r0.kind, r0.label = 0x1000, 0x2000, uvl.EDIT_BRUSH, 7
    r0.center[0], r0.center[1], r0.center[2], r0.radius = 0.25, -1.5, 3.0, 0.125
    r1 = uvl.CEdit()
    r1.geom, r1.layer, r1.kind, r1.label = 0x1000, 0x2000, uvl.EDIT_LASSO, 9
    keep = b._keep[1]
    r1.view_proj, r1.poly_xy, r1.npoly = keep[2].ctypes.data, keep[3].ctypes.data, 3
    r1.dw, r1.dh, r1.bias, r1.depth = 64, 48, np.float32(1e-4), d.data_ptr()
    assert raw == bytes(r0) + bytes(r1)
    # numeric edits: the layer slot is empty and the numeric descriptor,
    # mode and value fill the trailing fields
    nl = uvl.CNumeric(0x3000, 0x4000, 8, 8, uvl.F16)

    class FakeNum:
        c = nl

    b.numeric_brush(g, FakeNum(), (1.0, 2.0, 3.0), 0.5, uvl.ERASE, -2.25)
    raw = ctypes.string_at(b.array() + 2 * ctypes.sizeof(uvl.CEdit), ctypes.sizeof(uvl.CEdit))
    r2 = uvl.CEdit()
    r2.geom, r2.kind = 0x1000, uvl.EDIT_BRUSH
    r2.center[0], r2.center[1], r2.center[2], r2.radius = 1.0, 2.0, 3.0, 0.5
    r2.numeric, r2.mode, r2.value = ctypes.addressof(nl), uvl.ERASE, -2.25
    assert raw == bytes(r2)
    # a tool edit: its parameters, shape and sizes in the trailing fields
    shape = torch.ones((5, 7), dtype=torch.uint8)
    b.tool(g, lay, M, (640, 480, 320, 240, 100, 90), shape, d, 1e-4, 11)
    raw = ctypes.string_at(b.array() + 3 * ctypes.sizeof(uvl.CEdit), ctypes.sizeof(uvl.CEdit))
    keep = b._keep[3]
    r3 = uvl.CEdit()
    r3.geom, r3.layer, r3.kind, r3.label = 0x1000, 0x2000, uvl.EDIT_TOOL, 11
    r3.view_proj, r3.dw, r3.dh, r3.bias, r3.depth = keep[2].ctypes.data, 64, 48, np.float32(1e-4), d.data_ptr()
    r3.tool, r3.shape, r3.sw, r3.sh = keep[3].ctypes.data, shape.data_ptr(), 7, 5
    assert raw == bytes(r3) and list(keep[3]) == [640, 480, 320, 240, 100, 90]


def test_padding_validation(uvl):
    L = uvl.lib()
    g, l = _geom(uvl), _layer(uvl)
    c = (ctypes.c_float * 3)(0, 0, 0)
    s = None
    assert L.uvl_outline_workspace_bytes(0, 5) == 0 and L.uvl_outline_workspace_bytes(64, 32) >= 8
    n = ctypes.c_int64()
    ws_bytes = L.uvl_outline_workspace_bytes(64, 32)
    assert L.uvl_build_outline(None, 1, FAKE, 10, ctypes.byref(n), FAKE, ws_bytes, s) == -1
    assert L.uvl_build_outline(ctypes.byref(g), 9, FAKE, 10, ctypes.byref(n), FAKE, ws_bytes, s) == -1
    assert L.uvl_build_outline(ctypes.byref(g), -1, FAKE, 10, ctypes.byref(n), FAKE, ws_bytes, s) == -1
    assert L.uvl_build_outline(ctypes.byref(g), 1, FAKE, 10, None, FAKE, ws_bytes, s) == -1
    assert L.uvl_build_outline(ctypes.byref(g), 1, FAKE, 10, ctypes.byref(n), FAKE, ws_bytes - 1, s) == -4
    pad = lambda k=1, n_=4, label=1, layer=l, out=FAKE: L.uvl_pad_brush(
        ctypes.byref(g), ctypes.byref(layer), out, n_, k, c, 1.0, label, s)
    assert pad(k=9) == -1 and pad(k=-1) == -1
    assert pad(n_=-1) == -1 and pad(out=None) == -1
    assert pad(n_=64 * 32 + 1) == -2
    assert pad(label=256) == -3
    assert pad(layer=_layer(uvl, w=63)) == -2
    M = (ctypes.c_float * 16)(*([1.0] * 16))
    poly = (ctypes.c_float * 6)(0, 0, 1, 0, 0, 1)
    assert L.uvl_pad_lasso(ctypes.byref(g), ctypes.byref(l), FAKE, 4, 1, M, poly, 2, FAKE, 32, 32, 1e-4, 1, s) == -1
    assert L.uvl_pad_lasso(ctypes.byref(g), ctypes.byref(l), FAKE, 4, 1, M, poly, 3, None, 32, 32, 1e-4, 1, s) == -1


def test_tool_validation(uvl):
    L = uvl.lib()
    g, l = _geom(uvl), _layer(uvl)
    M = (ctypes.c_float * 16)(*([1.0] * 16))
    s = None
    ok = [1024.0, 768.0, 500.0, 400.0, 100.0, 100.0]

    def call(tool=ok, shape=FAKE, sw=16, sh=16, depth=FAKE, dw=32, dh=32, bias=1e-4, label=1, layer=l):
        t = (ctypes.c_double * 6)(*tool)
        return L.uvl_edit_tool(ctypes.byref(g), ctypes.byref(layer), M, t, shape, sw, sh, depth, dw, dh, bias,
                               label, s)

    assert call(tool=[1024, 768, 500, 400, 0, 100]) == -1
    assert call(tool=[0, 768, 500, 400, 10, 100]) == -1
    assert call(tool=[1024, 768, float("nan"), 400, 10, 100]) == -1
    assert call(shape=None) == -1 and call(depth=None) == -1
    assert call(sw=0) == -1 and call(sh=5000) == -1
    assert call(dw=0) == -1 and call(bias=float("inf")) == -1
    assert call(label=256) == -3
    assert call(layer=_layer(uvl, h=31)) == -2


def test_numeric_validation(uvl):
    """Numeric layers: every argument error is caught on the host, before the
    device check (which fails here without a GPU: -5 or -6 means the
    arguments passed)."""
    L = uvl.lib()
    g = _geom(uvl)
    c = (ctypes.c_float * 3)(0.0, 0.0, 0.0)
    passed = (-5, -6, 0)

    def nl(dt=uvl.F32, w=64, h=32, mask=FAKE):
        return uvl.CNumeric(FAKE, mask, w, h, dt)

    def brush(layer, mode=uvl.SET, value=1.0):
        return L.uvl_numeric_brush(ctypes.byref(g), ctypes.byref(layer), c, 1.0, mode, value, None)

    assert brush(nl(dt=6)) == -1 and brush(nl(dt=0)) == -1
    assert brush(nl(mask=None)) == -1 and brush(nl(mask=FAKE + 4)) == -1
    assert brush(nl(), mode=2) == -1
    assert brush(nl(), value=float("nan")) == -1
    assert brush(nl(), mode=uvl.ERASE, value=float("nan")) in passed
    assert brush(nl(h=31)) == -2
    for dt, bad, good in ((uvl.U8, 256, 255), (uvl.U8, -1, 0), (uvl.U16, 65536, 65535), (uvl.I32, 1.5, -7),
                          (uvl.I32, 2.0 ** 31, -2.0 ** 31), (uvl.F16, 65520.0, 65519.0),
                          (uvl.F32, 1e39, 3.4e38), (uvl.F32, float("inf"), -1e-45)):
        assert brush(nl(dt=dt), value=bad) == -3, (dt, bad)
        assert brush(nl(dt=dt), value=good) in passed, (dt, good)
    src, dst = nl(), _layer(uvl)
    sel = lambda lo=0.0, hi=1.0, d=dst, label=1: L.uvl_numeric_select(ctypes.byref(src), lo, hi, ctypes.byref(d),
                                                                      label, None)
    assert sel(lo=float("nan")) == -1 and sel(hi=float("nan")) == -1
    assert sel(d=_layer(uvl, dt=3)) == -3 and sel(label=256) == -3
    assert sel(d=_layer(uvl, w=32)) == -2
    assert sel(lo=2.0, hi=1.0) in passed
    st = lambda region=None, bins=FAKE, layer=src: L.uvl_numeric_stats(
        ctypes.byref(g), ctypes.byref(layer), None if region is None else ctypes.byref(region), bins, None, None)
    assert st(bins=None) == -1 and st(bins=FAKE + 4) == -1
    assert st(region=_layer(uvl, dt=3)) == -3 and st(region=_layer(uvl, h=16)) == -2
    assert st(layer=nl(w=32)) == -2
    assert st() in passed and st(region=_layer(uvl, dt=2)) in passed
    M = (ctypes.c_float * 16)(*([1.0] * 16))
    poly = (ctypes.c_float * 6)(0, 0, 1, 0, 0, 1)
    pb = lambda n=4, k=1, outline=FAKE, mode=uvl.SET, layer=src: L.uvl_numeric_pad_brush(
        ctypes.byref(g), ctypes.byref(layer), outline, n, k, c, 1.0, mode, 1.0, None)
    pl = lambda n=4, k=1, npoly=3: L.uvl_numeric_pad_lasso(ctypes.byref(g), ctypes.byref(src), FAKE, n, k, M, poly,
                                                           npoly, FAKE, 32, 32, 1e-4, uvl.SET, 1.0, None)
    assert pb(k=9) == -1 and pb(k=-1) == -1 and pb(outline=None) == -1 and pb(n=-1) == -1
    assert pb(n=64 * 32 + 1) == -2 and pb(mode=5) == -1 and pb(layer=nl(dt=7)) == -1
    assert pb(layer=nl(dt=uvl.U8)) in passed and pb(n=0, outline=None) in passed
    assert pl(npoly=2) == -1 and pl(k=9) == -1 and pl() in passed


def test_pool_validation(uvl):
    """Layer pool: argument errors are caught on the host (creation needs
    the device: -5 or -6 without one)."""
    L = uvl.lib()
    h = ctypes.c_void_p()
    assert L.uvl_pool_create(0, ctypes.byref(h)) == -1 and L.uvl_pool_create(65537, ctypes.byref(h)) == -1
    assert L.uvl_pool_create(8, None) == -1
    assert L.uvl_pool_create(8, ctypes.byref(h)) in (-5, -6, 0)
    if h.value:
        L.uvl_pool_destroy(h)
    p, s = ctypes.c_void_p(), ctypes.c_int32()
    assert L.uvl_pool_alloc(None, 64, 64, 1, ctypes.byref(p), ctypes.byref(s)) == -1
    assert L.uvl_pool_free(None, FAKE) == -1
    r, c, k = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_int32()
    assert L.uvl_pool_stats(None, ctypes.byref(r), ctypes.byref(c), ctypes.byref(k)) == -1
    assert L.uvl_pool_array(None, 64, 64, 1, ctypes.byref(p), ctypes.byref(ctypes.c_size_t()), ctypes.byref(s)) == -1
    assert L.uvl_pool_destroy(None) == -1


def test_ctypes_structs_match_the_header(uvl, tmp_path):
    """Sizes and field offsets of the binding's structures equal those a C
    compiler gives the header's (gcc, this machine's ABI)."""
    import subprocess
    structs = {"uvl_mesh": uvl.CMesh, "uvl_geom": uvl.CGeom, "uvl_layer": uvl.CLayer,
               "uvl_numeric": uvl.CNumeric, "uvl_edit": uvl.CEdit, "uvl_wave_outline": uvl.CWaveOutline}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "uvl.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f in cls._fields_:
            lines.append(f'printf("{cname}.{f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines.append('printf("uvl_numstat %zu\\n", sizeof(uvl_numstat));')
    for f in uvl.NUMSTAT.names:
        lines.append(f'printf("uvl_numstat.{f} %zu\\n", offsetof(uvl_numstat, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)]).decode().split("\n") if l)
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert int(got[f"{cname}.{f[0]}"]) == getattr(cls, f[0]).offset, (cname, f[0])
    assert int(got["uvl_numstat"]) == uvl.NUMSTAT.itemsize
    for f in uvl.NUMSTAT.names:
        assert int(got[f"uvl_numstat.{f}"]) == uvl.NUMSTAT.fields[f][1], f
