"""The allocation-free depth render (uvl_render_depth_noalloc) against the
workspace form (uvl_render_depth), through the C ABI: bit-identical depth
maps on two calls in a row, the second with a smaller mesh and map, so the
static scratch's left-over contents from the first call must not matter."""

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


def _pair(gpu, mesh, M, dw, dh):
    import torch
    dm = gpu.DeviceMesh.from_mesh(mesh)
    ref = torch.empty((dh, dw), dtype=torch.float32, device="cuda")
    got = torch.full((dh, dw), 7.0, dtype=torch.float32, device="cuda")
    gpu.render_depth(dm, M, ref)
    gpu.render_depth_noalloc(dm, M, got)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_depth_matches_workspace_form(gpu):
    print("case: sphere 65x33 grid at 640x480, vessel at 256x256, sphere 9x5 grid at 64x48", flush=True)
    # first call: a sphere seen from close by, many triangles larger than the
    # per-thread limit, so the scratch queue fills up
    big = synth.sphere(1.0, 65, 33)
    M1 = synth.edits.look_at_perspective((0.0, -1.5, 0.2), (0, 0, 0), (0, 0, 1))
    ref, got = _pair(gpu, big, M1, 640, 480)
    assert np.array_equal(ref, got)
    assert (ref < 1.0).sum() > 1000
    # second call: the vessel workload's first camera
    wl = synth.tiny_workload()
    ref, got = _pair(gpu, wl.mesh, wl.cameras[0], 256, 256)
    assert np.array_equal(ref, got)
    # third call, smaller again: fewer triangles, a smaller map
    small = synth.sphere(1.0, 9, 5)
    M3 = synth.edits.look_at_perspective((0.0, -1.8, 0.4), (0, 0, 0), (0, 0, 1))
    ref, got = _pair(gpu, small, M3, 64, 48)
    assert np.array_equal(ref, got)
    assert (ref < 1.0).any()


def test_noalloc_depth_refuses_too_many_triangles(gpu):
    import ctypes
    import torch
    n = gpu.lib().uvl_render_depth_noalloc
    m = gpu.CMesh(0x100000, None, 0x100000, 0x100000, 10, 4194305)
    d = torch.empty((4, 4), dtype=torch.float32, device="cuda")
    M = (ctypes.c_float * 16)()
    assert n(ctypes.byref(m), M, d.data_ptr(), 4, 4, None) == -4
