"""The layer pool on the GPU (uvl_pool_*): the layers of a (width, height,
dtype) key occupy consecutive slots of one reserved range, memory is
committed per layer and returned on free (a freed slot is reused), a full
key reports UVL_E_NOMEM, and edits on pool layers give exactly the layers
they give on ordinary device memory."""

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


def test_pool_slots_and_accounting(gpu):
    pool = gpu.LayerPool(slots_per_key=4)
    try:
        a = pool.alloc(1024, 1024, gpu.U8)
        b = pool.alloc(1024, 1024, gpu.U8)
        c = pool.alloc(300, 200, gpu.U16)
        base, stride, slots = pool.array(1024, 1024, gpu.U8)
        assert slots == 4 and stride >= 1024 * 1024 and a.ptr == base and b.ptr == base + stride
        assert (a.slot, b.slot, c.slot) == (0, 1, 0) and a.ptr % 256 == 0 and c.ptr % 256 == 0
        base16, stride16, _ = pool.array(300, 200, gpu.U16)
        assert c.ptr == base16 and stride16 >= 300 * 200 * 2
        reserved, committed, keys = pool.stats()
        assert keys == 2 and reserved == 4 * (stride + stride16) and committed == 2 * stride + stride16
        pool.free(b)
        assert pool.stats()[1] == stride + stride16
        b2 = pool.alloc(1024, 1024, gpu.U8)
        assert b2.slot == 1 and b2.ptr == base + stride
        more = [pool.alloc(1024, 1024, gpu.U8) for _ in range(2)]
        with pytest.raises(gpu.UvlError) as err:
            pool.alloc(1024, 1024, gpu.U8)
        assert err.value.code == -4
        pool.free(b2)
        with pytest.raises(gpu.UvlError):
            pool.free(b2)                      # no longer committed
        for x in [a, c] + more:
            pool.free(x)
        assert pool.stats()[1] == 0
    finally:
        pool.close()


def test_pool_layers_edit_like_device_layers(gpu):
    """Edits, algebra and areas on pool layers equal those on torch-backed
    layers, bit for bit."""
    import torch
    from paper_2501_14807_amd.model import Model
    wl = synth.scan_workload(n_brush=16, n_lasso=16, n_ops=0, W=512, n_charts=4, nx=64, ny=32, depth=256)
    m = Model.from_workload(wl).build()
    pool = gpu.LayerPool(slots_per_key=8)
    try:
        P = [gpu.create_layer(pool.alloc(wl.W, wl.H, dt)) for dt in (gpu.U8, gpu.U16)]
        T = [gpu.create_layer(gpu.Layer(wl.W, wl.H, dt)) for dt in (gpu.U8, gpu.U16)]
        for i, e in enumerate(wl.edits):
            label = 1 + e.label % 200           # fits both layers
            for layers in (P, T):
                lay = layers[i % 2]
                if e.kind == "brush":
                    gpu.edit_brush(m.geom, lay, e.centre, e.radius, label)
                else:
                    M = wl.cameras[e.camera]
                    gpu.edit_lasso(m.geom, lay, M, e.poly, m.depth_for(e.camera, M), m.bias, label)
        for layers in (P, T):
            gpu.layer_op(gpu.OR, layers[0], layers[0], layers[1], 0, 0, 5)
        torch.cuda.synchronize()
        for p_, t_ in zip(P, T):
            assert np.array_equal(p_.numpy(), t_.numpy())
        assert P[0].numpy().any()
        bins = torch.empty(gpu.nbins(P), dtype=torch.int64, device="cuda")
        ap = gpu.area_query(m.geom, P, bins)
        at = gpu.area_query(m.geom, T)
        for x, y in zip(ap, at):
            assert np.array_equal(x, y)
        # host upload into a pool layer
        ref = (np.arange(wl.W * wl.H) % 251).astype(np.uint8)
        P[0].copy_from(ref)
        assert np.array_equal(P[0].numpy(), ref)
    finally:
        torch.cuda.synchronize()
        pool.close()
