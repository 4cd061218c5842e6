"""Host logic of bench.py (no GPU): the one-GPU refusal, the bytes an area
query must read, the counter summary's source check and the headline
roofline object."""

import os
import subprocess
import sys
import types

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and not p.stdout


class _Layer:
    def __init__(self, data, dtype):
        self.data, self.dtype = data, dtype


def _model(layers, W, H, blk=True):
    geom = types.SimpleNamespace(width=W, height=H, area_blk=object() if blk else None)
    return types.SimpleNamespace(geom=geom, layers=layers)


def test_area_needed_bytes():
    torch = pytest.importorskip("torch")
    uvl = types.SimpleNamespace(U8=1, U16=2)
    W, H = 64, 16
    N = W * H
    a = torch.zeros(N + 64, dtype=torch.uint8)          # padded like the binding's planes
    b = torch.zeros(N + 64, dtype=torch.int16)
    a[3] = 7                                             # block (0, 0) mixed in layer a
    b[5 * W + 20] = 9                                    # block row 1, block column 2 mixed in b
    b[6 * W + 20] = 9                                    # the same block again
    one = bench.area_needed_bytes(_model([_Layer(a, 1)], W, H), uvl, torch)
    assert one == N * 1 + 8 * (N // 32) + 4 * 32 * 1
    two = bench.area_needed_bytes(_model([_Layer(a, 1), _Layer(b, 2)], W, H), uvl, torch)
    assert two == N * 3 + 8 * (N // 32) + 4 * 32 * 2
    # without block sums, with more than two layers, or sizes the blocks do
    # not tile: every weight
    assert bench.area_needed_bytes(_model([_Layer(a, 1)], W, H, blk=False), uvl, torch) == N + 4 * N
    three = [_Layer(a, 1)] * 3
    assert bench.area_needed_bytes(_model(three, W, H), uvl, torch) == 3 * N + 4 * N
    c = torch.zeros(60 * 16 + 64, dtype=torch.uint8)
    assert bench.area_needed_bytes(_model([_Layer(c, 1)], 60, 16), uvl, torch) == 60 * 16 * 5


def test_counters_need_the_current_sources(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel one")
    prof = tmp_path / "profiles"
    prof.mkdir()
    import hashlib
    import json
    sha = hashlib.sha256(b"kernel one").hexdigest()
    (prof / "pmc_counters.json").write_text(json.dumps({"edit_brush": {"source_sha256": sha, "bytes_per_launch": 5}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counters_from_profiles("edit_brush", ["k.hip"])["bytes_per_launch"] == 5
    src.write_text("kernel two")
    assert bench.counters_from_profiles("edit_brush", ["k.hip"]) is None
    assert bench.counters_from_profiles("edit_lasso", ["k.hip"]) is None


def test_headline_roofline_objects():
    """The headline object against the VALU issue peak for a kernel marked
    VALU-bound (the per-kernel rule: VALU fraction above the HBM fraction),
    against HBM otherwise; both fractions kept."""
    rl = {"bytes_per_launch": 1e9, "avg_us": 100.0, "traffic": None, "frac": 0.6, "achieved": 4800.0,
          "valu_frac": 0.9, "bound": "alu"}
    h = bench.headline_roofline("edit_lasso", rl)
    assert h["bound"] == "alu" and h["frac"] == 0.9 and h["hbm_frac"] == 0.6
    assert h["peak"] == pytest.approx(bench.VALU_PEAK_LANE_OPS / 1e12)
    assert h["achieved"] == pytest.approx(0.9 * bench.VALU_PEAK_LANE_OPS / 1e12)
    rl.update(valu_frac=0.2, bound="hbm")
    h = bench.headline_roofline("edit_brush", rl)
    assert h["bound"] == "hbm" and h["frac"] == 0.6 and h["unit"] == "GB/s" and h["peak"] == bench.HBM_PEAK_GBPS
    assert h["valu_frac"] == 0.2
