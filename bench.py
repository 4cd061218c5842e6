"""Benchmark of the texture-layer hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload scan|tiny] [--no-cpu-baseline]

Workload (default): the scan-scale model -- 64 displaced 256x128-vertex charts
(4,145,280 triangles) shelf-packed into an 8192^2 atlas, 8 u8 + 1 u16 layers,
1,000 brush edits, 1,000 lasso edits (3-32 vertex polygons, one camera per 8
lassos, 2048^2 depth maps), 256 layer operations, per-label areas of all 9
layers.  Inputs are synthetic and seeded, resident in HBM before timing.

One step = one pass of the whole path: build the geometry image, clear the
layers, apply the 2,000 edits in order (rendering a depth map whenever the
camera changes), apply the 256 layer operations, query all areas.  K steps
are timed between device synchronisations; the metric is edited texels per
second (every edit evaluates every texel of the atlas, as in the paper's
editing pass).  Per-kernel durations come from HIP events recorded on the
launch stream around every launch inside the timed steps.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="scan", choices=["scan", "tiny"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-rows", type=int, default=64, help="atlas rows in the oracle's timed sample")
    p.add_argument("--cpu-edits", type=int, default=200, help="edits in the oracle's timed sample")
    return p.parse_args()


def make_workload(name):
    import synth
    if name == "tiny":
        return synth.tiny_workload(), "vessel 128^2 vertices (32,258 tris), 512^2 atlas, 1 u8 layer, 64 edits"
    wl = synth.scan_workload()
    return wl, ("scan-scale: 64 displaced 256x128 charts (4,145,280 tris), 8192^2 atlas, 8 u8 + 1 u16 layers, "
                "1000 brush + 1000 lasso (2048^2 depth) + 256 layer ops + per-label area")


class Timer:
    """HIP events on the current (launch) stream around every launch."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = {}
        self.on = False

    def span(self, name):
        timer = self

        class _S:
            def __enter__(s):
                if timer.on:
                    s.a = timer.torch.cuda.Event(enable_timing=True)
                    s.a.record()

            def __exit__(s, *exc):
                if timer.on:
                    b = timer.torch.cuda.Event(enable_timing=True)
                    b.record()
                    timer.pairs.setdefault(name, []).append((s.a, b))
        return _S()

    def stats(self):
        out = {}
        for name, prs in self.pairs.items():
            ms = [a.elapsed_time(b) for a, b in prs]
            out[name] = {"count": len(ms), "avg_us": 1e3 * sum(ms) / len(ms), "total_ms": sum(ms)}
        return out


def run_step(m, wl, uvl, T):
    with T.span("build_geometry_image"):
        uvl.build_geometry_image(m.mesh, m.geom, m.build_ws)
    for l in m.layers:
        uvl.create_layer(l)
    m._depth.clear()
    for e in wl.edits:
        layer = m.layers[e.layer]
        if e.kind == "brush":
            with T.span("edit_brush"):
                uvl.edit_brush(m.geom, layer, e.centre, e.radius, e.label)
        else:
            M = wl.cameras[e.camera]
            if e.camera not in m._depth:
                with T.span("render_depth"):
                    m.depth_for(e.camera, M)
            d = m.depth_for(e.camera, M)
            with T.span("edit_lasso"):
                uvl.edit_lasso(m.geom, layer, M, e.poly, d, m.bias, e.label)
    for o in wl.ops:
        with T.span("layer_op"):
            m.apply_op(o)
    with T.span("area_query"):
        bins = m.areas(sync=False)
    return bins


def copy_bandwidth(torch, nbytes=2 << 30, reps=10):
    """Achievable HBM bandwidth of a plain device-to-device copy (read + write)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return 2 * nbytes / s / 1e9


def cpu_baseline(wl, rows, n_edits):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import oracle
    from oracle import workload
    oracle.build(force=False)
    edits = wl.edits[:n_edits]
    t0 = time.perf_counter()
    og = oracle.geometry_image(wl.mesh, wl.W, wl.H, rows=(0, rows))
    t1 = time.perf_counter()
    cache = {}
    for e in edits:     # depth maps for the sampled lassos, timed apart from the edits
        if e.kind == "lasso" and e.camera not in cache:
            cache[e.camera] = oracle.depth_map(wl.mesh, wl.cameras[e.camera], wl.depth_w, wl.depth_h)
    t2 = time.perf_counter()
    layers = workload.new_layers(wl, rows * wl.W)
    workload.apply_edits(wl, og, layers, edits, cache)
    t3 = time.perf_counter()
    texels = rows * wl.W * len(edits)
    return {
        "value": texels / (t3 - t2), "unit": "edited texels/s", "cores": 1, "kind": "oracle",
        "sample": (f"atlas rows 0-{rows - 1} ({rows * wl.W} texels) x first {len(edits)} edits; "
                   f"geometry band {t1 - t0:.2f} s, {len(cache)} depth maps {t2 - t1:.2f} s, "
                   f"edits {t3 - t2:.2f} s (single thread)"),
    }


def traffic_from_profiles(kernel_key, src_files):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources (else null)."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for s in src_files:
        with open(os.path.join(ROOT, s), "rb") as f:
            h.update(f.read())
    ent = rec.get(kernel_key)
    if not ent or ent.get("source_sha256") != h.hexdigest():
        return None
    return ent.get("bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (--gpus {args.gpus} requested)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2501_14807_amd import uvl
    from paper_2501_14807_amd.model import Model

    torch.cuda.set_device(0)
    uvl.device_check()
    t = time.perf_counter()
    wl, desc = make_workload(args.workload)
    log(f"workload generated in {time.perf_counter() - t:.1f} s: {desc}")
    m = Model.from_workload(wl)
    m.upload_luts(wl.ops)
    N = wl.W * wl.H
    T = Timer(torch)
    for k in range(args.warmup):
        run_step(m, wl, uvl, T)
        torch.cuda.synchronize()
        log(f"warmup step {k + 1}/{args.warmup} done")
    T.on = True
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        run_step(m, wl, uvl, T)
        log(f"timed step {k + 1}/{args.steps} issued")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    T.on = False
    stats = T.stats()
    n_edits = len(wl.edits)
    ms_step = 1e3 * dt / args.steps
    value = n_edits * N * args.steps / dt

    # roofline of the dominant edit kernel (algorithmic bytes: 12 B of
    # positions per texel; lassos also read their depth map once)
    dw, dh = wl.depth_w, wl.depth_h
    per_launch = {"edit_brush": 12.0 * N, "edit_lasso": 12.0 * N + 4.0 * dw * dh}
    kern = max(("edit_brush", "edit_lasso"), key=lambda k: stats.get(k, {"total_ms": 0})["total_ms"])
    avg_s = stats[kern]["avg_us"] * 1e-6
    achieved = per_launch[kern] / avg_s / 1e9
    srcs = ["paper_2501_14807_amd/csrc/edit.hip", "paper_2501_14807_amd/csrc/edit_texel.h"]
    traffic = traffic_from_profiles(kern, srcs)
    kernels = {}
    for k, s in stats.items():
        ent = dict(s)
        if k in per_launch:
            ent["gbps"] = per_launch[k] / (s["avg_us"] * 1e-6) / 1e9
            ent["texels_per_s"] = N / (s["avg_us"] * 1e-6)
        kernels[k] = ent
    layer_bytes = [1 if dt_ == uvl.U8 else 2 for dt_ in wl.layer_dtypes]
    if "area_query" in stats:
        ab = N * (4 + sum(layer_bytes))
        kernels["area_query"]["gbps"] = ab / (stats["area_query"]["avg_us"] * 1e-6) / 1e9
    copy_gbps = copy_bandwidth(torch)
    log(f"device copy bandwidth {copy_gbps:.0f} GB/s")

    out = {
        "metric": "edited texels/s (% HBM peak); batched edits/s + p50/p99 latency vs plain",
        "value": value,
        "unit": "edited texels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded displaced-grid charts and edit streams)",
        "config": {"workload": desc, "atlas": [wl.W, wl.H], "triangles": wl.mesh.nt,
                   "edits_per_step": n_edits, "layer_ops_per_step": len(wl.ops),
                   "depth_map": [dw, dh], "parallelism": "single GPU"},
        "edits_per_s": n_edits * args.steps / dt,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic, "kernel": kern,
                     "bytes_per_launch": per_launch[kern], "avg_us": stats[kern]["avg_us"]},
        "kernels": kernels,
        "copy_gbps": copy_gbps,
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_rows, args.cpu_edits)
        log("oracle sample done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
