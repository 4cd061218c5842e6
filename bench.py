"""Benchmark of the texture-layer hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload scan|max|tiny] [--no-cpu-baseline]

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

Beside the step, untimed by the step's clock and reported in their own
fields: the paper's screen-space tool, texture padding and numeric layers
(a value lasso, zonal statistics, range selection) on the same model, the
batched-wave comparison (256 models of uneven size, one launch per edit
against one wave) and the serving comparison (32 + 32 resident models,
Poisson requests swept over rates, p50/p99 and edits/s, plain against
continuous batching), then the oracle on a bounded sample (`cpu_baseline`:
one process per host core, up to 16, each on its own band of atlas rows,
beside the single-thread figure).

`--workload max` runs the same step on the 16384^2 model (8,258,048
triangles, 32 u8 layers, 10,000 edits, 80 operations) and then applies its
edits again as waves of 256.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz (one
# non-packed operation per lane per clock) = 39.3e12 lane-operations/s, i.e.
# 614e9 wave64 instructions/s
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
HOST_CORE_CAP = 16          # the GPU machine's host share for one GPU


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="scan", choices=["scan", "tiny", "max"],
                   help="scan: the 8192^2 scan-scale model (default); max: the 16384^2 model, 10,000 edits, "
                        "also applied as waves of 256; tiny: the vessel")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-rows", type=int, default=64, help="atlas rows in the oracle's timed sample")
    p.add_argument("--cpu-edits", type=int, default=None,
                   help="edits in the oracle's timed sample (default 200; 100 for --workload max)")
    p.add_argument("--batch-models", type=int, default=256,
                   help="models in the batched-wave comparison (0: skip it)")
    p.add_argument("--serve-models", type=int, default=32,
                   help="small + scan-scale models each in the serving comparison (0: skip it)")
    p.add_argument("--serve-requests", type=int, default=100000, help="measured requests per rate")
    p.add_argument("--serve-warmup", type=int, default=5000, help="warm-up requests per rate")
    p.add_argument("--serve-slo-ms", type=float, default=10.0, help="the p99 bound both modes are compared at")
    p.add_argument("--serve-rates", default=None,
                   help="comma-separated offered rates (requests/s) instead of the default sweep")
    p.add_argument("--serve-modes", default="plain,batched", help="serving modes to run (plain, batched)")
    return p.parse_args()


def make_workload(name):
    import synth
    if name == "tiny":
        return synth.tiny_workload(), "vessel 128^2 vertices (32,258 tris), 512^2 atlas, 1 u8 layer, 64 edits"
    if name == "max":
        return synth.max_workload(), ("max model: 256 displaced 128x128 charts (8,258,048 tris), 16384^2 atlas, "
                                      "32 u8 layers, 5000 brush + 5000 lasso (2048^2 depth) + 80 layer ops + "
                                      "per-label area (one fused pass per 8 layers)")
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


def area_needed_bytes(m, uvl, torch):
    """Bytes a fused area query over all of m's layers must read: every
    label and every texel's weight (4 B); a query of at most two layers on
    a geometry image with per-block area sums (8 B per block of 4 rows x 8
    columns) reads the weights only of the blocks whose labels differ within
    the block in some layer, the sums of the others."""
    W, H = m.geom.width, m.geom.height
    N = W * H
    labels = float(sum(N * (1 if l.dtype == uvl.U8 else 2) for l in m.layers))
    if m.geom.area_blk is None or len(m.layers) > 2 or W % 8 or H % 4:
        return labels + 4.0 * N
    mixed = None
    for l in m.layers:
        a = l.data[:N].view(H // 4, 4, W // 8, 8)
        u = (a == a[:, :1, :, :1]).all(dim=3).all(dim=1)
        mixed = ~u if mixed is None else (mixed | ~u)
    nmixed = int(mixed.sum().item())
    return labels + 8.0 * (N // 32) + 4.0 * 32 * nmixed


def bench_batched(n_models, reps, torch, uvl):
    """Batched waves against the plain path on many models of uneven size.

    256 models (triangles log-uniform in 1e4..1e6, atlases 1024^2..8192^2,
    one u8 layer each) with 1..64 pending edits each, half brushes, half
    lassos (one camera per 8 lassos, 1024^2 depth maps).  Plain: one launch
    per edit, depth maps rendered as the camera changes.  Batched: the same
    depth maps, then one wave launch for all edits of all models.  Both start
    from cleared layers and must end with identical layers.
    """
    import synth
    from paper_2501_14807_amd.model import Model
    t = time.perf_counter()
    wls = synth.batch_workload(n_models=n_models)
    log(f"batch workload generated in {time.perf_counter() - t:.1f} s")
    models = []
    for k, w in enumerate(wls):
        models.append(Model.from_workload(w, normals=False, bary=False).build())
        if (k + 1) % 32 == 0:
            log(f"batch models built: {k + 1}/{len(wls)}")
    n_edits = sum(len(w.edits) for w in wls)
    n_lassos = sum(1 for w in wls for e in w.edits if e.kind == "lasso")
    texels = sum(w.W * w.H for w in wls)
    batch = uvl.EditBatch()
    maps = [m.add_to_batch(batch, w.edits, w.cameras, render=False) for m, w in zip(models, wls)]
    wave = uvl.Wave(max(1, n_edits), max(1, n_lassos))
    for m, w, mp in zip(models, wls, maps):
        m.clear_layers()
        m.render_maps(mp, w.cameras)
    wave.tune(batch)
    tuned = {int(side): wave.tuned_chunks(side * side) for side in sorted({w.W for w in wls})}
    torch.cuda.synchronize()

    def plain():
        for m, w in zip(models, wls):
            m.clear_layers()
            m.apply_all(w.edits, w.cameras)

    def batched():
        for m, w, mp in zip(models, wls, maps):
            m.clear_layers()
            m.render_maps(mp, w.cameras)
        wave.submit(batch)

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) / 1e3)
        return best

    t_plain = timed(plain)
    ref = [m.layers[0].data[:m.layers[0].n].clone() for m in models]
    t_wave = timed(batched)
    same = all(torch.equal(m.layers[0].data[:m.layers[0].n], r) for m, r in zip(models, ref))
    # the wave kernel alone (depth maps already rendered)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    wave.submit(batch)
    e1.record()
    torch.cuda.synchronize()
    t_kernel = e0.elapsed_time(e1) / 1e3
    wave.close()
    log(f"batched: plain {t_plain * 1e3:.1f} ms, wave pass {t_wave * 1e3:.1f} ms, identical={same}")
    return {
        "workload": f"{n_models} models, triangles log-uniform 1e4-1e6, atlases 1024^2-8192^2 "
                    f"({texels / 1e9:.2f} G texels), 1-64 edits each, 1024^2 depth maps",
        "edits": n_edits, "lassos": n_lassos,
        "plain_edits_per_s": n_edits / t_plain, "batched_edits_per_s": n_edits / t_wave,
        "speedup": t_plain / t_wave, "plain_ms": t_plain * 1e3, "batched_ms": t_wave * 1e3,
        "wave_launch_ms": t_kernel * 1e3, "identical_layers": bool(same), "tuned_chunks": tuned,
    }


# offered request rates of the serving sweep (requests/s); a mode's sweep
# stops once its p99 passes SERVE_SATURATED_MS (higher rates only queue more)
SERVE_RATES = (12000.0, 13000.0, 14000.0, 15000.0, 16000.0, 24000.0, 40000.0, 48000.0, 52000.0, 56000.0, 60000.0,
               64000.0, 66000.0, 68000.0, 70000.0, 72000.0, 76000.0, 80000.0)
SERVE_SATURATED_MS = 200.0
SERVE_SLOS_MS = (5.0, 10.0, 20.0)


def bench_serving(n_each, n_requests, slo_ms, torch, uvl, warmup=5000, rates=SERVE_RATES,
                  modes=("plain", "batched")):
    """Continuous batching against plain one-launch-per-request serving.

    n_each vessel-size models (512^2) and n_each scan-scale models (8192^2,
    4,145,280 triangles), each with a u8 and a u16 layer, admitted up front
    within a 200 GB budget (their layers in the layer pool); Poisson
    arrivals, 60% brush / 25% lasso / 10% area / 5% layer operation, uniform
    model choice; a sweep of arrival rates, each run serving `warmup`
    requests first and measuring the next n_requests.  For each mode and
    p99 bound, the highest edits/s reached with p99 latency within it.
    """
    import synth
    from paper_2501_14807_amd.serve import GpuExecutor, ModelSpec, Request, Server
    t = time.perf_counter()
    meshes, sizes, depth = [], [], []
    for k in range(n_each):
        meshes.append(synth.vessel(seed=100 + k))
        sizes.append(512)
        depth.append(256)
    for k in range(n_each):
        meshes.append(synth.scan_mesh(seed=1100 + k)[0])
        sizes.append(8192)
        depth.append(1024)
        if (k + 1) % 8 == 0:
            log(f"serving: {k + 1}/{n_each} scan-scale meshes generated")
    dtypes = [[uvl.U8, uvl.U16]] * len(meshes)
    specs = [ModelSpec(m, s_, s_, dt, depth=d) for m, s_, dt, d in zip(meshes, sizes, dtypes, depth)]
    log(f"serving: {len(specs)} model specs after {time.perf_counter() - t:.1f} s")
    sweep = []
    done = {m: m not in modes for m in ("plain", "batched")}
    for qps in rates:
        if all(done.values()):
            break
        cams, stream = synth.serve_stream(meshes, dtypes, warmup + n_requests, qps, seed=int(qps))
        row = {"qps": qps}
        for mode in ("plain", "batched"):
            if done[mode]:
                continue
            t1 = time.perf_counter()
            ex = GpuExecutor(specs, cams, max_wave_edits=8192, keep_bins=(mode == "batched"))
            srv = Server(ex, len(specs), 200 << 30)
            srv.preload()
            torch.cuda.synchronize()
            log(f"serving qps {qps:.0f} {mode}: {len(srv.resident)} models admitted in "
                f"{time.perf_counter() - t1:.1f} s, serving {warmup} + {n_requests} requests")
            reqs = [Request(i, d["t"], d["model"], d["kind"], edit=d.get("edit"), op=d.get("op"),
                            layer=d.get("layer", 0)) for i, d in enumerate(stream)]
            st = srv.run(reqs, mode, warmup=warmup)
            torch.cuda.synchronize()
            ex.close()
            row[mode] = st.as_dict()
            done[mode] = st.p99_ms > SERVE_SATURATED_MS
            log(f"serving qps {qps:.0f} {mode}: p50 {st.p50_ms:.2f} ms p99 {st.p99_ms:.2f} ms "
                f"{st.edits_per_s:.0f} edits/s ({st.rounds} rounds)")
        sweep.append(row)

    def best(mode, bound):
        ok = [r[mode]["edits_per_s"] for r in sweep if mode in r and r[mode]["p99_ms"] <= bound]
        return max(ok) if ok else None

    at = {}
    for bound in sorted(set(SERVE_SLOS_MS) | {slo_ms}):
        bp, bb = best("plain", bound), best("batched", bound)
        at[f"{bound:g}"] = {"plain_edits_per_s": bp, "batched_edits_per_s": bb,
                            "ratio": (bb / bp) if bp and bb else None}
    return {"workload": f"{n_each} vessel-size (512^2) + {n_each} scan-scale (8192^2) models, u8+u16 layers, "
                        f"{warmup} warm-up + {n_requests} measured Poisson requests per rate, "
                        f"60/25/10/5 brush/lasso/area/op; batched area answers from wave-maintained bins (a layer written by an op "
                        f"is rescanned at its next area request)",
            "sweep": sweep, "slo_p99_ms": slo_ms, "at_p99_bound_ms": at,
            "plain_edits_per_s_at_slo": at[f"{slo_ms:g}"]["plain_edits_per_s"],
            "batched_edits_per_s_at_slo": at[f"{slo_ms:g}"]["batched_edits_per_s"],
            "ratio_at_slo": at[f"{slo_ms:g}"]["ratio"]}


def bench_tool(m, wl, uvl, torch, n_edits=100):
    """The paper's screen-space tool (§4.3.1) on the workload's model: a
    200-pixel disk tool at seeded positions on a window the size of the
    depth maps, with the workload's cameras; per-launch time and the
    position bytes it streams (12 per texel)."""
    rng = np.random.default_rng(5001)
    shape = uvl.disk_shape(256)
    Ww, Wh = wl.depth_w, wl.depth_h
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for k in range(n_edits):
        cam = int(rng.integers(0, len(wl.cameras)))
        M = wl.cameras[cam]
        d = m.depth_for(cam, M)
        tool = (Ww, Wh, float(rng.uniform(0.2, 0.8) * Ww), float(rng.uniform(0.2, 0.8) * Wh), 200.0, 200.0)
        lay = m.layers[k % len(m.layers)]
        fn = lambda: uvl.edit_tool(m.geom, lay, M, tool, shape, d, m.bias, 1 + k % 200)
        fn()
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e3)
    us = float(np.mean(ts))
    N = wl.W * wl.H
    return {"edits": n_edits, "tool_px": 200, "window": [Ww, Wh], "tool_us": us, "texels_per_s": N / (us * 1e-6),
            "gbps": 12.0 * N / (us * 1e-6) / 1e9}


def bench_padding(m, wl, uvl, torch, n_edits=200):
    """Texture padding (§4.3.2) on the workload's model: the outline list
    (radius 1, built once per model), the padding pass after each of the
    first n_edits edits (the paper's per-edit cost is editing + padding), and
    those edits as one wave without and with its padding."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    o = uvl.Outline(m.geom, 1)
    build_ms = 1e3 * (time.perf_counter() - t)
    per = {"brush": [], "lasso": []}
    for e in wl.edits[:n_edits]:
        lay = m.layers[e.layer]
        if e.kind == "brush":
            fn = lambda: uvl.pad_brush(m.geom, lay, o, e.centre, e.radius, e.label)
        else:
            M = wl.cameras[e.camera]
            d = m.depth_for(e.camera, M)
            fn = lambda: uvl.pad_lasso(m.geom, lay, o, M, e.poly, d, m.bias, e.label)
        fn()
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        per[e.kind].append(e0.elapsed_time(e1) * 1e3)
    # the same edits as one wave, without and with its padding
    wave = uvl.Wave(n_edits, n_edits)
    batch = uvl.EditBatch(n_edits)
    m.add_to_batch(batch, wl.edits[:n_edits], wl.cameras)
    wave_ms = {}
    for name, outlines in (("plain", None), ("padded", [(m.geom, o)])):
        wave.submit(batch, outlines=outlines)
        e0.record()
        wave.submit(batch, outlines=outlines)
        e1.record()
        torch.cuda.synchronize()
        wave_ms[name] = e0.elapsed_time(e1)
    wave.close()
    return {"outline_texels": o.n, "outline_build_ms": build_ms, "edits": n_edits,
            "pad_brush_us": float(np.mean(per["brush"])) if per["brush"] else None,
            "pad_lasso_us": float(np.mean(per["lasso"])) if per["lasso"] else None,
            "wave_ms": wave_ms["plain"], "padded_wave_ms": wave_ms["padded"]}


def bench_numeric(m, wl, uvl, torch, n_edits=100, reps=10):
    """Numeric layers (§4.2) on the workload's model: a binary32 layer with a
    validity mask.  Per-launch time of a lasso that SETs a value (next to the
    same lasso on a label layer), of zonal statistics (no region, the u8
    and u16 label layers as regions) and of a range selection, with the
    bytes each streams: statistics read tri_id, area_w and the data (4
    bytes each per texel), the mask (1/8) and the region (1 or 2); the
    selection reads the data and the mask."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, k=1):
        fn()
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / k

    N = wl.W * wl.H
    L = uvl.numeric_create(uvl.NumericLayer(wl.W, wl.H, uvl.F32))
    lab = uvl.create_layer(uvl.Layer(wl.W, wl.H, uvl.U8))
    t_num, t_lab = [], []
    for i, e in enumerate([e for e in wl.edits if e.kind == "lasso"][:n_edits]):
        M = wl.cameras[e.camera]
        d = m.depth_for(e.camera, M)
        t_num.append(timed(lambda: uvl.numeric_lasso(m.geom, L, M, e.poly, d, m.bias, uvl.SET, 0.5 + i)))
        t_lab.append(timed(lambda: uvl.edit_lasso(m.geom, lab, M, e.poly, d, m.bias, 1 + i % 200)))
    rng = np.random.default_rng(6001)
    L.copy_from(rng.normal(0.0, 1.0, N).astype(np.float32), rng.random(N) < 0.9)
    bins = torch.empty(65536 * uvl.NUMSTAT.itemsize, dtype=torch.uint8, device="cuda")
    stats = {}
    regions = [("none", None, 0)] + [(("u8" if l.dtype == uvl.U8 else "u16"), l, 1 if l.dtype == uvl.U8 else 2)
                                     for l in m.layers]
    for name, reg, rb in regions:
        if name in stats:
            continue
        us = timed(lambda: uvl.numeric_stats(m.geom, L, reg, bins, host=False), reps)
        stats[name] = {"us": us, "gbps": N * (12.125 + rb) / (us * 1e-6) / 1e9}
    sel_us = timed(lambda: uvl.numeric_select(L, -0.5, 0.5, lab, 7), reps)
    return {"dtype": "f32", "lasso_edits": len(t_num), "lasso_set_us": float(np.mean(t_num)),
            "label_lasso_us": float(np.mean(t_lab)), "stats": stats,
            "select_us": sel_us, "select_gbps": N * 4.125 / (sel_us * 1e-6) / 1e9}


def bench_radius(m, wl, uvl, torch, reps=20):
    """Brush time against radius (the paper's edit cost does not depend on
    the tool size): one centre from the workload, radii 0.01 .. 0.2."""
    e = next(x for x in wl.edits if x.kind == "brush")
    lay = m.layers[e.layer]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = []
    for r in (0.01, 0.02, 0.05, 0.1, 0.2):
        uvl.edit_brush(m.geom, lay, e.centre, r, 1)
        e0.record()
        for _ in range(reps):
            uvl.edit_brush(m.geom, lay, e.centre, r, 1)
        e1.record()
        torch.cuda.synchronize()
        out.append({"radius": r, "us": e0.elapsed_time(e1) * 1e3 / reps})
    us = [x["us"] for x in out]
    return {"sweep": out, "max_over_min": max(us) / min(us)}


def bench_max_waves(m, wl, uvl, torch, per_wave=256):
    """The max model's edits again as waves of `per_wave` edits (one launch
    each), against the layers of the timed plain step (edits, then layer
    operations)."""
    ref = [l.numpy().copy() for l in m.layers]
    for l in m.layers:
        uvl.create_layer(l)
    wave = uvl.Wave(per_wave, per_wave, max_cull_words=1 << 24)
    batches = []
    for i in range(0, len(wl.edits), per_wave):
        b = uvl.EditBatch(per_wave)
        m.add_to_batch(b, wl.edits[i:i + per_wave], wl.cameras)
        batches.append(b)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for b in batches:
        wave.submit(b)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t)
    for o in wl.ops:          # the step's layer operations, untimed, before comparing
        m.apply_op(o)
    same = all(np.array_equal(l.numpy(), r) for l, r in zip(m.layers, ref))
    wave.close()
    return {"edits": len(wl.edits), "per_wave": per_wave, "waves": len(batches), "ms": ms,
            "edits_per_s": len(wl.edits) / (ms * 1e-3), "identical_to_plain": same,
            "note": "edits only (depth maps rendered before timing); compared after the step's layer operations"}


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


def _oracle_band(args):
    """One worker of the all-cores oracle timing (its own process, no GPU):
    the geometry band and depth maps untimed, then the timed edits."""
    wl_name, r0, rows, n_edits, barrier = args
    import oracle
    from oracle import workload
    wl, _ = make_workload(wl_name)
    edits = wl.edits[:n_edits]
    og = oracle.geometry_image(wl.mesh, wl.W, wl.H, rows=(r0, r0 + rows))
    cache = {}
    for e in edits:
        if e.kind == "lasso" and e.camera not in cache:
            cache[e.camera] = oracle.depth_map(wl.mesh, wl.cameras[e.camera], wl.depth_w, wl.depth_h)
    layers = workload.new_layers(wl, rows * wl.W)
    barrier.wait()
    t = time.perf_counter()
    workload.apply_edits(wl, og, layers, edits, cache)
    return time.perf_counter() - t


def cpu_baseline(wl, wl_name, rows, n_edits):
    """The oracle, as it stands, on a bounded sample of the same workload:
    one thread, then one process per host core (up to 16) on disjoint bands
    of `rows` atlas rows each with the same edits, timed from a common start."""
    import multiprocessing as mp

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
    single = texels / (t3 - t2)
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    procs = max(1, min(HOST_CORE_CAP, avail, wl.H // rows))
    ctx = mp.get_context("spawn")           # fresh interpreters: nothing inherited from the GPU process
    with ctx.Manager() as mgr:
        barrier = mgr.Barrier(procs + 1)
        with ctx.Pool(procs) as pool:
            res = pool.map_async(_oracle_band, [(wl_name, k * rows, rows, n_edits, barrier) for k in range(procs)])
            barrier.wait()
            ta = time.perf_counter()
            res.get()
            wall = time.perf_counter() - ta
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    value = procs * texels / wall
    return {
        "value": value, "unit": "edited texels/s", "cores": procs, "kind": "oracle",
        "single_thread_value": single,
        "host": {"nproc": os.cpu_count(), "affinity_cpus": avail, "cpu_model": model,
                 "process_cap": HOST_CORE_CAP},
        # the step's edits over the whole atlas at the sampled rate
        "extrapolated_step_edits_s": len(wl.edits) * wl.W * wl.H / value,
        "sample": (f"{procs} processes (one per host core, at most {HOST_CORE_CAP}: the box's share for one GPU), "
                   f"each atlas rows of its own {rows}-row band ({rows * wl.W} texels) x the "
                   f"first {len(edits)} edits, wall time from a common start; single thread on rows 0-{rows - 1}: "
                   f"geometry band {t1 - t0:.2f} s, {len(cache)} depth maps {t2 - t1:.2f} s, "
                   f"edits {t3 - t2:.2f} s"),
    }


def counters_from_profiles(kernel_key, src_files):
    """Per-launch counter figures of a kernel from the committed rocprofv3
    summary (HBM bytes from FETCH_SIZE / WRITE_SIZE, VALU wave instructions
    from SQ_INSTS_VALU), if it was taken on the current kernel sources (else
    null)."""
    path = os.path.join(ROOT, "profiles", "pmc_counters.json")
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
    return ent


def headline_roofline(kernel, rl):
    """The contract's roofline object for the dominant kernel: against HBM,
    or against the VALU issue peak when the measured instruction count
    bounds it more tightly (both fractions kept)."""
    out = {"kernel": kernel, "bytes_per_launch": rl["bytes_per_launch"], "avg_us": rl["avg_us"],
           "traffic": rl["traffic"], "hbm_frac": rl["frac"], "valu_frac": rl["valu_frac"]}
    if rl["bound"] == "alu":
        achieved = rl["valu_frac"] * VALU_PEAK_LANE_OPS / 1e12
        out.update({"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_LANE_OPS / 1e12,
                    "unit": "T VALU lane-ops/s", "frac": rl["valu_frac"]})
    else:
        out.update({"bound": "hbm", "achieved": rl["achieved"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": rl["frac"]})
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (--gpus {args.gpus} requested)",
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

    # algorithmic bytes per launch (what the method must move):
    #   brush: 12 B of positions per texel; lasso: the same plus its depth
    #   map once; layer operation: the operands and the destination per
    #   texel (REMAP: one operand); area: every layer's label per texel, the
    #   per-block area sums and the 4 B weights of the blocks whose labels
    #   are not all equal in some layer (area_needed_bytes); geometry image: 40 B of planes per texel (tri_id,
    #   position, normal, barycentrics, area), the tile bounds, and the mesh
    #   (positions, normals, uv per vertex, indices per triangle); depth map:
    #   4 B per pixel written and the mesh's positions and indices read
    dw, dh = wl.depth_w, wl.depth_h
    lb = [1 if dt_ == uvl.U8 else 2 for dt_ in wl.layer_dtypes]
    nv, nt = wl.mesh.pos.shape[0], wl.mesh.tri.shape[0]
    tiles = -(-wl.W // 32) * -(-wl.H // 32)
    op_bytes = [N * (lb[o.a] + lb[o.dst] + (0 if o.op == uvl.REMAP else lb[o.b])) for o in wl.ops]
    per_launch = {
        "edit_brush": 12.0 * N,
        "edit_lasso": 12.0 * N + 4.0 * dw * dh,
        "layer_op": float(sum(op_bytes)) / max(1, len(op_bytes)),
        "area_query": area_needed_bytes(m, uvl, torch),
        "build_geometry_image": 40.0 * N + 24.0 * tiles + 32.0 * nv + 12.0 * nt,
        "render_depth": 4.0 * dw * dh + 12.0 * nv + 12.0 * nt,
    }
    edit_src = ["paper_2501_14807_amd/csrc/edit.hip", "paper_2501_14807_amd/csrc/edit_texel.h",
                "paper_2501_14807_amd/csrc/sink.h"]
    # the committed counter summaries were taken on the scan-scale workload
    counters = {k: counters_from_profiles(k, edit_src) if args.workload == "scan" else None
                for k in ("edit_brush", "edit_lasso")}
    rooflines, kernels = {}, {}
    for k, st in stats.items():
        ent = dict(st)
        if k in per_launch:
            avg_s = st["avg_us"] * 1e-6
            gbps = per_launch[k] / avg_s / 1e9
            ent["gbps"] = gbps
            if k.startswith("edit_"):
                ent["texels_per_s"] = N / avg_s
            rl = {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                  "frac": gbps / HBM_PEAK_GBPS, "bytes_per_launch": per_launch[k], "avg_us": st["avg_us"],
                  "traffic": None, "valu_frac": None}
            c = counters.get(k)
            if c:
                rl["traffic"] = c.get("bytes_per_launch")
                if c.get("valu_insts_per_launch"):
                    # measured VALU wave instructions per launch against the issue peak
                    rl["valu_frac"] = c["valu_insts_per_launch"] * 64 / avg_s / VALU_PEAK_LANE_OPS
                    if rl["valu_frac"] > rl["frac"]:
                        rl["bound"] = "alu"
            rooflines[k] = rl
        kernels[k] = ent
    kern = max(("edit_brush", "edit_lasso"), key=lambda k: stats.get(k, {"total_ms": 0})["total_ms"])
    tool = padding = numeric = radius = max_waves = None
    if args.workload == "max":
        max_waves = bench_max_waves(m, wl, uvl, torch)
        log(f"max model as waves of 256: {max_waves['ms']:.1f} ms for {max_waves['edits']} edits "
            f"(identical: {max_waves['identical_to_plain']})")
    else:
        tool = bench_tool(m, wl, uvl, torch)
        log(f"screen-space tool: {tool['tool_us']:.1f} us per edit ({tool['gbps']:.0f} GB/s)")
        # the statistics group by the model's label layers as the step and the
        # tool left them (the padding section rewrites them with a wave)
        numeric = bench_numeric(m, wl, uvl, torch)
        log(f"numeric f32: lasso SET {numeric['lasso_set_us']:.1f} us (label {numeric['label_lasso_us']:.1f} us), "
            + ", ".join(f"stats[{k}] {v['us']:.1f} us {v['gbps']:.0f} GB/s" for k, v in numeric["stats"].items())
            + f", select {numeric['select_us']:.1f} us")
        padding = bench_padding(m, wl, uvl, torch)
        log(f"padding: {padding['outline_texels']} outline texels, brush {padding['pad_brush_us']:.1f} us, "
            f"lasso {padding['pad_lasso_us']:.1f} us per edit; a {padding['edits']}-edit wave "
            f"{padding['wave_ms']:.2f} ms, padded {padding['padded_wave_ms']:.2f} ms")
        radius = bench_radius(m, wl, uvl, torch)
        log("brush time by radius: " + ", ".join(f"{x['radius']}: {x['us']:.1f} us" for x in radius["sweep"]))
    copy_gbps = copy_bandwidth(torch)
    log(f"device copy bandwidth {copy_gbps:.0f} GB/s")
    batched = None
    if args.batch_models > 0 and args.workload != "max":
        del m
        torch.cuda.empty_cache()
        batched = bench_batched(args.batch_models, 2, torch, uvl)
        torch.cuda.empty_cache()
    serving = None
    if args.serve_models > 0 and args.workload != "max":
        rates = SERVE_RATES if not args.serve_rates else tuple(float(x) for x in args.serve_rates.split(","))
        serving = bench_serving(args.serve_models, args.serve_requests, args.serve_slo_ms, torch, uvl,
                                warmup=args.serve_warmup, rates=rates, modes=tuple(args.serve_modes.split(",")))

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
        "roofline": headline_roofline(kern, rooflines[kern]),
        "rooflines": rooflines,
        "kernels": kernels,
        "copy_gbps": copy_gbps,
        "tool": tool,
        "padding": padding,
        "numeric": numeric,
        "radius_sweep": radius,
        "max_waves": max_waves,
        "batched": batched,
        "serving": serving,
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample ...")
        n_cpu = args.cpu_edits if args.cpu_edits is not None else (100 if args.workload == "max" else 200)
        out["cpu_baseline"] = cpu_baseline(wl, args.workload, args.cpu_rows, n_cpu)
        log("oracle sample done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
