"""Serving loop: continuous batching of layer requests over resident models.

The paper's system keeps every layer and the geometry resident on the GPU
and sends only a few bytes per edit (§4: structures live on the GPU; §5,
Fig. 8: 64 bytes per edit); its Texture Manager groups layers into texture
arrays by (width, height, dtype) and commits memory only for the layers that
exist (§4.2).  A server built on that keeps many models resident and serves
a stream of requests -- brush and lasso edits, per-label area queries, layer
operations -- from many clients.

Residency: a model is admitted when a request for it arrives and its HBM
footprint (geometry image, layers, area bins, depth maps, mesh) fits the
budget; its layers are committed in the layer pool (uvl_pool_*).  When it
does not fit, the least recently used resident models with no queued work
are frozen (no new work is launched for them), and once no round in flight
touches them they are evicted: their layers go to host memory and their
pool memory is released.  A re-admitted model rebuilds its geometry image
and gets its layers back, so every request sees the state its model's
earlier requests left.  A model larger than the whole budget is refused.

Ordering: requests of one model take effect in arrival order; requests of
different models are independent.  All device work goes to one stream, so
launch order is execution order.

Batched mode (continuous batching): the scheduler runs rounds.  A round
takes, for every resident model with queued requests, the prefix of its
queue up to the first non-edit request; all those edits go into one wave
launch (uvl_wave_submit), which also keeps each layer's per-label area bins
up to date; then each such model's following area / algebra requests are
launched in order (an area request copies the maintained bins, a layer
operation refreshes its destination's bins).  Up to `max_inflight` rounds
are on the device at once; requests that arrive while rounds run join the
next round.  A round starts at once when the device is idle; with rounds in
flight, the next one waits for `min_batch` queued requests or for its oldest
request to have waited `max_wait_s`, so that a busy device gets fewer,
larger waves.

Plain mode: every request is launched on arrival, one launch per request
(an area request scans its layer).

Texture padding (§4.3.2), when the executor is given a radius: batched
rounds pad inside their waves, plain mode launches each edit's padding after
it; both leave the layers of edit-then-pad in arrival order.

Latency of a request = completion time observed on the host (its round's
event) - arrival time.  The executor is pluggable: GpuExecutor drives the HIP
library; SimExecutor (host only, simulated durations, injectable failures)
drives the same scheduler in tests without a GPU.
"""

from __future__ import annotations

import gc
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

EDIT_KINDS = ("brush", "lasso")


@dataclass
class Request:
    rid: int
    t_arrival: float
    model: int
    kind: str                      # brush | lasso | area | algebra
    edit: object = None            # brush / lasso parameters (synth-style edit)
    op: object = None              # algebra: a LayerOp-like object
    layer: int = 0                 # area: which layer
    t_done: Optional[float] = None
    result: object = None          # area: numpy bins; failures: an error string
    ok: bool = True


@dataclass
class Round:
    handle: object
    requests: List[Request]


# ---------------------------------------------------------------------------
# executors


class Executor:
    """Device work for the server.  launch_* enqueue work in order and return
    nothing; close_round() returns a handle whose completion covers everything
    launched since the previous close_round().  admit() makes a model
    resident (its state as its last eviction left it, or new); evict() saves
    its state to the host and releases its device memory (nothing in flight
    touches it)."""

    def footprint(self, model: int) -> int:
        raise NotImplementedError

    def admit(self, model: int):
        pass

    def evict(self, model: int):
        pass

    def launch_wave(self, reqs: Sequence[Request]):
        raise NotImplementedError

    def launch_single(self, req: Request):
        raise NotImplementedError

    def close_round(self, reqs: Sequence[Request]):
        raise NotImplementedError

    def done(self, handle) -> bool:
        raise NotImplementedError

    def finish(self, handle, reqs: Sequence[Request]):
        """Fill results of completed requests (area bins)."""


class SimExecutor(Executor):
    """Host-only executor with simulated device time (a single in-order
    queue), for testing the scheduler.  `fail_models`: launches touching these
    models fail (their requests complete with ok=False)."""

    def __init__(self, footprints: Sequence[int], edit_s=100e-6, wave_edit_s=10e-6, wave_fixed_s=50e-6,
                 single_s=50e-6, fail_models=()):
        self.fp = list(footprints)
        self.edit_s, self.wave_edit_s, self.wave_fixed_s, self.single_s = edit_s, wave_edit_s, wave_fixed_s, single_s
        self.fail = set(fail_models)
        self.busy_until = 0.0
        self.t0 = time.perf_counter()
        self.pending = 0.0
        self.failed: List[Request] = []
        self.log: List[tuple] = []            # (kind, model, rid) in launch order
        self.state: Dict[int, List[int]] = {}  # model -> applied request ids (survives eviction)
        self.resident = set()
        self.admissions = self.evictions = 0

    def _now(self):
        return time.perf_counter() - self.t0

    def footprint(self, model):
        return self.fp[model]

    def admit(self, model):
        assert model not in self.resident
        self.resident.add(model)
        self.admissions += 1
        self.log.append(("admit", model, -1))

    def evict(self, model):
        assert model in self.resident
        self.resident.discard(model)
        self.evictions += 1
        self.log.append(("evict", model, -1))

    def launch_wave(self, reqs):
        self.pending += self.wave_fixed_s + self.wave_edit_s * len(reqs)
        for r in reqs:
            self._apply(r)

    def launch_single(self, req):
        self.pending += self.edit_s if req.kind in EDIT_KINDS else self.single_s
        self._apply(req)

    def _apply(self, r):
        assert r.model in self.resident, "work launched for a model that is not resident"
        self.log.append((r.kind, r.model, r.rid))
        if r.model in self.fail:
            r.ok = False
            r.result = "injected device error"
            return
        self.state.setdefault(r.model, []).append(r.rid)
        if r.kind == "area":
            r.result = tuple(self.state[r.model])     # what the query saw

    def close_round(self, reqs):
        start = max(self.busy_until, self._now())
        self.busy_until = start + self.pending
        self.pending = 0.0
        return self.busy_until

    def done(self, handle):
        return self._now() >= handle

    def finish(self, handle, reqs):
        pass


@dataclass
class ModelSpec:
    """What the server needs to (re)build a model on admission."""
    mesh: object                    # host mesh (synth.Mesh-like: pos, nrm, uv, tri)
    width: int
    height: int
    layer_dtypes: Sequence[int]
    depth: int = 256                # depth-map side
    bias: float = 1e-4


class GpuExecutor(Executor):
    """The HIP library behind the server: resident models as Model objects
    with their layers in a layer pool, edits through waves (batched) or
    single launches (plain).  keep_bins: the waves keep each layer's area
    bins up to date and area requests copy them (batched serving); otherwise
    an area request scans its layer.  Kept bins are computed lazily: a layer
    is stale from admission or from a layer operation writing it until an
    area request scans it, and the waves update only fresh layers' bins."""

    def __init__(self, specs: Sequence[ModelSpec], cameras, max_wave_edits=4096, pad_k=None, keep_bins=True,
                 pool_slots=256):
        import torch
        from . import uvl
        self.torch, self.uvl = torch, uvl
        self.specs = list(specs)
        self.cameras = cameras                # per model: list of view-proj matrices
        self.pad_k = pad_k                    # texture padding (§4.3.2) after every edit
        self.keep_bins = keep_bins
        self.pool = uvl.LayerPool(pool_slots)
        self.models: Dict[int, object] = {}   # resident Model objects
        self.bins: Dict[int, list] = {}       # per resident model, one device bins tensor per layer
        self.stale: set = set()               # (model, layer) whose kept bins are out of date
        self.depth: Dict[tuple, object] = {}  # (model, camera) -> depth map of a resident model
        self.outlines: Dict[int, object] = {}
        self.saved: Dict[int, list] = {}      # evicted models' layers (host)
        self.wave = uvl.Wave(max_wave_edits, max_wave_edits)
        self.max_wave_edits = max_wave_edits
        self._keep = []                       # host arrays of launched batches until their round ends
        self.admissions = self.evictions = 0

    def footprint(self, model):
        sp, uvl = self.specs[model], self.uvl
        n = sp.width * sp.height
        geom = uvl.lib().uvl_geom_bytes(sp.width, sp.height, 7 | 16)
        layers = sum(n * (1 if dt == uvl.U8 else 2) for dt in sp.layer_dtypes)
        bins = sum(8 * (256 if dt == uvl.U8 else 65536) for dt in sp.layer_dtypes)
        depth = len(self.cameras[model]) * sp.depth * sp.depth * 4
        mesh = sp.mesh.pos.shape[0] * 32 + sp.mesh.tri.shape[0] * 12
        return int(geom + layers + bins + depth + mesh)

    def admit(self, model):
        from .model import Model
        sp, uvl, torch = self.specs[model], self.uvl, self.torch
        m = Model(sp.mesh, sp.width, sp.height, sp.layer_dtypes, depth_w=sp.depth, depth_h=sp.depth, bias=sp.bias,
                  pool=self.pool).build()
        saved = self.saved.pop(model, None)
        if saved is not None:
            for l, a in zip(m.layers, saved):
                l.copy_from(a)
        self.models[model] = m
        wide = 2 if m.geom.wide else 1
        self.bins[model] = [torch.empty(wide * (256 if l.dtype == uvl.U8 else 65536), dtype=torch.int64,
                                        device=m.device) for l in m.layers]
        self.stale.update((model, k) for k in range(len(m.layers)))
        for ci in range(len(self.cameras[model])):
            self._depth(model, ci)
        if self.pad_k is not None:
            self.outlines[model] = uvl.Outline(m.geom, int(self.pad_k))
        self.admissions += 1

    def evict(self, model):
        m = self.models.pop(model)
        self.torch.cuda.synchronize()
        self.saved[model] = [l.numpy().copy() for l in m.layers]
        m.release()                           # pool memory back (waits for the device)
        self.bins.pop(model, None)
        self.stale.difference_update({k for k in self.stale if k[0] == model})
        self.outlines.pop(model, None)
        for key in [k for k in self.depth if k[0] == model]:
            del self.depth[key]
        self.evictions += 1

    def layers_of(self, model):
        """Host copies of a model's layers (resident or saved)."""
        if model in self.models:
            self.torch.cuda.synchronize()
            return [l.numpy().copy() for l in self.models[model].layers]
        return self.saved.get(model)

    def _depth(self, model, cam):
        key = (model, cam)
        d = self.depth.get(key)
        if d is None:
            m = self.models[model]
            d = self.torch.empty((m.depth_h, m.depth_w), dtype=self.torch.float32, device=m.device)
            self.uvl.render_depth(m.mesh, self.cameras[model][cam], d, m.depth_ws)
            self.depth[key] = d
        return d

    def launch_wave(self, reqs):
        batch = self.uvl.EditBatch()
        for r in reqs:
            m, e = self.models[r.model], r.edit
            layer = m.layers[e.layer]
            bins = self.bins[r.model][e.layer] if self.keep_bins and (r.model, e.layer) not in self.stale else None
            if r.kind == "brush":
                batch.brush(m.geom, layer, e.centre, e.radius, e.label, bins=bins)
            else:
                batch.lasso(m.geom, layer, self.cameras[r.model][e.camera], e.poly, self._depth(r.model, e.camera),
                            m.bias, e.label, bins=bins)
        outlines = None
        if self.pad_k is not None:
            outlines = [(self.models[mi].geom, self.outlines[mi]) for mi in sorted({r.model for r in reqs})]
        self.wave.submit(batch, outlines=outlines)
        self._keep.append(batch)

    def launch_single(self, r):
        m = self.models[r.model]
        o = self.outlines.get(r.model)
        if r.kind == "brush":
            e = r.edit
            self.uvl.edit_brush(m.geom, m.layers[e.layer], e.centre, e.radius, e.label)
            if o is not None:
                self.uvl.pad_brush(m.geom, m.layers[e.layer], o, e.centre, e.radius, e.label)
        elif r.kind == "lasso":
            e = r.edit
            M, d = self.cameras[r.model][e.camera], self._depth(r.model, e.camera)
            self.uvl.edit_lasso(m.geom, m.layers[e.layer], M, e.poly, d, m.bias, e.label)
            if o is not None:
                self.uvl.pad_lasso(m.geom, m.layers[e.layer], o, M, e.poly, d, m.bias, e.label)
        elif r.kind == "algebra":
            op = r.op
            b = None if op.op == self.uvl.REMAP else m.layers[op.b]
            self.uvl.layer_op(op.op, m.layers[op.dst], m.layers[op.a], b, op.sel_a, op.sel_b, op.out_label, op.lut)
            if self.keep_bins:
                self.stale.add((r.model, op.dst))
        elif r.kind == "area":
            if self.keep_bins:
                bins = self.bins[r.model][r.layer]
                if (r.model, r.layer) in self.stale:
                    self.uvl.area_query(m.geom, [m.layers[r.layer]], bins=bins, sync=False)
                    self.stale.discard((r.model, r.layer))
            else:
                bins = self.uvl.area_query(m.geom, [m.layers[r.layer]], sync=False)
            host = self.torch.empty(bins.shape, dtype=bins.dtype, pin_memory=True)
            host.copy_(bins, non_blocking=True)
            r.result = (host, m.geom.area_scale)
        else:
            raise ValueError(r.kind)

    def close_round(self, reqs):
        ev = self.torch.cuda.Event()
        ev.record()
        keep, self._keep = self._keep, []
        return (ev, keep)

    def done(self, handle):
        return handle[0].query()

    def finish(self, handle, reqs):
        for r in reqs:
            if r.kind == "area" and isinstance(r.result, tuple):
                host, scale = r.result
                r.result = host.numpy().view(np.uint64).copy()

    def close(self):
        self.torch.cuda.synchronize()
        for mi in list(self.models):
            self.models.pop(mi).release()
        self.wave.close()
        self.pool.close()


# ---------------------------------------------------------------------------
# the server


@dataclass
class Stats:
    mode: str
    n: int
    wall_s: float
    p50_ms: float
    p99_ms: float
    edits_per_s: float
    requests_per_s: float
    rounds: int
    failed: int
    refused: int
    admissions: int = 0
    evictions: int = 0
    latencies_ms: np.ndarray = field(repr=False, default=None)

    def as_dict(self):
        return {"mode": self.mode, "requests": self.n, "wall_s": self.wall_s, "p50_ms": self.p50_ms,
                "p99_ms": self.p99_ms, "edits_per_s": self.edits_per_s, "requests_per_s": self.requests_per_s,
                "rounds": self.rounds, "failed": self.failed, "refused": self.refused,
                "admissions": self.admissions, "evictions": self.evictions}


class Server:
    def __init__(self, executor: Executor, n_models: int, budget_bytes: int, max_wave_edits: int = 4096,
                 max_inflight: int = 2, min_batch: int = 32, max_wait_s: float = 2e-3):
        self.ex = executor
        self.n_models = n_models
        self.budget = int(budget_bytes)
        self.max_wave_edits = max_wave_edits
        self.max_inflight = max_inflight
        # a round starts at once when the device is idle; while rounds are in
        # flight, a further one starts only with min_batch requests queued or
        # once the oldest has waited max_wait_s (small rounds pay the fixed
        # cost of a launch each)
        self.min_batch = min_batch
        self.max_wait_s = max_wait_s
        self.fp = [executor.footprint(m) for m in range(n_models)]
        self.resident: set = set()
        self.used_bytes = 0
        self.last_use: Dict[int, float] = {}
        self.frozen: set = set()              # chosen for eviction: no new work is launched for them

    # -- residency ------------------------------------------------------------
    def admit(self, model: int):
        self.ex.admit(model)
        self.resident.add(model)
        self.used_bytes += self.fp[model]

    def evict(self, model: int):
        self.ex.evict(model)
        self.resident.discard(model)
        self.frozen.discard(model)
        self.used_bytes -= self.fp[model]

    def preload(self, models: Optional[Sequence[int]] = None):
        """Admit models up front (in order, while they fit)."""
        for m in (range(self.n_models) if models is None else models):
            if m not in self.resident and self.used_bytes + self.fp[m] <= self.budget:
                self.admit(m)

    def _residency(self, queues, busy, t):
        """Admit waiting models (oldest request first) as memory allows;
        freeze and evict least recently used idle models to make room."""
        waiting = sorted((q[0].t_arrival, m) for m, q in queues.items() if q and m not in self.resident)
        for _, m in waiting:
            need = self.used_bytes + self.fp[m] - self.budget
            if need <= 0:
                self.admit(m)
                self.last_use[m] = t
                continue
            # victims: resident, nothing queued, least recently used first
            idle = sorted((self.last_use.get(v, -1.0), v) for v in self.resident
                          if not queues.get(v) and v not in self.frozen)
            freed = sum(self.fp[v] for v in self.frozen)
            for _, v in idle:
                if freed >= need:
                    break
                self.frozen.add(v)
                freed += self.fp[v]
            for v in [v for v in self.frozen if v not in busy]:
                self.evict(v)
            if self.used_bytes + self.fp[m] <= self.budget:
                self.admit(m)
                self.last_use[m] = t
            else:
                break                          # wait for frozen models to leave the device

    # -- serving ----------------------------------------------------------------
    def run(self, requests: Sequence[Request], mode: str = "batched", spin_s: float = 20e-6,
            warmup: int = 0) -> Stats:
        """Serve `requests` (arrival times in seconds from now).  The first
        `warmup` requests (in arrival order) are served but left out of the
        statistics, whose time span then starts at the first measured
        arrival.  Python's cyclic garbage collector is paused meanwhile: its
        pauses land in the latency tail."""
        assert mode in ("batched", "plain")
        was = gc.isenabled()
        gc.disable()
        try:
            return self._run(requests, mode, spin_s, warmup)
        finally:
            if was:
                gc.enable()

    def _run(self, requests, mode, spin_s, warmup=0) -> Stats:
        reqs = sorted(requests, key=lambda r: (r.t_arrival, r.rid))
        queues: Dict[int, deque] = {}
        inflight: deque = deque()
        busy: Dict[int, int] = {}              # model -> rounds in flight touching it
        nxt = 0
        rounds = 0
        refused = 0
        adm0, ev0 = getattr(self.ex, "admissions", 0), getattr(self.ex, "evictions", 0)
        t0 = time.perf_counter()
        n = len(reqs)
        completed = 0
        nq = 0                                  # queued requests of resident, unfrozen models

        def now():
            return time.perf_counter() - t0

        def runnable(m):
            return m in self.resident and m not in self.frozen

        while completed < n:
            t = now()
            # arrivals
            while nxt < n and reqs[nxt].t_arrival <= t:
                r = reqs[nxt]
                nxt += 1
                if self.fp[r.model] > self.budget:
                    r.ok, r.result, r.t_done = False, "model larger than the budget", t
                    refused += 1
                    completed += 1
                    continue
                queues.setdefault(r.model, deque()).append(r)
            # completions (in order: one in-order device queue)
            while inflight and self.ex.done(inflight[0].handle):
                rd = inflight.popleft()
                self.ex.finish(rd.handle, rd.requests)
                tt = now()
                for r in rd.requests:
                    r.t_done = tt
                for m in {r.model for r in rd.requests}:
                    busy[m] -= 1
                    if not busy[m]:
                        del busy[m]
                completed += len(rd.requests)
            # residency: admit waiting models, evict idle ones to make room
            if any(q and m not in self.resident for m, q in queues.items()) or self.frozen:
                self._residency(queues, busy, t)
            nq = sum(len(q) for m, q in queues.items() if runnable(m))
            # launch a round if a slot is free (see min_batch / max_wait_s)
            if nq and len(inflight) < self.max_inflight:
                go = not inflight or mode == "plain" or nq >= self.min_batch
                if not go:
                    oldest = min(q[0].t_arrival for m, q in queues.items() if q and runnable(m))
                    go = now() - oldest >= self.max_wait_s
                if go:
                    launched = self._round(queues, mode, runnable)
                    rounds += 1
                    for m in {r.model for r in launched}:
                        busy[m] = busy.get(m, 0) + 1
                        self.last_use[m] = t
                    inflight.append(Round(self.ex.close_round(launched), launched))
                    continue
            if spin_s > 0:
                time.sleep(spin_s)
        meas = reqs[warmup:] if warmup < n else []
        wall = now() - (meas[0].t_arrival if meas and warmup else 0.0)
        lat = np.array([(r.t_done - r.t_arrival) * 1e3 for r in meas if r.ok], dtype=np.float64)
        edits = sum(1 for r in meas if r.ok and r.kind in EDIT_KINDS)
        nm = len(meas)
        return Stats(mode, nm, wall, float(np.percentile(lat, 50)) if lat.size else float("nan"),
                     float(np.percentile(lat, 99)) if lat.size else float("nan"), edits / wall, nm / wall, rounds,
                     sum(1 for r in reqs if not r.ok) - refused, refused,
                     getattr(self.ex, "admissions", 0) - adm0, getattr(self.ex, "evictions", 0) - ev0, lat)

    def _round(self, queues, mode, runnable) -> List[Request]:
        launched: List[Request] = []
        if mode == "plain":
            # every queued request of a runnable model, one launch each, in
            # arrival order
            allq = sorted((r for m, q in queues.items() if runnable(m) for r in q),
                          key=lambda r: (r.t_arrival, r.rid))
            for m in list(queues.keys()):
                if runnable(m):
                    del queues[m]
            for r in allq:
                self.ex.launch_single(r)
                launched.append(r)
            return launched
        # batched: per model, the prefix of edits up to the first non-edit
        wave: List[Request] = []
        tails: List[List[Request]] = []
        for m in list(queues.keys()):
            if not runnable(m):
                continue
            q = queues[m]
            while q and q[0].kind in EDIT_KINDS and len(wave) < self.max_wave_edits:
                wave.append(q.popleft())
            tail = []
            while q and q[0].kind not in EDIT_KINDS:
                tail.append(q.popleft())
            if tail:
                tails.append(tail)
            if not q:
                del queues[m]
        if wave:
            self.ex.launch_wave(wave)
            launched.extend(wave)
        for tail in tails:
            for r in tail:
                self.ex.launch_single(r)
                launched.append(r)
        return launched
