"""Serving loop: continuous batching of layer requests over resident models.

The paper's system keeps every layer and the geometry resident on the GPU
and sends only a few bytes per edit (§4: structures live on the GPU; §5,
Fig. 8: 64 bytes per edit).  A server built on that keeps many models
resident (admitted by HBM footprint within a budget) and serves a stream of
requests -- brush and lasso edits, per-label area queries, layer operations
-- from many clients.

Ordering: requests of one model take effect in arrival order; requests of
different models are independent.  All device work goes to one stream, so
launch order is execution order.

Batched mode (continuous batching): the scheduler runs rounds.  A round
takes, for every model with queued requests, the prefix of its queue up to
the first non-edit request; all those edits go into one wave launch
(uvl_wave_submit); then each such model's following area / algebra requests
are launched in order.  Up to `max_inflight` rounds are on the device at
once; requests that arrive while rounds run join the next round.  A round
starts at once when the device is idle; with rounds in flight, the next one
waits for `min_batch` queued requests or for its oldest request to have
waited `max_wait_s`, so that a busy device gets fewer, larger waves.

Plain mode: every request is launched on arrival, one launch per request.

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
    launched since the previous close_round()."""

    def footprint(self, model: int) -> int:
        raise NotImplementedError

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
        self.state: Dict[int, List[int]] = {}  # model -> applied request ids

    def _now(self):
        return time.perf_counter() - self.t0

    def footprint(self, model):
        return self.fp[model]

    def launch_wave(self, reqs):
        self.pending += self.wave_fixed_s + self.wave_edit_s * len(reqs)
        for r in reqs:
            self._apply(r)

    def launch_single(self, req):
        self.pending += self.edit_s if req.kind in EDIT_KINDS else self.single_s
        self._apply(req)

    def _apply(self, r):
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


class GpuExecutor(Executor):
    """The HIP library behind the server: models resident as Model objects,
    edits through waves (batched) or single launches (plain)."""

    def __init__(self, models, cameras, max_wave_edits=4096, pad_k=None):
        import torch
        from . import uvl
        self.torch, self.uvl = torch, uvl
        self.models = models                  # list of Model
        # texture padding (§4.3.2) after every edit when pad_k is set: one
        # outline per model, padded inside the waves (batched) or after each
        # edit launch (plain)
        self.outlines = None if pad_k is None else [uvl.Outline(m.geom, int(pad_k)) for m in models]
        self.models_resident = set(range(len(models)))
        self.cameras = cameras                # per model: list of view-proj matrices
        self.depth: Dict[tuple, object] = {}  # (model, camera) -> resident depth map
        self.wave = uvl.Wave(max_wave_edits, max_wave_edits)
        self.max_wave_edits = max_wave_edits
        self._keep = []                       # host arrays of launched batches until their round ends

    def footprint(self, model):
        m = self.models[model]
        return m.geom.nbytes() + sum(l.data.numel() * l.data.element_size() for l in m.layers)

    def prerender(self):
        """Render every (model, camera) depth map now (the cameras are known
        up front), so that no request pays for a first render."""
        for mi, cams in enumerate(self.cameras):
            if mi in self.models_resident:
                for ci in range(len(cams)):
                    self._depth(mi, ci)

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
            if r.kind == "brush":
                batch.brush(m.geom, layer, e.centre, e.radius, e.label)
            else:
                batch.lasso(m.geom, layer, self.cameras[r.model][e.camera], e.poly, self._depth(r.model, e.camera),
                            m.bias, e.label)
        outlines = None
        if self.outlines is not None:
            outlines = [(self.models[mi].geom, self.outlines[mi]) for mi in sorted({r.model for r in reqs})]
        self.wave.submit(batch, outlines=outlines)
        self._keep.append(batch)

    def launch_single(self, r):
        m = self.models[r.model]
        o = None if self.outlines is None else self.outlines[r.model]
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
            o = r.op
            b = None if o.op == self.uvl.REMAP else m.layers[o.b]
            self.uvl.layer_op(o.op, m.layers[o.dst], m.layers[o.a], b, o.sel_a, o.sel_b, o.out_label, o.lut)
        elif r.kind == "area":
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
    latencies_ms: np.ndarray = field(repr=False, default=None)

    def as_dict(self):
        return {"mode": self.mode, "requests": self.n, "wall_s": self.wall_s, "p50_ms": self.p50_ms,
                "p99_ms": self.p99_ms, "edits_per_s": self.edits_per_s, "requests_per_s": self.requests_per_s,
                "rounds": self.rounds, "failed": self.failed, "refused": self.refused}


class Server:
    def __init__(self, executor: Executor, n_models: int, budget_bytes: int, max_wave_edits: int = 4096,
                 max_inflight: int = 2, min_batch: int = 32, max_wait_s: float = 2e-3):
        self.ex = executor
        self.max_wave_edits = max_wave_edits
        self.max_inflight = max_inflight
        # a round starts at once when the device is idle; while rounds are in
        # flight, a further one starts only with min_batch requests queued or
        # once the oldest has waited max_wait_s (small rounds pay the fixed
        # cost of a launch each)
        self.min_batch = min_batch
        self.max_wait_s = max_wait_s
        # admission by HBM footprint, in model order, within the budget
        self.resident = set()
        used = 0
        for m in range(n_models):
            f = executor.footprint(m)
            if used + f <= budget_bytes:
                self.resident.add(m)
                used += f
        self.used_bytes = used

    def run(self, requests: Sequence[Request], mode: str = "batched", spin_s: float = 20e-6) -> Stats:
        """Serve `requests` (arrival times in seconds from now).  Python's
        cyclic garbage collector is paused meanwhile: its pauses land in the
        latency tail."""
        assert mode in ("batched", "plain")
        was = gc.isenabled()
        gc.disable()
        try:
            return self._run(requests, mode, spin_s)
        finally:
            if was:
                gc.enable()

    def _run(self, requests, mode, spin_s) -> Stats:
        reqs = sorted(requests, key=lambda r: (r.t_arrival, r.rid))
        queues: Dict[int, deque] = {}
        inflight: deque = deque()
        nxt = 0
        rounds = 0
        refused = 0
        t0 = time.perf_counter()
        n = len(reqs)
        completed = 0
        nq = 0                                  # queued requests

        def now():
            return time.perf_counter() - t0

        while completed < n:
            t = now()
            # arrivals
            while nxt < n and reqs[nxt].t_arrival <= t:
                r = reqs[nxt]
                nxt += 1
                if r.model not in self.resident:
                    r.ok, r.result, r.t_done = False, "model not resident", t
                    refused += 1
                    completed += 1
                    continue
                queues.setdefault(r.model, deque()).append(r)
                nq += 1
            # completions (in order: one in-order device queue)
            while inflight and self.ex.done(inflight[0].handle):
                rd = inflight.popleft()
                self.ex.finish(rd.handle, rd.requests)
                tt = now()
                for r in rd.requests:
                    r.t_done = tt
                completed += len(rd.requests)
            # launch a round if a slot is free (see min_batch / max_wait_s)
            if nq and len(inflight) < self.max_inflight:
                go = not inflight or mode == "plain" or nq >= self.min_batch
                if not go:
                    oldest = min(q[0].t_arrival for q in queues.values() if q)
                    go = now() - oldest >= self.max_wait_s
                if go:
                    launched = self._round(queues, mode)
                    nq -= len(launched)
                    rounds += 1
                    inflight.append(Round(self.ex.close_round(launched), launched))
                    continue
            if spin_s > 0:
                time.sleep(spin_s)
        wall = now()
        lat = np.array([(r.t_done - r.t_arrival) * 1e3 for r in reqs if r.ok], dtype=np.float64)
        edits = sum(1 for r in reqs if r.ok and r.kind in EDIT_KINDS)
        return Stats(mode, n, wall, float(np.percentile(lat, 50)) if lat.size else float("nan"),
                     float(np.percentile(lat, 99)) if lat.size else float("nan"), edits / wall, n / wall, rounds,
                     sum(1 for r in reqs if not r.ok) - refused, refused, lat)

    def _round(self, queues, mode) -> List[Request]:
        launched: List[Request] = []
        if mode == "plain":
            # every queued request, one launch each, in arrival order
            allq = sorted((r for q in queues.values() for r in q), key=lambda r: (r.t_arrival, r.rid))
            for q in queues.values():
                q.clear()
            for r in allq:
                self.ex.launch_single(r)
                launched.append(r)
            return launched
        # batched: per model, the prefix of edits up to the first non-edit
        wave: List[Request] = []
        tails: List[List[Request]] = []
        for m in list(queues.keys()):
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
