"""The serving scheduler on the host (simulated device): per-model FIFO
semantics, continuous batching, admission by footprint, failure isolation."""

import numpy as np
import pytest

from paper_2501_14807_amd.serve import Request, Server, SimExecutor

KINDS = ["brush", "lasso", "area", "algebra"]


def _stream(n, n_models, qps, seed=0):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / qps, n))
    kinds = rng.choice(4, n, p=[0.6, 0.25, 0.1, 0.05])
    models = rng.integers(0, n_models, n)
    return [Request(i, float(t[i]), int(models[i]), KINDS[kinds[i]]) for i in range(n)]


def _expected_seen(reqs):
    """For each area request, the ids of its model's requests up to itself."""
    out = {}
    by_model = {}
    for r in sorted(reqs, key=lambda r: (r.t_arrival, r.rid)):
        by_model.setdefault(r.model, []).append(r.rid)
        if r.kind == "area":
            out[r.rid] = tuple(by_model[r.model])
    return out


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_fifo_per_model(mode):
    reqs = _stream(3000, 7, 40000.0)
    ex = SimExecutor([1] * 7)
    st = Server(ex, 7, 100).run(reqs, mode)
    assert st.failed == 0 and st.refused == 0
    want = _expected_seen(reqs)
    for r in reqs:
        assert r.t_done is not None and r.t_done >= r.t_arrival
        if r.kind == "area":
            assert r.result == want[r.rid]
    # per model, launches happen in arrival order
    for m in range(7):
        launched = [rid for _, mm, rid in ex.log if mm == m and rid >= 0]
        arrived = [r.rid for r in sorted(reqs, key=lambda r: (r.t_arrival, r.rid)) if r.model == m]
        assert launched == arrived


def test_continuous_batching_beats_plain_under_load():
    # simulated costs: 100 us per single edit launch, 50 us + 10 us per edit per wave
    reqs = _stream(4000, 16, 30000.0, seed=1)
    st_b = Server(SimExecutor([1] * 16), 16, 100).run([Request(**{**r.__dict__}) for r in reqs], "batched")
    st_p = Server(SimExecutor([1] * 16), 16, 100).run([Request(**{**r.__dict__}) for r in reqs], "plain")
    assert st_b.rounds < len(reqs) / 2          # requests were grouped
    assert st_b.p99_ms < st_p.p99_ms            # the plain queue falls behind
    assert st_b.wall_s <= st_p.wall_s + 0.05


def test_admission_by_footprint_and_eviction():
    """Four models of footprint 40 under a budget of 100: at most two are
    resident at once; models are admitted as their requests arrive and the
    least recently used idle ones evicted; every request completes, in
    per-model arrival order, seeing its model's earlier requests."""
    reqs = _stream(1500, 4, 20000.0, seed=2)
    ex = SimExecutor([40, 40, 40, 40])
    srv = Server(ex, 4, 100)
    st = srv.run(reqs, "batched")
    assert st.failed == 0 and st.refused == 0
    assert st.evictions > 0 and st.admissions > 4
    want = _expected_seen(reqs)
    for r in reqs:
        assert r.ok
        if r.kind == "area":
            assert r.result == want[r.rid]
    # replay the log: the resident set never exceeds the budget, and no work
    # is launched for a model that is not resident
    resident = set()
    for kind, m, _ in ex.log:
        if kind == "admit":
            resident.add(m)
            assert 40 * len(resident) <= 100
        elif kind == "evict":
            resident.discard(m)
        else:
            assert m in resident
    for m in range(4):
        launched = [rid for kind, mm, rid in ex.log if mm == m and rid >= 0]
        arrived = [r.rid for r in sorted(reqs, key=lambda r: (r.t_arrival, r.rid)) if r.model == m]
        assert launched == arrived


def test_model_larger_than_the_budget_is_refused():
    reqs = _stream(400, 3, 20000.0, seed=6)
    ex = SimExecutor([40, 200, 40])
    st = Server(ex, 3, 100).run(reqs, "plain")
    for r in reqs:
        assert r.ok == (r.model != 1)
        if r.model == 1:
            assert r.result == "model larger than the budget"
    assert st.refused == sum(1 for r in reqs if r.model == 1)


def test_preload():
    ex = SimExecutor([40, 40, 40])
    srv = Server(ex, 3, 100)
    srv.preload()
    assert srv.resident == {0, 1} and srv.used_bytes == 80


def test_failure_is_isolated():
    reqs = _stream(800, 5, 20000.0, seed=3)
    ex = SimExecutor([1] * 5, fail_models={3})
    st = Server(ex, 5, 100).run(reqs, "batched")
    want = _expected_seen([r for r in reqs if r.model != 3])
    for r in reqs:
        assert r.ok == (r.model != 3)
        if r.model != 3 and r.kind == "area":
            assert r.result == want[r.rid]
    assert st.failed == sum(1 for r in reqs if r.model == 3)


def test_inflight_limit():
    class Counting(SimExecutor):
        def __init__(self, *a, **k):
            super().__init__(*a, **k)
            self.handles = []
            self.max_seen = 0

        def close_round(self, reqs):
            h = super().close_round(reqs)
            self.handles.append(h)
            live = sum(1 for x in self.handles if not self.done(x))
            self.max_seen = max(self.max_seen, live)
            return h

    reqs = _stream(2000, 8, 50000.0, seed=4)
    ex = Counting([1] * 8, wave_fixed_s=500e-6)
    Server(ex, 8, 100, max_inflight=2).run(reqs, "batched")
    assert ex.max_seen <= 2


def test_busy_device_gets_larger_rounds():
    # a large fixed cost per wave: eager rounds (one per free slot) pay it
    # often, the default policy waits for a batch while a round is in flight
    # (the simulated device runs on the wall clock, so only the round count
    # is compared)
    reqs = _stream(3000, 16, 20000.0, seed=5)

    def run(**kw):
        ex = SimExecutor([1] * 16, wave_fixed_s=300e-6, wave_edit_s=5e-6)
        return Server(ex, 16, 100, **kw).run([Request(**{**r.__dict__}) for r in reqs], "batched")

    eager = run(min_batch=1)
    adaptive = run()
    assert adaptive.rounds < 0.9 * eager.rounds
    assert adaptive.failed == 0 and adaptive.refused == 0
    assert adaptive.n == eager.n == len(reqs)
