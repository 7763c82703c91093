"""Host logic of the serving loop (admission, continuous batching, FIFO order),
with an injected engine that computes nothing on a device."""

import threading
import time

import numpy as np
import pytest

from paper_2502_06715_amd import inputs, serve


class FakeEngine:
    """count = (lo * 7 + hi) per request; estimate = per_query * n + width; records passes."""

    def __init__(self, per_query=100, delay=0.0, index_bytes=0):
        self.per_query = per_query
        self.delay = delay
        self.index_bytes = index_bytes
        self.passes = []
        self.lock = threading.Lock()
        self.reserved_now = 0
        self.est_of = {}

    def group_key(self, r):
        return (r.graph, r.query)

    def weight(self, r):
        return float(r.hi - r.lo)

    def estimate(self, key, n, width):
        return self.per_query * n + width

    def run(self, slot, key, reqs, fused):
        assert all(self.group_key(r) == key for r in reqs)
        ranges = [(r.lo, r.hi) for r in reqs]
        with self.lock:
            self.passes.append((slot, key, list(ranges), fused))
        if self.delay:
            time.sleep(self.delay)
        return [lo * 7 + hi for lo, hi in ranges]


def _reqs(n, keys, seed=0, gap=0.0):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        g, q = keys[int(rng.integers(len(keys)))]
        lo = int(rng.integers(0, 1000))
        out.append(serve.Request(id=i, graph=g, query=q, lo=lo, hi=lo + int(rng.integers(1, 17)), t_arrival=i * gap))
    return out


def test_every_request_answered_with_its_own_count():
    eng = FakeEngine(delay=0.002)
    reqs = _reqs(300, [(0, "triangle"), (1, "cycle4"), (2, "clique4")], gap=0.0002)
    srv = serve.Server(eng, budget_bytes=10 ** 9, n_slots=3, max_batch=64)
    wall = serve.replay(srv, reqs)
    assert all(r.error is None and r.count == r.lo * 7 + r.hi for r in reqs)
    # a pass only holds requests of one (graph, shape)
    for slot, key, ranges, fused in eng.passes:
        assert fused and len(ranges) <= 64
    assert sum(len(p[2]) for p in eng.passes) == len(reqs)
    s = serve.summarize(reqs, wall)
    assert s["answered"] == 300 and s["p99_ms"] >= s["p50_ms"] >= 0


def test_requests_arriving_during_a_pass_are_fused_into_the_next():
    eng = FakeEngine(delay=0.05)
    reqs = _reqs(60, [(0, "triangle")], gap=0.001)
    srv = serve.Server(eng, budget_bytes=10 ** 9, n_slots=1, max_batch=256)
    serve.replay(srv, reqs)
    sizes = [len(p[2]) for p in eng.passes]
    assert sizes[0] == 1 and max(sizes) > 10 and sum(sizes) == 60


def test_unfused_mode_runs_one_request_per_pass():
    eng = FakeEngine()
    reqs = _reqs(40, [(0, "triangle"), (0, "cycle4")])
    srv = serve.Server(eng, budget_bytes=10 ** 9, n_slots=2, fuse=False)
    serve.replay(srv, reqs)
    assert all(len(p[2]) == 1 and not p[3] for p in eng.passes)
    assert all(r.count == r.lo * 7 + r.hi for r in reqs)


def test_admission_never_exceeds_budget_and_halves_batches():
    # free budget 1000 bytes; one request costs 100 + width -> at most ~8 per pass
    eng = FakeEngine(per_query=100, delay=0.002, index_bytes=500)
    reqs = _reqs(200, [(0, "triangle")])
    srv = serve.Server(eng, budget_bytes=1500, n_slots=3, max_batch=256)
    serve.replay(srv, reqs)
    assert srv.free0 == 1000 and srv.peak_reserved <= 1000
    assert all(len(p[2]) * 100 <= 1000 for p in eng.passes)
    assert all(r.error is None for r in reqs)


def test_request_larger_than_the_budget_fails_alone():
    eng = FakeEngine(per_query=100)
    reqs = _reqs(10, [(0, "triangle")])
    reqs[3].hi = reqs[3].lo + 5000        # its estimate (100 + 5000) exceeds the free budget
    srv = serve.Server(eng, budget_bytes=2000, n_slots=2, max_batch=1)
    serve.replay(srv, reqs)
    assert reqs[3].error is not None and reqs[3].count is None
    assert all(r.error is None for i, r in enumerate(reqs) if i != 3)


def test_budget_below_resident_indexes_is_refused():
    with pytest.raises(ValueError):
        serve.Server(FakeEngine(index_bytes=10 ** 6), budget_bytes=10 ** 5)


def test_serve_stream_is_seeded_and_poisson():
    from paper_2502_06715_amd import inputs
    gs = inputs.serve_graph_specs()
    a = inputs.serve_stream(gs, 4000, qps=1000.0)
    assert a == inputs.serve_stream(gs, 4000, qps=1000.0)
    gaps = np.diff([0.0] + [r["t"] for r in a])
    assert abs(gaps.mean() * 1000.0 - 1.0) < 0.1          # mean gap 1/qps
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.1       # exponential: cv = 1
    frac = {k: sum(r["query"] == k for r in a) / len(a) for k in ("triangle", "cycle4", "clique4")}
    assert abs(frac["triangle"] - 0.5) < 0.03 and abs(frac["cycle4"] - 0.3) < 0.03
    assert all(0 <= r["lo"] < r["hi"] <= gs[r["graph"]]["n"] for r in a)
    ms = [s["m"] for s in gs]
    assert ms[0] == 1 << 16 and ms[-1] == 1 << 24 and len(gs) == 16


def test_weight_budget_keeps_heavy_requests_apart():
    """With max_weight, a pass carries at most that much work (its first request
    always): a heavy request runs without the light ones queued behind it."""
    eng = FakeEngine(delay=0.01)
    reqs = [serve.Request(id=i, graph=0, query="triangle", lo=0, hi=(100 if i == 3 else 2)) for i in range(12)]
    srv = serve.Server(eng, budget_bytes=10 ** 9, n_slots=1, max_batch=64, max_weight=10.0)
    serve.replay(srv, reqs)
    for slot, key, ranges, fused in eng.passes:
        w = sum(hi - lo for lo, hi in ranges)
        assert w <= 10.0 or len(ranges) == 1
    assert any(ranges == [(0, 100)] for _, _, ranges, _ in eng.passes)
    assert all(r.count == r.lo * 7 + r.hi for r in reqs)


def test_full_query_stream_shapes_and_graphs():
    """Full-query requests cover the whole id range of their graph; triangles go to
    any graph, 4-cycles and 4-cliques only to graphs of at most max_edges edges; the
    stream is a pure function of its seed."""
    specs = inputs.serve_graph_specs()
    a = inputs.serve_full_stream(specs, 300, qps=40.0)
    assert a == inputs.serve_full_stream(specs, 300, qps=40.0)
    small = {s["g"] for s in specs if s["m"] <= inputs.FULL_MAX_EDGES}
    assert small and len(small) < len(specs)
    shapes = set()
    for r in a:
        assert r["full"] and r["lo"] == 0 and r["hi"] == specs[r["graph"]]["n"]
        shapes.add(r["query"])
        if r["query"] != "triangle":
            assert r["graph"] in small
    assert shapes == {"triangle", "cycle4", "clique4"}
    assert {r["graph"] for r in a if r["query"] == "triangle"} - small
    t = [r["t"] for r in a]
    assert all(x < y for x, y in zip(t, t[1:]))
