"""GPU parity of the served path: hc_join_count_multi (many instances of one query,
each with its own id block on the first variable, in one pass) against the same
instances counted alone and against the oracle (Section 2: the range predicate
selects a sub-relation of the first variable's values), and the serving loop's
answers in a concurrent, fused mix against the same requests run alone."""

import numpy as np
import pytest

from paper_2502_06715_amd import hc, inputs, serve
from oracle import oracle
from tests.gpu_util import log

pytestmark = pytest.mark.gpu
BIG = 1 << 40


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return hc.Context(0)


@pytest.fixture(scope="module")
def graph():
    return inputs.rmat(11, 9000, 32)


def _alone(ctx, shape, coco, lo, hi):
    n, atoms = inputs.QUERIES[shape]
    q = hc.Query(n, atoms, var_lo=[lo] + [0] * (n - 1), var_hi=[hi] + [BIG] * (n - 1))
    return hc.join_count(ctx, q, [coco] * len(atoms), list(range(n)))


@pytest.mark.parametrize("shape", ["triangle", "cycle4", "clique4"])
def test_multi_equals_alone_and_oracle(ctx, graph, shape):
    import torch
    n, atoms = inputs.QUERIES[shape]
    coco = hc.build_coco(ctx, torch.from_numpy(graph).to("cuda:0"), [0, 1], symmetric=True)
    rng = np.random.default_rng(7)
    ranges = [(0, 1), (0, 16), (5, 5), (10, 3), (2040, 5000), (1 << 33, 1 << 34), (0, BIG)]
    for _ in range(40):
        lo = int(rng.integers(0, 2048))
        ranges.append((lo, lo + int(rng.integers(1, 65))))
    log("multi %s: %d ranges" % (shape, len(ranges)))
    got = hc.join_count_multi(ctx, hc.Query(n, atoms), [coco] * len(atoms), list(range(n)), ranges)
    for (lo, hi), c in zip(ranges, got):
        exp = 0 if lo >= hi else oracle.gj(n, atoms, [graph] * len(atoms), lo=[lo] + [0] * (n - 1),
                                           hi=[hi] + [BIG] * (n - 1)).count
        assert int(c) == exp, (lo, hi)
        if lo < hi:
            assert _alone(ctx, shape, coco, lo, hi) == exp
    # the whole id space is the plain count
    assert int(got[6]) == hc.join_count(ctx, hc.Query(n, atoms), [coco] * len(atoms), list(range(n)))
    coco.free()


def test_multi_single_and_empty_batches(ctx, graph):
    import torch
    n, atoms = inputs.QUERIES["triangle"]
    coco = hc.build_coco(ctx, torch.from_numpy(graph).to("cuda:0"), [0, 1], symmetric=True)
    q = hc.Query(n, atoms)
    assert hc.join_count_multi(ctx, q, [coco] * 3, [0, 1, 2], np.zeros((0, 2), np.int64)).size == 0
    one = hc.join_count_multi(ctx, q, [coco] * 3, [0, 1, 2], [(3, 9)])
    assert int(one[0]) == _alone(ctx, "triangle", coco, 3, 9)
    coco.free()


def test_workspace_bound_covers_the_peak(ctx, graph):
    import torch
    n, atoms = inputs.QUERIES["clique4"]
    coco = hc.build_coco(ctx, torch.from_numpy(graph).to("cuda:0"), [0, 1], symmetric=True)
    q = hc.Query(n, atoms)
    ranges = [(i * 8, i * 8 + 8) for i in range(200)]
    bound = hc.join_workspace_bound(ctx, q, [coco] * 6, list(range(n)), None, 0, n_queries=len(ranges),
                                    first_width=8)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    hc.join_count_multi(ctx, q, [coco] * 6, list(range(n)), ranges)
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() - base
    log("workspace bound %d bytes, peak %d bytes" % (bound, peak))
    assert 0 < peak <= bound
    full = hc.join_workspace_bound(ctx, q, [coco] * 6, list(range(n)), [1, 1, 0, 0], 0)
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    hc.join_count(ctx, q, [coco] * 6, list(range(n)), [1, 1, 0, 0])
    torch.cuda.synchronize()
    assert torch.cuda.max_memory_allocated() - base <= full
    coco.free()


@pytest.mark.parametrize("shared", [False, True])
def test_server_mix_equals_alone(ctx, shared):
    """Requests answered by the serving loop (3 slots on their own streams, fused
    passes, admission by the workspace bound; one CoCo per graph, or all graphs in
    one segmented CoCo) equal the same requests run alone, one per launch on
    per-graph CoCos, and the oracle on a sample."""
    specs = inputs.serve_graph_specs(n_graphs=3, log2_lo=11.0, log2_hi=13.0)
    graphs = [inputs.serve_graph(s) for s in specs]
    stream = inputs.serve_stream(specs, 400, qps=20000.0, seed=inputs.SEED_SERVE + 99)
    eng = serve.GpuEngine(graphs, n_slots=3, shared_index=shared)
    ref = serve.GpuEngine(graphs, n_slots=1) if shared else eng
    srv = serve.Server(eng, budget_bytes=16 << 30, n_slots=3, max_batch=64)
    reqs = serve.requests_from_stream(stream)
    wall = serve.replay(srv, reqs)
    summ = serve.summarize(reqs, wall)
    log("served (shared index %s) %s" % (shared, summ))
    assert summ["answered"] == len(reqs) and summ["mean_batch"] > 1.0
    for r in reqs:
        alone = ref.run(0, ref.group_key(r), [r], fused=False)[0]
        assert r.count == alone, (r, alone)
    for r in reqs[:40]:
        n, atoms = inputs.QUERIES[r.query]
        exp = oracle.gj(n, atoms, [graphs[r.graph]] * len(atoms), lo=[r.lo] + [0] * (n - 1),
                        hi=[r.hi] + [BIG] * (n - 1)).count
        assert r.count == exp
    if shared:
        ref.close()
    eng.close()


def test_batch_ranges_must_stay_in_one_segment(ctx):
    import torch
    from paper_2502_06715_amd import batch
    gs = [inputs.rmat(8, 600, 5), inputs.rmat(8, 700, 6)]
    mb = batch.id_bits(gs)
    rel, seg = batch.union_relation(gs, mb)
    c = hc.build_coco(ctx, torch.from_numpy(rel).to("cuda:0"), [0, 1], key_bits=mb, segment_bits=seg,
                      symmetric=True)
    q = hc.Query(*inputs.QUERIES["triangle"])
    with pytest.raises(hc.HCError):
        hc.join_count_multi(ctx, q, [c] * 3, [0, 1, 2], [((1 << mb) - 4, (1 << mb) + 4)])
    got = hc.join_count_multi(ctx, q, [c] * 3, [0, 1, 2], [(0, 1 << mb), (1 << mb, 2 << mb)])
    assert [int(x) for x in got] == [6 * oracle.textbook_triangles(g) for g in gs]
    c.free()


def test_full_queries_in_the_mix_equal_alone(ctx):
    """Full-query requests (the whole query on a resident graph) served together with
    id-block requests of the same shapes, concurrently and fused: each answer equals
    the same request alone and the oracle's full count."""
    specs = inputs.serve_graph_specs(n_graphs=3, log2_lo=11.0, log2_hi=13.0)
    graphs = [inputs.serve_graph(s) for s in specs]
    blocks = inputs.serve_stream(specs, 200, qps=20000.0, seed=inputs.SEED_SERVE + 98)
    fulls = inputs.serve_full_stream(specs, 30, qps=20000.0, seed=inputs.SEED_SERVE + 97, max_edges=6000)
    assert {f["query"] for f in fulls} == {"triangle", "cycle4", "clique4"}
    stream = sorted(blocks + [dict(f, id=1000 + f["id"]) for f in fulls], key=lambda r: r["t"])
    eng = serve.GpuEngine(graphs, n_slots=3, shared_index=True)
    ref = serve.GpuEngine(graphs, n_slots=1)
    srv = serve.Server(eng, budget_bytes=16 << 30, n_slots=3, max_batch=64)
    reqs = serve.requests_from_stream(stream)
    wall = serve.replay(srv, reqs)
    summ = serve.summarize(reqs, wall)
    log("served with full queries: %s" % summ)
    assert summ["answered"] == len(reqs)
    full_exp = {}
    for r in reqs:
        assert r.count == ref.run(0, ref.group_key(r), [r], fused=False)[0], r
        if r.full:
            key = (r.graph, r.query)
            if key not in full_exp:
                n, atoms = inputs.QUERIES[r.query]
                full_exp[key] = oracle.gj(n, atoms, [graphs[r.graph]] * len(atoms)).count
            assert r.count == full_exp[key], r
    assert sum(r.full for r in reqs) == 30
    ref.close()
    eng.close()


def test_grid_limit_keeps_results(ctx, graph):
    """A context whose persistent kernels use at most a few workgroups (a serving
    slot's device share) gets the same counts as the default grid."""
    import torch
    c = hc.build_coco(ctx, torch.from_numpy(graph).to("cuda:0"), [0, 1], symmetric=True)
    small = hc.Context(0)
    for name in ["triangle", "clique4"]:
        n, atoms = inputs.QUERIES[name]
        q = hc.Query(n, atoms)
        exp = hc.join_count(ctx, q, [c] * len(atoms), list(range(n)), [1] * n)
        for lim in [8, 64, 1000]:
            small.set_grid_limit(lim)
            assert hc.join_count(small, q, [c] * len(atoms), list(range(n)), [1] * n) == exp
        small.set_grid_limit(0)
    with pytest.raises(hc.HCError):
        small.set_grid_limit(-1)
    c.free()
