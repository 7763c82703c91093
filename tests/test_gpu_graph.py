"""GPU parity of the captured (device-sized) joins, hc_join_graph_*, against the
CPU oracle and the eager calls.

A captured join replays a fixed launch sequence whose kernels read the frontier
sizes from device memory.  Every replay must give the oracle's count (per-cell
counts, emitted rows) exactly, also when replays alternate with eager calls on
the same context, and a replay whose data exceeds the graph's capacities must
still return the exact result (through the eager path)."""

import json
import os

import numpy as np
import pytest

from paper_2502_06715_amd import batch, hc, inputs
from oracle import cells, oracle
from tests.gpu_util import config_graph, log, sort_rows

pytestmark = pytest.mark.gpu
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "workloads.json")))
SEED = 0x2545F491


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return hc.Context(0)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def test_graph_count_config1_replays(ctx):
    """Workload 1 (ER, 2^12 vertices): the count of every replay equals the oracle's,
    with eager counts, builds and host syncs between the replays."""
    import torch
    E = config_graph(1)
    n, atoms = inputs.QUERIES["triangle"]
    c = hc.build_coco(ctx, _dev(E), [0, 1], symmetric=True)
    q = hc.Query(n, atoms)
    expect = GOLD["1"]["count"]
    for order in ([0, 1, 2], [2, 0, 1]):
        log("graph count config1 order=%s" % order)
        g = hc.JoinGraph(ctx, q, [c] * 3, order, [0, 0, 0])
        for r in range(4):
            cnt, _, rep = g.run()
            assert rep and cnt == expect, (r, cnt, expect)
            assert hc.join_count(ctx, q, [c] * 3, order, [0, 0, 0]) == expect
            c2 = hc.build_coco(ctx, _dev(E[: 1000]), [0, 1])
            c2.free()
            torch.cuda.synchronize()
        g.free()


def test_graph_emit_rows_equal_eager_and_oracle(ctx):
    """Emitted rows of a replay equal the eager hc_join_emit's byte for byte (both in
    frontier order) and, sorted, the oracle's rows; a second replay rewrites them."""
    import torch
    E = config_graph(1)
    n, atoms = inputs.QUERIES["triangle"]
    c = hc.build_coco(ctx, _dev(E), [0, 1], symmetric=True)
    q = hc.Query(n, atoms)
    expect = oracle.gj(n, atoms, [E] * 3, emit=True)
    cap = expect.count + 64
    eager, n_e = hc.join_emit(ctx, q, [c] * 3, [0, 1, 2], [0, 0, 0], capacity=cap)
    out = torch.empty((cap, 3), dtype=torch.int32, device="cuda:0")
    g = hc.JoinGraph(ctx, q, [c] * 3, [0, 1, 2], [0, 0, 0], mode="emit", out=out)
    for r in range(2):
        out.fill_(-1)
        cnt, rows, rep = g.run()
        assert rep and cnt == n_e == expect.count
        got = rows.cpu().numpy()
        assert np.array_equal(got, eager.cpu().numpy())
        assert np.array_equal(sort_rows(got), expect.rows)
    g.free()


def test_graph_emit_overflow_reports_exact_count(ctx):
    E = config_graph(1)
    n, atoms = inputs.QUERIES["triangle"]
    import torch
    c = hc.build_coco(ctx, _dev(E), [0, 1], symmetric=True)
    q = hc.Query(n, atoms)
    out = torch.empty((100, 3), dtype=torch.int32, device="cuda:0")
    g = hc.JoinGraph(ctx, q, [c] * 3, [0, 1, 2], [0, 0, 0], mode="emit", out=out)
    with pytest.raises(hc.HCError) as ei:
        g.run()
    assert ei.value.status == hc.HC_ERR_OVERFLOW
    assert ei.value.n_out == GOLD["1"]["count"]
    g.free()


@pytest.mark.parametrize("case", ["config1", "rmat14", "cycle4"])
def test_graph_cells_equal_oracle_cells(ctx, case):
    """Per-cell counts of a replay against the oracle's cells mode (Generic Join per
    HyperCube cell, cells checked to partition the output)."""
    if case == "config1":
        E, name, b, order, shares = config_graph(1), "triangle", 12, [0, 1, 2], [3, 3, 2]
    elif case == "rmat14":
        E, name, b, order, shares = inputs.rmat(14, 1 << 17, 0x4843_0002), "triangle", 14, [2, 0, 1], [2, 2, 2]
    else:
        E, name, b, order, shares = inputs.erdos_renyi(1 << 9, 3000, 91), "cycle4", 9, [0, 1, 2, 3], [2, 1, 1, 2]
    n, atoms = inputs.QUERIES[name]
    c = hc.build_coco(ctx, _dev(E), [0, 1], key_bits=b, seed=SEED, symmetric=True)
    q = hc.Query(n, atoms)
    log("graph cells %s order=%s shares=%s" % (case, order, shares))
    exp, _ = cells.cells(n, atoms, [E] * len(atoms), shares, b, SEED, order=order)
    g = hc.JoinGraph(ctx, q, [c] * len(atoms), order, shares, mode="cells", cell_group=0)
    for _ in range(3):
        total, got, rep = g.run()
        assert rep
        assert total == int(exp.sum())
        assert np.array_equal(got, exp)
    g.free()


def test_graph_batched_segments_equal_oracle(ctx):
    """A fused batch of small triangle and 4-cycle queries (segmented CoCo, one query
    per segment, 2^extra cells each): per-query counts of every replay against the
    oracle, query by query."""
    specs = inputs.batch_spec(48, log2_lo=10.0, log2_hi=12.0)
    graphs = inputs.batch_graphs(specs)
    for shape in ("triangle", "cycle4"):
        idx = [i for i, s in enumerate(specs) if s["query"] == shape]
        gs = [graphs[i] for i in idx]
        mb = batch.id_bits(gs)
        rel, seg = batch.union_relation(gs, mb)
        c = hc.build_coco(ctx, _dev(rel), [0, 1], key_bits=mb, segment_bits=seg, symmetric=True)
        n, atoms = inputs.QUERIES[shape]
        q = hc.Query(n, atoms)
        expect = np.array([oracle.gj(n, atoms, [g] * len(atoms)).count for g in gs], dtype=np.uint64)
        for extra in (0, 2):
            shares = [0] * n
            shares[0] = seg + extra
            log("graph batch %s: %d queries, extra %d" % (shape, len(gs), extra))
            # the 4-cycles' third frontier holds every 2-path (a, b, c) of the batch
            caps = dict(frontier_cap=1 << 25, item_cap=1 << 26) if shape == "cycle4" else {}
            g = hc.JoinGraph(ctx, q, [c] * len(atoms), list(range(n)), shares, mode="cells", cell_group=extra,
                             **caps)
            for _ in range(2):
                total, per, rep = g.run()
                assert np.array_equal(per[: len(gs)], expect)
                assert total == int(expect.sum())
                assert rep
            g.free()
        c.free()


def test_graph_overflow_falls_back_exactly(ctx):
    """Capacities far below the frontiers: the replay raises its overflow flag and the
    result (count, per-cell counts, rows) still equals the oracle's."""
    import torch
    E = config_graph(1)
    n, atoms = inputs.QUERIES["triangle"]
    c = hc.build_coco(ctx, _dev(E), [0, 1], key_bits=12, seed=SEED, symmetric=True)
    q = hc.Query(n, atoms)
    g = hc.JoinGraph(ctx, q, [c] * 3, [0, 1, 2], [0, 0, 0], frontier_cap=64, item_cap=4096)
    cnt, _, rep = g.run()
    assert not rep and cnt == GOLD["1"]["count"]
    g.free()
    shares = [3, 3, 2]
    exp, _ = cells.cells(n, atoms, [E] * 3, shares, 12, SEED, order=[0, 1, 2])
    g = hc.JoinGraph(ctx, q, [c] * 3, [0, 1, 2], shares, mode="cells", cell_group=1, frontier_cap=64, item_cap=512)
    total, per, rep = g.run()
    assert not rep and total == int(exp.sum())
    assert np.array_equal(per, exp.reshape(-1, 2).sum(axis=1))
    g.free()
    expect = oracle.gj(n, atoms, [E] * 3, emit=True)
    out = torch.empty((expect.count, 3), dtype=torch.int32, device="cuda:0")
    g = hc.JoinGraph(ctx, q, [c] * 3, [0, 1, 2], [0, 0, 0], mode="emit", out=out, item_cap=1024)
    cnt, rows, rep = g.run()
    assert not rep and cnt == expect.count
    assert np.array_equal(sort_rows(rows.cpu().numpy()), expect.rows)
    g.free()


def test_graph_clique4_rewritten_and_plain(ctx):
    """The 4-clique with the rewriting (its lifted intersections run inside the
    graph, pools and (offset, length) words included) and without it (three operands
    at the deepest level): counts, per-cell counts and emitted rows against the
    oracle; capacities below the lifted intersections' sizes fall back exactly; a
    per-element search method is HC_ERR_UNSUPPORTED."""
    import torch
    E = inputs.chung_lu(2048, 12000, 77)
    n, atoms = inputs.QUERIES["clique4"]
    c = hc.build_coco(ctx, _dev(E), [0, 1], key_bits=11, seed=SEED, symmetric=True)
    q = hc.Query(n, atoms)
    exp = oracle.gj(n, atoms, [E] * 6, emit=True)
    assert exp.count > 0
    for flags, shares in ((0, [1, 1, 1, 0]), (hc.HC_NO_REWRITE, [1, 1, 1, 0]), (0, [0, 0, 0, 0])):
        log("graph clique4 flags=%d shares=%s" % (flags, shares))
        g = hc.JoinGraph(ctx, q, [c] * 6, [0, 1, 2, 3], shares, flags=flags)
        for _ in range(2):
            cnt, _, rep = g.run()
            assert rep and cnt == exp.count
        g.free()
        want, _ = cells.cells(n, atoms, [E] * 6, shares, 11, SEED, order=[0, 1, 2, 3])
        g = hc.JoinGraph(ctx, q, [c] * 6, [0, 1, 2, 3], shares, flags=flags, mode="cells", cell_group=0)
        tot, per, rep = g.run()
        assert rep and tot == exp.count and np.array_equal(per, want)
        g.free()
        # emitting materialises the deepest level: without the rewriting its three-operand
        # elements exceed the default item capacity
        out = torch.empty((exp.count + 2, n), dtype=torch.int32, device="cuda:0")
        g = hc.JoinGraph(ctx, q, [c] * 6, [0, 1, 2, 3], shares, flags=flags, mode="emit", out=out,
                         item_cap=1 << 25)
        cnt, rows, rep = g.run()
        assert cnt == exp.count
        assert np.array_equal(sort_rows(rows.cpu().numpy()), exp.rows)
        assert rep
        g.free()
    g = hc.JoinGraph(ctx, q, [c] * 6, [0, 1, 2, 3], [0, 0, 0, 0], item_cap=256)
    cnt, _, rep = g.run()
    assert not rep and cnt == exp.count
    g.free()
    with pytest.raises(hc.HCError) as ei:
        hc.JoinGraph(ctx, q, [c] * 6, [0, 1, 2, 3], [0, 0, 0, 0], flags=hc.HC_NO_REWRITE | hc.HC_SEARCH_EXPONENTIAL)
    assert ei.value.status == hc.HC_ERR_UNSUPPORTED


def _atom_cocos(ctx, atoms, rels, var_order, b, seed=0):
    import torch
    pos = {v: i for i, v in enumerate(var_order)}
    out = []
    for a, r in zip(atoms, rels):
        co = sorted(range(len(a)), key=lambda c: pos[a[c]])
        out.append(hc.build_coco(ctx, torch.from_numpy(np.ascontiguousarray(r)).to("cuda:0"), co, key_bits=b,
                                 seed=seed))
    return out


def test_graph_int64_ids_count_cells_and_emit(ctx):
    """Ids above 2^31 stored as int64 (three different relations): a replay's count,
    per-cell counts and emitted int64 rows against the oracle."""
    import torch
    n, atoms = inputs.QUERIES["triangle"]
    base = (1 << 31) + 12345
    rels = [inputs.random_relation(600 + 40 * j, 60, 610 + j).astype(np.int64) * 7919 + base for j in range(3)]
    exp = oracle.gj(n, atoms, rels, emit=True)
    assert exp.count > 0
    for order, shares in (([0, 1, 2], [0, 0, 0]), ([2, 1, 0], [2, 1, 3])):
        cocos = _atom_cocos(ctx, atoms, rels, order, 32, seed=SEED)
        assert cocos[0].info.dtype == hc.HC_I64
        q = hc.Query(n, atoms)
        log("graph int64 order=%s shares=%s" % (order, shares))
        g = hc.JoinGraph(ctx, q, cocos, order, shares)
        cnt, _, rep = g.run()
        assert rep and cnt == exp.count
        g.free()
        want, _ = cells.cells(n, atoms, rels, shares, 32, SEED, order=order)
        g = hc.JoinGraph(ctx, q, cocos, order, shares, mode="cells", cell_group=0)
        tot, per, rep = g.run()
        assert rep and tot == exp.count and np.array_equal(per, want)
        g.free()
        out = torch.empty((exp.count + 5, n), dtype=torch.int64, device="cuda:0")
        g = hc.JoinGraph(ctx, q, cocos, order, shares, mode="emit", out=out)
        cnt, rows, rep = g.run()
        assert rep and cnt == exp.count
        assert np.array_equal(sort_rows(rows.cpu().numpy()), exp.rows)
        g.free()


def test_graph_range_predicates_equal_oracle(ctx):
    """Range predicates on every variable (pushed into the levels): replayed counts and
    rows against the oracle with the same predicates, for two ranges per query."""
    import torch
    E = config_graph(1)
    n, atoms = inputs.QUERIES["triangle"]
    c = hc.build_coco(ctx, _dev(E), [0, 1], symmetric=True)
    for lo, hi in (([100, 0, 50], [900, 3000, 4096]), ([0, 2000, 0], [4096, 4096, 1500])):
        exp = oracle.gj(n, atoms, [E] * 3, lo=lo, hi=hi, emit=True)
        q = hc.Query(n, atoms, lo, hi)
        log("graph predicates lo=%s hi=%s: %d rows" % (lo, hi, exp.count))
        g = hc.JoinGraph(ctx, q, [c] * 3, [0, 1, 2], [0, 0, 0])
        cnt, _, rep = g.run()
        assert rep and cnt == exp.count
        g.free()
        out = torch.empty((exp.count + 1, n), dtype=torch.int32, device="cuda:0")
        g = hc.JoinGraph(ctx, q, [c] * 3, [0, 1, 2], [0, 0, 0], mode="emit", out=out)
        cnt, rows, rep = g.run()
        assert rep and cnt == exp.count
        assert np.array_equal(sort_rows(rows.cpu().numpy()), exp.rows)
        g.free()


def test_direct_small_joins_within_workspace_bound(ctx):
    """Joins small enough to run the device-sized sequence directly (counts, per-cell
    counts, predicates): results equal the oracle's, and the device memory of each
    call, measured by torch's allocator, stays within hc_join_workspace_bound, which
    admission relies on."""
    import torch
    E = config_graph(1)
    n, atoms = inputs.QUERIES["triangle"]
    c = hc.build_coco(ctx, _dev(E), [0, 1], key_bits=12, seed=SEED, symmetric=True)
    cases = [(hc.Query(n, atoms), [0, 0, 0]), (hc.Query(n, atoms), [2, 1, 1]),
             (hc.Query(n, atoms, [0, 100, 0], [3000, 4096, 4096]), [0, 0, 0])]
    for q, shares in cases:
        exp = oracle.gj(n, atoms, [E] * 3, lo=q.var_lo, hi=q.var_hi).count
        bound = hc.join_workspace_bound(ctx, q, [c] * 3, [0, 1, 2], shares)
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        torch.cuda.reset_peak_memory_stats()
        got = hc.join_count(ctx, q, [c] * 3, [0, 1, 2], shares)
        torch.cuda.synchronize()
        peak = torch.cuda.max_memory_allocated() - base
        log("direct small join shares=%s: %d, peak %d bytes, bound %d" % (shares, got, peak, bound))
        assert got == exp
        assert 0 < peak <= bound
        if q.var_lo is None:
            want, _ = cells.cells(n, atoms, [E] * 3, shares, 12, SEED, order=[0, 1, 2])
            base = torch.cuda.memory_allocated()
            torch.cuda.reset_peak_memory_stats()
            per, tot = hc.join_count_cells(ctx, q, [c] * 3, [0, 1, 2], shares)
            torch.cuda.synchronize()
            assert tot == exp and np.array_equal(per, want)
            assert torch.cuda.max_memory_allocated() - base <= bound
