"""More GPU parity against the CPU oracle: per-cell outputs, 64-bit ids, levels
with more than four operands, sorted emission, the forced intersection methods,
and the full-size 4-clique chunks compared row by row.

All comparisons are exact: per-cell u64 counts, emitted rows byte for byte."""

import itertools
import json
import os

import numpy as np
import pytest

from paper_2502_06715_amd import hc, inputs
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


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def _atom_cocos(ctx, atoms, rels, var_order, b, seed=0, dtype=None):
    pos = {v: i for i, v in enumerate(var_order)}
    out = []
    for a, r in zip(atoms, rels):
        co = sorted(range(len(a)), key=lambda c: pos[a[c]])
        out.append(hc.build_coco(ctx, _dev(r, dtype), co, key_bits=b, seed=seed))
    return out


# ---------------------------------------------------------------- per-cell outputs (Section 5)
@pytest.mark.parametrize("case", ["config1", "rmat14", "clique4"])
def test_cell_counts_equal_oracle_cells(ctx, case):
    """hc_join_count_cells cell by cell against the oracle's cells mode, which runs
    Generic Join on every cell's fragments and checks that the cells partition Q(D)."""
    if case == "config1":
        E, name, b, runs = config_graph(1), "triangle", 12, [([0, 1, 2], [3, 3, 2]), ([2, 0, 1], [2, 1, 3])]
    elif case == "rmat14":
        E, name, b, runs = inputs.rmat(14, 1 << 17, 0x4843_0002), "triangle", 14, [([2, 0, 1], [2, 2, 2])]
    else:
        E, name, b, runs = inputs.chung_lu(2048, 12000, 77), "clique4", 11, [([1, 0, 2, 3], [1, 1, 1, 1])]
    n, atoms = inputs.QUERIES[name]
    c = hc.build_coco(ctx, _dev(E), [0, 1], key_bits=b, seed=SEED, symmetric=True)
    q = hc.Query(n, atoms)
    for order, shares in runs:
        log("cells %s order=%s shares=%s" % (case, order, shares))
        exp, _ = cells.cells(n, atoms, [E] * len(atoms), shares, b, SEED, order=order)
        got, total = hc.join_count_cells(ctx, q, [c] * len(atoms), order, shares)
        assert total == int(exp.sum())
        assert np.array_equal(got, exp)


# ---------------------------------------------------------------- 64-bit ids
def test_int64_ids_count_and_emit(ctx):
    """Ids at and above 2^31 (they do not fit int32), stored as int64: counts, digests,
    sorted emitted rows (int64) and per-cell counts equal the oracle's."""
    n, atoms = inputs.QUERIES["triangle"]
    base = (1 << 31) + 12345
    rels = [inputs.random_relation(600 + 40 * j, 60, 610 + j).astype(np.int64) * 7919 + base
            for j in range(3)]
    assert all(int(r.max()) < (1 << 32) for r in rels)
    exp = oracle.gj(n, atoms, rels, emit=True, digest=True)
    assert exp.count > 0
    for order in [[0, 1, 2], [2, 1, 0]]:
        cocos = _atom_cocos(ctx, atoms, rels, order, 32, seed=SEED)
        assert cocos[0].info.dtype == hc.HC_I64
        q = hc.Query(n, atoms)
        for shares in [[0, 0, 0], [2, 1, 3]]:
            log("int64 order=%s shares=%s" % (order, shares))
            assert hc.join_count(ctx, q, cocos, order, shares, digest=True) == (exp.count, exp.digest)
            rows, n_out = hc.join_emit(ctx, q, cocos, order, shares, capacity=exp.count + 3)
            assert rows.dtype.itemsize == 8 and n_out == exp.count
            assert np.array_equal(sort_rows(rows.cpu().numpy()), exp.rows)
            rows, n_out = hc.join_emit(ctx, q, cocos, order, shares, flags=hc.HC_EMIT_SORTED, capacity=exp.count)
            assert np.array_equal(rows.cpu().numpy(), exp.rows)
        per, tot = hc.join_count_cells(ctx, q, cocos, order, [1, 1, 1])
        want, _ = cells.cells(n, atoms, rels, [1, 1, 1], 32, SEED, order=order)
        assert tot == exp.count and np.array_equal(per, want)


# ---------------------------------------------------------------- levels with more than four operands
def _wide_query():
    # variable 0 appears in six atoms: one binary edge relation and five unary filters
    return 2, [(0, 1), (0,), (0,), (0,), (0,), (0,)]


def test_levels_with_more_than_four_operands(ctx):
    """A variable in six atoms: without the rewriting its level intersects six
    operands, with it the five unary filters form one lifted group of five; both
    exceed the four operands of the cursor kernel, so the per-element kernels
    (k_probe, k_materialize) run for counting, digests, per-cell counts, frontier
    expansion, lifted pools and emitted rows."""
    n, atoms = _wide_query()
    rng = np.random.default_rng(5)
    R = inputs.random_relation(900, 40, 77)
    units = [np.sort(rng.choice(40, 32, replace=False)).astype(np.int32).reshape(-1, 1) for _ in range(5)]
    rels = [R] + units
    exp = oracle.gj(n, atoms, rels, emit=True, digest=True)
    assert exp.count > 0
    for order in [[0, 1], [1, 0]]:
        cocos = _atom_cocos(ctx, atoms, rels, order, 6)
        q = hc.Query(n, atoms)
        plan = hc.plan_describe(q, order)
        log("wide order=%s plan=%s" % (order, json.dumps(plan)))
        for flags in [0, hc.HC_NO_REWRITE]:
            for shares in [[0, 0], [1, 2]]:
                assert hc.join_count(ctx, q, cocos, order, shares, flags=flags, digest=True) == \
                    (exp.count, exp.digest)
                rows, n_out = hc.join_emit(ctx, q, cocos, order, shares, flags=flags | hc.HC_EMIT_SORTED,
                                           capacity=exp.count + 1)
                assert n_out == exp.count and np.array_equal(rows.cpu().numpy(), exp.rows)
            per, tot = hc.join_count_cells(ctx, q, cocos, order, [1, 1], flags=flags)
            want, _ = cells.cells(n, atoms, rels, [1, 1], 6, 0, order=order)
            assert tot == exp.count and np.array_equal(per, want)


def test_six_clique_five_child_operands(ctx):
    """The 6-clique query (15 binary atoms) without the rewriting: its deepest level
    intersects five child lists.  On K_n the count is n(n-1)(n-2)(n-3)(n-4)(n-5); on
    a random graph it equals the oracle's."""
    n = 6
    atoms = [(i, j) for i in range(n) for j in range(i + 1, n)]
    q = hc.Query(n, atoms)
    for k in [6, 9]:
        E = inputs.complete_graph(k)
        c = hc.build_coco(ctx, _dev(E), [0, 1], key_bits=4, symmetric=True)
        want = k * (k - 1) * (k - 2) * (k - 3) * (k - 4) * (k - 5)
        for flags in [0, hc.HC_NO_REWRITE]:
            assert hc.join_count(ctx, q, [c] * len(atoms), list(range(n)), [1, 0, 0, 0, 0, 1], flags=flags) == want
    E = inputs.chung_lu(256, 3000, 19)
    exp = oracle.gj(n, atoms, [E] * len(atoms), digest=True)
    assert exp.count > 0
    c = hc.build_coco(ctx, _dev(E), [0, 1], key_bits=8, symmetric=True)
    for flags in [0, hc.HC_NO_REWRITE]:
        log("6-clique flags=%d" % flags)
        assert hc.join_count(ctx, q, [c] * len(atoms), list(range(n)), [1, 1, 0, 0, 0, 1], flags=flags,
                             digest=True) == (exp.count, exp.digest)


# ---------------------------------------------------------------- sorted emission
def test_emit_sorted_config1_byte_equal(ctx):
    """Workload 1: HC_EMIT_SORTED returns the oracle's sorted rows byte for byte (no
    host-side sort), for several orders and share vectors."""
    E = config_graph(1)
    n, atoms = inputs.QUERIES["triangle"]
    exp = oracle.gj(n, atoms, [E] * 3, emit=True)
    c = hc.build_coco(ctx, _dev(E), [0, 1], key_bits=12, symmetric=True)
    q = hc.Query(n, atoms)
    for order, shares in [([0, 1, 2], [0, 0, 0]), ([1, 2, 0], [3, 3, 2]), ([2, 0, 1], [0, 6, 0])]:
        rows, n_out = hc.join_emit(ctx, q, [c] * 3, order, shares, flags=hc.HC_EMIT_SORTED, capacity=exp.count)
        assert n_out == exp.count
        got = rows.cpu().numpy()
        assert got.dtype == np.int32
        assert got.tobytes() == exp.rows.astype(np.int32).tobytes()


def test_emit_sorted_wide_rows(ctx):
    """Rows wider than 64 bits of keys (4 columns of 20 bits) take the per-column
    passes: still the oracle's sorted rows."""
    E = inputs.chung_lu(1 << 20, 20000, 31)
    n, atoms = inputs.QUERIES["clique4"]
    exp = oracle.gj(n, atoms, [E] * 6, emit=True)
    c = hc.build_coco(ctx, _dev(E), [0, 1], key_bits=20, symmetric=True)
    assert 4 * c.info.key_bits > 64
    rows, n_out = hc.join_emit(ctx, hc.Query(n, atoms), [c] * 6, [0, 1, 2, 3], [2, 1, 1, 0],
                               flags=hc.HC_EMIT_SORTED, capacity=exp.count)
    assert n_out == exp.count and np.array_equal(rows.cpu().numpy(), exp.rows)


# ---------------------------------------------------------------- forced methods and flag checks
def test_forced_methods_and_flag_rejection(ctx):
    E = inputs.chung_lu(2048, 12000, 77)
    c = hc.build_coco(ctx, _dev(E), [0, 1], key_bits=11, symmetric=True)
    n, atoms = inputs.QUERIES["clique4"]
    q = hc.Query(n, atoms)
    exp = oracle.gj(n, atoms, [E] * 6, digest=True)
    for flags in [hc.HC_FORCE_MERGE, hc.HC_FORCE_GALLOP, hc.HC_FORCE_MERGE | hc.HC_SEARCH_LINEAR,
                  hc.HC_FORCE_GALLOP | hc.HC_SEARCH_EXPONENTIAL]:
        assert hc.join_count(ctx, q, [c] * 6, [0, 1, 2, 3], [1, 1, 0, 1], flags=flags, digest=True) == \
            (exp.count, exp.digest)
    bad = [hc.HC_FORCE_MERGE | hc.HC_FORCE_GALLOP, hc.HC_FORCE_MERGE | hc.HC_SEARCH_EXPONENTIAL,
           hc.HC_FORCE_GALLOP | hc.HC_SEARCH_QUADRATIC, 0x1000, hc.HC_KEEP_ORDER, hc.HC_EMIT_SORTED]
    for flags in bad:
        with pytest.raises(hc.HCError) as ei:
            hc.join_count(ctx, q, [c] * 6, [0, 1, 2, 3], None, flags=flags)
        assert ei.value.status == hc.HC_ERR_INVALID, flags
    with pytest.raises(hc.HCError) as ei:
        hc.join_emit(ctx, q, [c] * 6, [0, 1, 2, 3], None, flags=0x800, capacity=0)
    assert ei.value.status == hc.HC_ERR_INVALID
    with pytest.raises(hc.HCError) as ei:
        hc.compute_shares(ctx, q, [c] * 6, 4, flags=hc.HC_EMIT_SORTED)
    assert ei.value.status == hc.HC_ERR_INVALID


# ---------------------------------------------------------------- workload 3 chunks row by row
@pytest.mark.parametrize("k", range(3))
def test_config3_chunk_rows(ctx, k):
    """Range-restricted chunks of the full-size 4-clique output, emitted sorted on the
    device and compared row by row with the oracle's rows (and its stored digest)."""
    E = config_graph(3)
    n, atoms = inputs.QUERIES["clique4"]
    ch = GOLD["3"]["chunks"][k]
    big = 1 << 31
    lo, hi = [ch["lo"], 0, 0, 0], [ch["hi"], big, big, big]
    exp = oracle.gj(n, atoms, [E] * 6, lo=lo, hi=hi, emit=True, digest=True, capacity=ch["count"])
    assert exp.count == ch["count"] and exp.digest == (int(ch["digest"][0]), int(ch["digest"][1]))
    c = hc.build_coco(ctx, _dev(E), [0, 1], key_bits=18, symmetric=True)
    log("config3 chunk %d: %d rows" % (k, ch["count"]))
    rows, n_out = hc.join_emit(ctx, hc.Query(n, atoms, lo, hi), [c] * 6, [0, 1, 2, 3], [3, 4, 3, 2],
                               flags=hc.HC_EMIT_SORTED, capacity=ch["count"])
    assert n_out == ch["count"]
    assert np.array_equal(rows.cpu().numpy(), exp.rows)


def _table_count(name, g):
    """Expected count of a query-table query: Generic Join for the triangle, else the
    closed forms pinned against it (closed 4-walks, sum of 2 t(e)^2, K4 x 24, sum of
    (2 t(v))^2), since Q2, Q4 and Q8 have 10^8 to 10^11 results at this size."""
    if name == "triangle":
        n, atoms = inputs.QUERIES[name]
        return oracle.gj(n, atoms, [g] * len(atoms), threads=8).count
    if name == "loop4":
        return oracle.textbook_cycle4(g, threads=8)
    if name == "clique4":
        return 24 * oracle.textbook_4cliques(g, threads=8)
    q4, q8 = oracle.textbook_diamond_twotriangle(g, threads=8)
    return q4 if name == "diamond4" else q8


@pytest.mark.parametrize("name", ["triangle", "loop4", "diamond4", "clique4", "twotriangle"])
def test_query_table_optimizer_plans(ctx, name):
    """The query table (Q1, Q2, Q4, Q6, Q8) with the order and shares the cost model
    picks (cache rule), on the workload-3 recipe at 2^12 vertices / 2^16 edges."""
    g = inputs.config_graph(3, scale_down=6)
    n, atoms = inputs.QUERIES[name]
    log("query table %s on %d tuples" % (name, g.shape[0]))
    want = _table_count(name, g)
    c = hc.build_coco(ctx, _dev(g), [0, 1], symmetric=True)
    q = hc.Query(n, atoms)
    order, shares = hc.compute_shares(ctx, q, [c] * len(atoms), 8, flags=hc.HC_CACHE_SHARES)
    assert hc.join_count(ctx, q, [c] * len(atoms), order, shares) == want
    c.free()


@pytest.mark.parametrize("name", ["loop4", "diamond4"])
def test_query_table_full_size(ctx, name):
    """Q2 and Q4 at the query table's size (2^16 vertices, 2^20 edges: 4.6e10 and
    1.9e10 ordered tuples) against the stored closed-form counts."""
    rec = [r for r in GOLD["9"]["queries"] if r["query"] == name][0]
    g = inputs.config_graph(3, scale_down=rec["scale_down"])
    n, atoms = inputs.QUERIES[name]
    log("query table %s at full size, %d tuples" % (name, g.shape[0]))
    c = hc.build_coco(ctx, _dev(g), [0, 1], symmetric=True)
    q = hc.Query(n, atoms)
    order, shares = hc.compute_shares(ctx, q, [c] * len(atoms), 12, flags=hc.HC_CACHE_SHARES)
    assert hc.join_count(ctx, q, [c] * len(atoms), order, shares) == int(rec["count"])
    c.free()
