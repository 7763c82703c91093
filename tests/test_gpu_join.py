"""GPU parity of the Generic Join hot path against the CPU oracle.

Bit-exact: the u64 count, and the sorted set of emitted head-order rows.  The
result must not depend on the variable order, the shares, the rewriting or the
chunking (Section 5: cells partition the output; Section 6.1: the lift is an
exact re-association of sorted-set intersections)."""

import itertools
import json
import os

import numpy as np
import pytest

from paper_2502_06715_amd import hc, inputs
from oracle import oracle
from tests.gpu_util import config_graph, log, sort_rows

pytestmark = pytest.mark.gpu
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "workloads.json")))


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return hc.Context(0)


def _coco(ctx, rel, order=(0, 1), b=0, symmetric=False):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(rel)).to("cuda:0")
    return hc.build_coco(ctx, t, list(order), key_bits=b, symmetric=symmetric)


def _atom_cocos(ctx, atoms, rels, var_order, b):
    """One CoCo per atom, columns ordered by the variable order."""
    pos = {v: i for i, v in enumerate(var_order)}
    out = []
    for a, r in zip(atoms, rels):
        co = sorted(range(len(a)), key=lambda c: pos[a[c]])
        out.append(_coco(ctx, r, co, b))
    return out


def _emit_sorted(ctx, q, cocos, order, shares, cap, flags=0):
    rows, n = hc.join_emit(ctx, q, cocos, order, shares, flags=flags, capacity=cap)
    return sort_rows(rows.cpu().numpy()), n


def test_config1_triangle_all_orders_shares(ctx):
    E = config_graph(1)
    n, atoms = inputs.QUERIES["triangle"]
    q = hc.Query(n, atoms)
    exp = oracle.gj(n, atoms, [E] * 3, emit=True, digest=True)
    assert exp.count == GOLD["1"]["count"]
    c = _coco(ctx, E, b=12, symmetric=True)
    for order in itertools.permutations(range(3)):
        for shares in [[0, 0, 0], [1, 2, 3], [4, 4, 4], [12, 0, 0], [0, 0, 12], [2, 0, 5]]:
            sh = [0] * 3
            for i, v in enumerate(order):
                sh[v] = shares[i]
            log("config1 order=%s shares=%s" % (order, sh))
            cnt, dg = hc.join_count(ctx, q, [c] * 3, list(order), sh, digest=True)
            assert cnt == exp.count
            assert dg == exp.digest
    rows, n_out = _emit_sorted(ctx, q, [c] * 3, [0, 1, 2], [3, 3, 2], exp.count + 5)
    assert n_out == exp.count
    assert np.array_equal(rows, exp.rows)


@pytest.mark.parametrize("name", list(inputs.QUERIES))
def test_random_relations_all_queries(ctx, name):
    n, atoms = inputs.QUERIES[name]
    for trial in range(3):
        ternary = any(len(a) > 2 for a in atoms)
        rels = [inputs.random_relation(300 + 50 * j, 9 if ternary else 40, 500 + 31 * trial + j, arity=len(atoms[j]))
                for j in range(len(atoms))]
        exp = oracle.gj(n, atoms, rels, emit=True)
        for k, order in enumerate(itertools.islice(itertools.permutations(range(n)), 0, None, 7)):
            order = list(order)
            cocos = _atom_cocos(ctx, atoms, rels, order, 6)
            q = hc.Query(n, atoms)
            shares = [(k + v) % 2 for v in range(n)]
            log("%s trial=%d order=%s shares=%s" % (name, trial, order, shares))
            for flags in [0, hc.HC_NO_REWRITE]:
                cnt = hc.join_count(ctx, q, cocos, order, shares, flags=flags)
                assert cnt == exp.count
            rows, n_out = _emit_sorted(ctx, q, cocos, order, shares, exp.count + 1)
            assert n_out == exp.count
            assert np.array_equal(rows, exp.rows)


@pytest.mark.parametrize("name", ["clique4", "diamond4", "twotriangle", "cycle4"])
def test_rewrite_on_off_symmetric_graph(ctx, name):
    n, atoms = inputs.QUERIES[name]
    E = inputs.chung_lu(2048, 12000, 77)
    c = _coco(ctx, E, b=11, symmetric=True)
    q = hc.Query(n, atoms)
    exp = oracle.gj(n, atoms, [E] * len(atoms), digest=True)
    for order in itertools.islice(itertools.permutations(range(n)), 0, None, 5):
        for flags in [0, hc.HC_NO_REWRITE]:
            log("%s order=%s flags=%d" % (name, order, flags))
            cnt, dg = hc.join_count(ctx, q, [c] * len(atoms), list(order), [1] * n, flags=flags, digest=True)
            assert (cnt, dg) == (exp.count, exp.digest)


def test_empty_and_disjoint_relations(ctx):
    n, atoms = inputs.QUERIES["triangle"]
    q = hc.Query(n, atoms)
    empty = np.zeros((0, 2), np.int32)
    R = inputs.random_relation(100, 20, 3)
    cocos = [_coco(ctx, R, b=5), _coco(ctx, empty, b=5), _coco(ctx, R, b=5)]
    assert hc.join_count(ctx, q, cocos, [0, 1, 2], [1, 1, 1]) == 0
    rows, n_out = hc.join_emit(ctx, q, cocos, [0, 1, 2], None, capacity=0)
    assert n_out == 0


def test_emit_overflow_reports_exact_count(ctx):
    E = config_graph(1)
    n, atoms = inputs.QUERIES["triangle"]
    c = _coco(ctx, E, b=12, symmetric=True)
    with pytest.raises(hc.HCError) as ei:
        hc.join_emit(ctx, hc.Query(n, atoms), [c] * 3, [0, 1, 2], [2, 2, 2], capacity=100)
    assert ei.value.status == hc.HC_ERR_OVERFLOW
    assert ei.value.n_out == GOLD["1"]["count"]


def test_range_predicate_chunks_union(ctx):
    n, atoms = inputs.QUERIES["clique4"]
    E = inputs.chung_lu(1024, 8000, 5)
    c = _coco(ctx, E, b=10, symmetric=True)
    full = oracle.gj(n, atoms, [E] * 6, emit=True)
    parts = []
    for a in range(0, 1024, 200):
        lo, hi = [a, 0, 0, 0], [a + 200, 1 << 20, 1 << 20, 1 << 20]
        q = hc.Query(n, atoms, lo, hi)
        exp = oracle.gj(n, atoms, [E] * 6, lo=lo, hi=hi, emit=True)
        rows, n_out = _emit_sorted(ctx, q, [c] * 6, [1, 0, 2, 3], [1, 1, 0, 1], exp.count + 1)
        assert n_out == exp.count and np.array_equal(rows, exp.rows)
        parts.append(rows)
    allr = sort_rows(np.concatenate(parts))
    assert np.array_equal(allr, full.rows)


def test_emit_is_deterministic(ctx):
    E = config_graph(1)
    n, atoms = inputs.QUERIES["triangle"]
    c = _coco(ctx, E, b=12, symmetric=True)
    q = hc.Query(n, atoms)
    first = None
    for _ in range(10):
        rows, _ = hc.join_emit(ctx, q, [c] * 3, [0, 1, 2], [2, 3, 1], capacity=GOLD["1"]["count"])
        r = rows.cpu().numpy()
        if first is None:
            first = r
        assert np.array_equal(r, first)


def test_errors_mismatched_cocos(ctx):
    n, atoms = inputs.QUERIES["triangle"]
    R = inputs.random_relation(100, 20, 3)
    a, b = _coco(ctx, R, b=5), _coco(ctx, R, b=6)
    with pytest.raises(hc.HCError) as ei:
        hc.join_count(ctx, hc.Query(n, atoms), [a, b, a], [0, 1, 2])
    assert ei.value.status == hc.HC_ERR_INVALID
    # column order that contradicts the variable order (non-symmetric relation)
    t = _coco(ctx, R, order=(1, 0), b=5)
    with pytest.raises(hc.HCError) as ei:
        hc.join_count(ctx, hc.Query(n, atoms), [t, a, a], [0, 1, 2])
    assert ei.value.status == hc.HC_ERR_INVALID
    with pytest.raises(hc.HCError):
        hc.join_count(ctx, hc.Query(n, atoms), [a, a, a], [0, 1, 2], [6, 0, 0])   # share > key_bits


def test_share_sweep_invariance_rmat(ctx):
    """All share vectors with sum 6 over the three variables (cf. Section 7.5)."""
    E = inputs.rmat(14, 1 << 17, 0x4843_0002)
    n, atoms = inputs.QUERIES["triangle"]
    exp = oracle.textbook_triangles(E) * 6
    c = _coco(ctx, E, b=14, symmetric=True)
    q = hc.Query(n, atoms)
    for ka in range(7):
        for kb in range(7 - ka):
            sh = [ka, kb, 6 - ka - kb]
            assert hc.join_count(ctx, q, [c] * 3, [0, 1, 2], sh) == exp, sh


def test_config2_triangle_count(ctx):
    E = config_graph(2)
    n, atoms = inputs.QUERIES["triangle"]
    q = hc.Query(n, atoms)
    c = _coco(ctx, E, b=20, symmetric=True)
    order, shares = hc.compute_shares(ctx, q, [c] * 3, 12)
    log("config2 order=%s shares=%s" % (order, shares))
    assert hc.join_count(ctx, q, [c] * 3, order, shares) == GOLD["2"]["count"]
    assert hc.join_count(ctx, q, [c] * 3, [0, 1, 2], [0, 0, 0]) == GOLD["2"]["count"]
    # the cache share rule (the bench's default): count and output digest
    order, shares = hc.compute_shares(ctx, q, [c] * 3, 12, flags=hc.HC_CACHE_SHARES)
    log("config2 cache rule order=%s shares=%s" % (order, shares))
    cnt, dg = hc.join_count(ctx, q, [c] * 3, order, shares, digest=True)
    assert cnt == GOLD["2"]["count"]
    assert dg == (int(GOLD["2"]["digest"][0]), int(GOLD["2"]["digest"][1]))


def _config3(ctx):
    E = config_graph(3)
    n, atoms = inputs.QUERIES["clique4"]
    c = _coco(ctx, E, b=18, symmetric=True)
    return E, n, atoms, c


def test_config3_clique4_count_and_digest(ctx):
    """Full-size 4-clique workload: count and output digest against the oracle's values
    (oriented K4 enumeration; Generic Join digest pinned to it on smaller graphs)."""
    E, n, atoms, c = _config3(ctx)
    q = hc.Query(n, atoms)
    order, shares = hc.compute_shares(ctx, q, [c] * 6, 12)
    log("config3 order=%s shares=%s" % (order, shares))
    cnt, dg = hc.join_count(ctx, q, [c] * 6, order, shares, digest=True)
    g = GOLD["3"]
    assert cnt == g["count"]
    assert dg == (int(g["digest"][0]), int(g["digest"][1]))
    assert hc.join_count(ctx, q, [c] * 6, order, shares, flags=hc.HC_NO_REWRITE) == g["count"]
    order, shares = hc.compute_shares(ctx, q, [c] * 6, 12, flags=hc.HC_CACHE_SHARES)
    log("config3 cache rule order=%s shares=%s" % (order, shares))
    assert hc.join_count(ctx, q, [c] * 6, order, shares) == g["count"]


def test_config3_chunked_emit(ctx):
    """Range-restricted chunks of the materialised output (predicate on variable 0)."""
    E, n, atoms, c = _config3(ctx)
    for ch in GOLD["3"]["chunks"]:
        lo = [ch["lo"], 0, 0, 0]
        hi = [ch["hi"], 1 << 31, 1 << 31, 1 << 31]
        q = hc.Query(n, atoms, lo, hi)
        rows, n_out = hc.join_emit(ctx, q, [c] * 6, [0, 1, 2, 3], [3, 4, 3, 2], capacity=ch["count"] + 16)
        assert n_out == ch["count"]
        r = rows.cpu().numpy().astype(np.int64)
        assert oracle.digest_rows(r) == (int(ch["digest"][0]), int(ch["digest"][1]))
        assert np.all((r[:, 0] >= ch["lo"]) & (r[:, 0] < ch["hi"]))


def test_config3_emit_capacity_2_28(ctx):
    """Materialising the full output into 2^28 rows overflows with the exact total."""
    E, n, atoms, c = _config3(ctx)
    q = hc.Query(n, atoms)
    with pytest.raises(hc.HCError) as ei:
        hc.join_emit(ctx, q, [c] * 6, [0, 1, 2, 3], [6, 6, 0, 0], capacity=1 << 28)
    assert ei.value.status == hc.HC_ERR_OVERFLOW
    assert ei.value.n_out == GOLD["3"]["count"]


@pytest.mark.parametrize("name", ["lw", "ct"])
def test_ternary_dense_cubes_closed_form(ctx, name):
    """Full Cartesian products: Loomis-Whitney over four [N]^3 cubes has N^4 tuples;
    the clover-triangle over U x [N] x [N] relations has |U| N^3."""
    n, atoms = inputs.QUERIES[name]
    N, U = 24, 3
    g = np.stack(np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij"), -1).reshape(-1, 3)
    if name == "ct":
        g = g[g[:, 0] < U]
    rels = [g.astype(np.int32)] * len(atoms)
    expect = N ** 4 if name == "lw" else U * N ** 3
    for order in [[0, 1, 2, 3], [3, 2, 1, 0], [1, 3, 0, 2]]:
        cocos = _atom_cocos(ctx, atoms, rels, order, 0)
        for shares in [[0, 0, 0, 0], [2, 1, 0, 1]]:
            for flags in [0, hc.HC_NO_REWRITE]:
                log("%s cubes order=%s shares=%s flags=%d" % (name, order, shares, flags))
                assert hc.join_count(ctx, hc.Query(n, atoms), cocos, order, shares, flags=flags) == expect


def test_ternary_mixed_arity_query(ctx):
    """Atoms of arity 1, 2 and 3 in one query (unary filter, binary edge, ternary
    hyperedge), every order, against the oracle's emitted rows."""
    n, atoms = 4, [(0, 1, 2), (2, 3), (1,), (0, 3)]
    rels = [inputs.random_relation(900, 10, 71, 3), inputs.random_relation(60, 10, 72, 2),
            inputs.random_relation(6, 10, 73, 1), inputs.random_relation(50, 10, 74, 2)]
    exp = oracle.gj(n, atoms, rels, emit=True)
    assert exp.count > 0
    for order in itertools.permutations(range(n)):
        order = list(order)
        cocos = _atom_cocos(ctx, atoms, rels, order, 5)
        rows, n_out = _emit_sorted(ctx, hc.Query(n, atoms), cocos, order, [1, 0, 1, 0], exp.count + 1)
        assert n_out == exp.count and np.array_equal(rows, exp.rows)


@pytest.mark.parametrize("name", ["lw", "ct"])
def test_st_sparse_small_against_oracle(ctx, name):
    """The ST-Sparse recipe at small domains (LW: 4 distinct random relations at density
    0.22; CT: 3 relations of random pairs under both first-attribute values)."""
    ds = inputs.st_sparse(n=30, rows=6000, m=120, rows2=2500)
    n, atoms = inputs.QUERIES[name]
    rels = ds[name]
    exp = oracle.gj(n, atoms, rels, emit=True)
    assert exp.count > 0
    for order in [[0, 1, 2, 3], [2, 0, 3, 1]]:
        cocos = _atom_cocos(ctx, atoms, rels, order, 0)
        q = hc.Query(n, atoms)
        for shares in [[0, 0, 0, 0], [1, 1, 1, 0]]:
            log("st_sparse %s order=%s shares=%s" % (name, order, shares))
            assert hc.join_count(ctx, q, cocos, order, shares) == exp.count
        rows, n_out = _emit_sorted(ctx, q, cocos, order, [1, 0, 1, 0], exp.count + 1)
        assert n_out == exp.count and np.array_equal(rows, exp.rows)


@pytest.mark.parametrize("method", ["window", "exponential", "quadratic", "linear", "by_size"])
def test_search_methods_agree(ctx, method):
    """Section 5's search methods (and the LDS windows) only change how operands are
    searched: counts, digests and emitted rows are identical."""
    flags = hc.SEARCH_METHODS[method]
    E = inputs.chung_lu(2048, 12000, 77)
    c = _coco(ctx, E, b=11, symmetric=True)
    for name in ["triangle", "cycle4", "clique4"]:
        n, atoms = inputs.QUERIES[name]
        exp = oracle.gj(n, atoms, [E] * len(atoms), digest=True)
        for shares in [[0] * n, [2] + [1] * (n - 1)]:
            log("search %s %s shares=%s" % (method, name, shares))
            got = hc.join_count(ctx, hc.Query(n, atoms), [c] * len(atoms), list(range(n)), shares, flags=flags,
                                digest=True)
            assert got == (exp.count, exp.digest)
    n, atoms = inputs.QUERIES["lw"]
    rels = [inputs.random_relation(500, 9, 900 + j, 3) for j in range(4)]
    exp = oracle.gj(n, atoms, rels, emit=True)
    cocos = _atom_cocos(ctx, atoms, rels, list(range(n)), 0)
    rows, n_out = _emit_sorted(ctx, hc.Query(n, atoms), cocos, list(range(n)), [1, 0, 1, 0], exp.count + 1,
                               flags=flags)
    assert n_out == exp.count and np.array_equal(rows, exp.rows)
    if method == "window":
        with pytest.raises(hc.HCError):
            hc.join_count(ctx, hc.Query(*inputs.QUERIES["triangle"]), [c] * 3, [0, 1, 2], flags=0x700)
