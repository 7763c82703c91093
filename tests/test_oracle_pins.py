"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each pin is chosen so that a plausible mistake in the oracle (a dropped atom, a
wrong column order, a transposed operand, a lost predicate) fails one of them:
brute-force enumeration on tiny inputs, closed forms on complete graphs,
spectral identities (trace of A^3 and A^4 by scipy.sparse), classical
triangle/4-clique counters, and the worked examples of Sections 4 and 5.
"""

import itertools
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2502_06715_amd import inputs
from oracle import brute, cells, coco, oracle, rewrite

GOLD = os.path.join(os.path.dirname(__file__), "golden")
Q = inputs.QUERIES


def _sym(edges):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    return np.unique(np.concatenate([e, e[:, ::-1]]), axis=0)


def test_splitmix_stream_matches_scalar_definition():
    seed = 0x1234_5678_9ABC
    v = inputs.splitmix64(seed, 5, 7)
    for i in range(7):
        assert int(v[i]) == inputs.splitmix64_scalar(seed, 5 + i)
    # published first output of SplitMix64 seeded with 0: 0xE220A8397B1DCDAF
    assert inputs.splitmix64_scalar(0, 0) == 0xE220A8397B1DCDAF


def test_generators_are_simple_symmetric_graphs():
    for E in [inputs.erdos_renyi(64, 300, 7), inputs.rmat(8, 500, 8), inputs.chung_lu(256, 600, 9)]:
        assert E.dtype == np.int32 and E.shape[1] == 2
        assert np.all(E[:, 0] != E[:, 1])
        und = np.unique(np.sort(E, axis=1), axis=0)
        assert und.shape[0] * 2 == E.shape[0]        # no duplicates
        assert np.array_equal(_sym(E), np.unique(E.astype(np.int64), axis=0))


@pytest.mark.parametrize("name", list(Q))
def test_gj_equals_brute_force_random(name):
    n, atoms = Q[name]
    rng_seed = 100
    for trial in range(6):
        rels = []
        for j, _ in enumerate(atoms):
            rows = 0 if (trial == 5 and j == 1) else 12 + 3 * j   # one case with an empty relation
            k = len(atoms[j])
            rels.append(inputs.random_relation(rows * (1 + 2 * (k > 2)), 5, rng_seed + 17 * trial + j, arity=k)
                        if rows else np.zeros((0, k), np.int32))
        expect = brute.brute(n, atoms, rels)
        for order in itertools.islice(itertools.permutations(range(n)), 0, None, 5):
            r = oracle.gj(n, atoms, rels, order=order, emit=True)
            assert r.count == len(expect)
            assert [tuple(x) for x in r.rows.tolist()] == expect


@pytest.mark.parametrize("name", ["triangle", "cycle4", "clique4", "diamond4", "twotriangle"])
def test_gj_equals_brute_force_symmetric_graph(name):
    n, atoms = Q[name]
    E = inputs.erdos_renyi(8, 14, 3)
    expect = brute.brute(n, atoms, [E] * len(atoms))
    for order in itertools.permutations(range(n)):
        r = oracle.gj(n, atoms, [E] * len(atoms), order=order)
        assert r.count == len(expect)


def test_triangle_closed_form_complete_graph():
    n, atoms = Q["triangle"]
    for k in [3, 4, 7, 12]:
        E = inputs.complete_graph(k)
        assert oracle.gj(n, atoms, [E] * 3).count == k * (k - 1) * (k - 2)


def test_cycle4_closed_forms():
    n, atoms = Q["cycle4"]
    for k in [3, 4, 6]:
        E = inputs.complete_graph(k)
        assert oracle.gj(n, atoms, [E] * 4).count == k * (k - 1) * (k * k - 3 * k + 3)
    for s, t in [(2, 3), (3, 5)]:
        E = inputs.complete_bipartite(s, t)
        assert oracle.gj(n, atoms, [E] * 4).count == 2 * s * s * t * t


def test_clique4_closed_forms():
    n, atoms = Q["clique4"]
    for k in [4, 5, 8]:
        E = inputs.complete_graph(k)
        assert oracle.gj(n, atoms, [E] * 6).count == k * (k - 1) * (k - 2) * (k - 3)
    E = inputs.complete_bipartite(3, 4)
    assert oracle.gj(n, atoms, [E] * 6).count == 0
    assert oracle.gj(*Q["triangle"], [E] * 3).count == 0


def _adj(E):
    n = int(E.max()) + 1
    return sp.csr_matrix((np.ones(E.shape[0], np.float64), (E[:, 0], E[:, 1])), shape=(n, n))


def test_triangle_trace_a3_config1():
    """Workload 1 exactly: ordered triangles = trace(A^3) (float64 exact below 2^53)."""
    E = inputs.config_graph(1)
    A = _adj(E)
    tr = int(round((A @ A).multiply(A).sum()))
    assert oracle.gj(*Q["triangle"], [E] * 3).count == tr
    assert oracle.textbook_triangles(E) * 6 == tr


def test_cycle4_sum_of_squared_a2():
    E = inputs.erdos_renyi(256, 1500, 11)
    A = _adj(E)
    A2 = (A @ A).toarray()
    assert oracle.gj(*Q["cycle4"], [E] * 4).count == int(round((A2 * A2).sum()))


def test_triangle_textbook_rmat():
    E = inputs.rmat(13, 60000, 12)
    assert oracle.gj(*Q["triangle"], [E] * 3, threads=4).count == 6 * oracle.textbook_triangles(E)


def test_clique4_textbook_chung_lu():
    E = inputs.chung_lu(4096, 40000, 13)
    assert oracle.gj(*Q["clique4"], [E] * 6, threads=4).count == 24 * oracle.textbook_4cliques(E)


def test_clique4_digest_textbook_equals_gj():
    """The textbook 4-clique digest (each K4 once, all 24 orderings hashed) equals the
    Generic Join digest, so the full-size 4-clique digest can come from the former."""
    E = inputs.chung_lu(4096, 30000, 14)
    r = oracle.gj(*Q["clique4"], [E] * 6, digest=True, threads=4)
    k, dg = oracle.textbook_4clique_digest(E)
    assert r.count == 24 * k
    assert r.digest == dg


def test_set_semantics_duplicates_ignored():
    n, atoms = Q["triangle"]
    E = inputs.complete_graph(5)
    dup = np.concatenate([E, E[::3], E[::7]])
    assert oracle.gj(n, atoms, [dup, E, dup]).count == 60


def test_range_predicates_and_chunk_union():
    n, atoms = Q["clique4"]
    E = inputs.erdos_renyi(16, 60, 5)
    full = oracle.gj(n, atoms, [E] * 6, emit=True, digest=True)
    lo = [0, 3, 0, 0]
    hi = [16, 11, 16, 16]
    exp = brute.brute(n, atoms, [E] * 6, lo=lo, hi=hi)
    r = oracle.gj(n, atoms, [E] * 6, lo=lo, hi=hi, emit=True)
    assert [tuple(x) for x in r.rows.tolist()] == exp
    # chunks on the first variable partition the output
    rows = []
    for a in range(0, 16, 5):
        r = oracle.gj(n, atoms, [E] * 6, lo=[a, 0, 0, 0], hi=[a + 5, 16, 16, 16], emit=True)
        rows.append(r.rows)
    rows = np.concatenate(rows)
    assert rows.shape[0] == full.count
    assert oracle.digest_rows(rows) == full.digest


def test_digest_is_order_independent():
    n, atoms = Q["triangle"]
    E = inputs.erdos_renyi(32, 150, 21)
    r = oracle.gj(n, atoms, [E] * 3, emit=True, digest=True)
    perm = np.random.default_rng(0).permutation(r.count)
    assert oracle.digest_rows(r.rows[perm]) == r.digest


def test_work_counter_hand_example():
    """Triangle on K_4 (all degrees 3, |R.X| = 4): level 1: m=4, other op 4 -> 4 + min(4, 4*1);
    level 2 (per x): |R[x]|=3 vs |S.X|=4 -> 3 + min(4, 3*ceil(log2(1+4/3))=3*2) = 7, times 4;
    level 3 (per (x,y)): 3 vs 3 -> 3 + min(3, 3*1) = 6, times 12."""
    E = inputs.complete_graph(4)
    r = oracle.gj(*Q["triangle"], [E] * 3, work=True)
    assert r.work == [8, 4 * 7, 12 * 6]


def test_partition_example_exclusive_prefix():
    g = json.load(open(os.path.join(GOLD, "partition_example.json")))
    rel = np.array(g["relation"])
    ids = [[g[h][str(v)] for v in rel[:, c]] for c, h in enumerate(["h_X", "h_Y", "h_Z"])]
    B, Bp = coco.partition_sizes_by_ids(ids, g["shares"])
    assert B[0, 1, 0] == g["expect"]["B_010"]
    assert Bp[0, 1, 0] == g["expect"]["Bpref_010"]
    assert B[1, 0, 0] == g["expect"]["B_100"]
    # the partitioned array holds partition (0,1,0) at its start position
    flat = np.ravel_multi_index(ids, g["shares"])
    part = rel[np.argsort(flat, kind="stable")]
    s = Bp[0, 1, 0]
    assert part[s:s + B[0, 1, 0]].tolist() == g["expect"]["partition_010"]


def test_coco_join_example_level_restriction():
    g = json.load(open(os.path.join(GOLD, "coco_join_example.json")))
    R = coco.coco_levels(np.array(g["R"]), [0, 1, 2], None)
    S = coco.coco_levels(np.array(g["S"]), [0, 1, 2], None)
    e = g["expect"]
    i = int(np.searchsorted(R["V"][0], e["x"]))
    assert i == e["index_in_VX"]
    lo, hi = int(R["O"][0][i]), int(R["O"][0][i + 1])
    assert [lo, hi] == e["OX_range"]
    assert R["V"][1][lo:hi].tolist() == e["R_VY_slice"]
    j = int(np.searchsorted(S["V"][0], e["x"]))
    s_slice = S["V"][1][S["O"][0][j]:S["O"][0][j + 1]].tolist()
    assert s_slice == e["S_VY_slice"]
    assert sorted(set(R["V"][1][lo:hi].tolist()) & set(s_slice)) == e["Y"]


def test_coco_levels_against_nested_dict():
    """CoCo by definition equals the sorted trie built with Python dicts."""
    rel = inputs.random_relation(200, 9, 77, arity=3)
    b, seed = 4, 5
    c = coco.coco_levels(rel, [2, 0, 1], b, seed)
    trie = {}
    for row in rel.tolist():
        k = [coco.mix_scalar(row[cc], b, seed) for cc in [2, 0, 1]]
        trie.setdefault(k[0], {}).setdefault(k[1], set()).add(k[2])
    V0 = sorted(trie)
    assert c["V"][0].tolist() == V0
    v1, o0, v2, o1 = [], [0], [], [0]
    for a in V0:
        for bb in sorted(trie[a]):
            v1.append(bb)
            v2.extend(sorted(trie[a][bb]))
            o1.append(len(v2))
        o0.append(len(v1))
    assert c["V"][1].tolist() == v1 and c["V"][2].tolist() == v2
    assert c["O"][0].tolist() == o0 and c["O"][1].tolist() == o1
    assert c["n_unique"] == len(v2)


@pytest.mark.parametrize("b", [1, 2, 3, 5, 8, 13, 16, 20])
def test_mixer_is_bijective(b):
    x = np.arange(1 << b, dtype=np.uint64)
    y = coco.mix(x, b, seed=0x9E37)
    assert np.unique(y).size == x.size and int(y.max()) < (1 << b)


def test_mixer_32bit_is_lowbias32():
    """At b = 32 with seed 0 the mixer reduces to Wellons' lowbias32 (hash-prospector),
    written here as its published 32-bit steps."""
    def lowbias32(x):
        x ^= x >> 16
        x = (x * 0x7FEB352D) & 0xFFFFFFFF
        x ^= x >> 15
        x = (x * 0x846CA68B) & 0xFFFFFFFF
        x ^= x >> 16
        return x
    for v in [0, 1, 2, 12345, 0xDEADBEEF, 0xFFFFFFFF]:
        assert coco.mix_scalar(v, 32) == lowbias32(v)
        assert int(coco.mix(np.array([v]), 32)[0]) == lowbias32(v)


def test_rewrite_plan_matches_paper_q6():
    g = json.load(open(os.path.join(GOLD, "q6_rewrite_plan.json")))
    plan = rewrite.derive_plan(g["n_vars"], [tuple(a) for a in g["atoms"]], g["order"])
    for lvl, exp in g["lifts"].items():
        got = plan[int(lvl)]["lift"]
        assert (None if got is None else [got[0], got[1]]) == exp


@pytest.mark.parametrize("name", ["clique4", "diamond4", "twotriangle", "cycle4", "triangle"])
def test_rewritten_program_equals_plain_gj(name):
    n, atoms = Q[name]
    E = inputs.erdos_renyi(16, 50, 31)
    base = oracle.gj(n, atoms, [E] * len(atoms), emit=True)
    for order in itertools.islice(itertools.permutations(range(n)), 0, None, 3):
        c1, rows1 = rewrite.run_rewritten(n, atoms, [E] * len(atoms), order, rewrite=True)
        c0, rows0 = rewrite.run_rewritten(n, atoms, [E] * len(atoms), order, rewrite=False)
        assert c1 == c0 == base.count
        assert rows1 == [tuple(x) for x in base.rows.tolist()]


def test_textbook_cycle4_closed_forms_and_gj():
    """trace(A^4) of K_k is (k-1)^4 + (k-1) (eigenvalues k-1 once, -1 k-1 times), of
    K_{s,t} it is 2 s^2 t^2; on a random graph it equals the Generic Join count."""
    for k in [3, 5, 9]:
        assert oracle.textbook_cycle4(inputs.complete_graph(k)) == (k - 1) ** 4 + (k - 1)
    for s, t in [(2, 3), (4, 7)]:
        assert oracle.textbook_cycle4(inputs.complete_bipartite(s, t)) == 2 * s * s * t * t
    E = inputs.rmat(10, 6000, 21)
    assert oracle.textbook_cycle4(E) == oracle.gj(*Q["cycle4"], [E] * 4, threads=4).count
    assert oracle.textbook_cycle4(np.zeros((0, 2), np.int64)) == 0


@pytest.mark.parametrize("b,seg", [(4, 3), (9, 5), (16, 12)])
def test_segmented_mixer_keeps_segment_and_mixes_low_bits(b, seg):
    """Segmented keys: the segment number (bits above b) is kept, the low b bits are
    H_b, so each segment is a bijection of its own block of 2^b ids."""
    n = min(1 << (b + seg), 1 << 20)
    x = np.arange(n, dtype=np.uint64)
    y = coco.mix_segmented(x, b, seed=77)
    assert np.array_equal(y >> np.uint64(b), x >> np.uint64(b))
    assert np.array_equal(y & np.uint64((1 << b) - 1), coco.mix(x & np.uint64((1 << b) - 1), b, seed=77))
    assert np.unique(y).size == n


def test_batch_spec_deterministic_and_mixed():
    a = inputs.batch_spec(256)
    b = inputs.batch_spec(256)
    assert a == b
    shapes = {s["query"] for s in a}
    kinds = {s["kind"] for s in a}
    assert shapes == {"triangle", "cycle4"} and kinds == {"er", "rmat"}
    ms = np.array([s["m"] for s in a])
    assert ms.min() >= 1 << 10 and ms.max() <= 1 << 18
    for s in a[:16]:
        g = inputs.batch_graph(s)
        assert g.shape[0] == 2 * s["m"] and int(g.max()) < s["n"]


def test_ternary_closed_forms():
    """Loomis-Whitney over four full [N]^3 cubes: N^4 tuples; clover-triangle over
    three full U x [N] x [N] relations: |U| N^3; one missing hyperedge of R1 removes
    exactly the N tuples that extend it."""
    N, U = 5, 2
    g = np.stack(np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij"), -1).reshape(-1, 3)
    n, atoms = Q["lw"]
    assert oracle.gj(n, atoms, [g] * 4).count == N ** 4
    r1 = g[~((g[:, 0] == 1) & (g[:, 1] == 2) & (g[:, 2] == 3))]
    assert oracle.gj(n, atoms, [r1, g, g, g]).count == N ** 4 - N
    n, atoms = Q["ct"]
    gu = g[g[:, 0] < U]
    assert oracle.gj(n, atoms, [gu] * 3).count == U * N ** 3


@pytest.mark.parametrize("name,shares", [("triangle", [1, 2, 1]), ("cycle4", [1, 0, 1, 1]),
                                         ("clique4", [1, 1, 1, 0]), ("lw", [1, 1, 0, 1])])
def test_cells_mode_equals_brute_force_partition(name, shares):
    """Cells mode against the definition of Section 5: every brute-force result tuple
    t belongs to the one cell (h(t_1), .., h(t_n)); the per-cell counts must be the
    histogram of those cells, in the library's cell packing, for every order."""
    n, atoms = Q[name]
    b, seed = 4, 0x51
    ternary = any(len(a) > 2 for a in atoms)
    rels = [inputs.random_relation(40 if ternary else 30, 4 if ternary else 10, 900 + j, arity=len(a))
            for j, a in enumerate(atoms)]
    exp = np.asarray(brute.brute(n, atoms, rels), dtype=np.int64).reshape(-1, n)
    assert exp.shape[0] > 0
    for order in itertools.islice(itertools.permutations(range(n)), 0, None, 7):
        got, rows = cells.cells(n, atoms, rels, shares, b, seed, order=order)
        want = np.zeros(got.size, dtype=np.uint64)
        for t in exp:
            c = [int(coco.mix_scalar(int(t[v]), b, seed)) >> (b - shares[v]) for v in range(n)]
            cid, shift = 0, 0   # the library's packing: first variable of the order lowest
            for v in order:
                cid |= c[v] << shift
                shift += shares[v]
            want[cid] += 1
        assert np.array_equal(got, want)
        assert int(got.sum()) == exp.shape[0]


def test_gj_timed_sample():
    """The CPU-baseline sampler: with no deadline it runs every first-variable value
    (the Generic Join count); with a zero deadline and one thread it runs exactly one
    value, whose count is the number of result tuples with that first value; the
    seeded order does not depend on the thread count."""
    n, atoms = Q["clique4"]
    E = inputs.chung_lu(1024, 6000, 45)
    res = oracle.gj(n, atoms, [E] * 6, emit=True)
    full = res.count
    r = oracle.gj_timed(n, atoms, [E] * 6, budget_s=1e9, seed=7, threads=2)
    assert r["count"] == full and r["runs_done"] == r["runs"]
    assert 0 <= r["busy"] <= 2 * r["wall"] + 1e-3
    per_value = {int(v): int(c) for v, c in zip(*np.unique(res.rows[:, 0], return_counts=True))}
    firsts = set()
    for seed in range(1, 9):
        one = oracle.gj_timed(n, atoms, [E] * 6, budget_s=0.0, seed=seed, threads=1)
        assert one["runs_done"] == 1
        firsts.add(one["count"])
        assert one["count"] == 0 or one["count"] in per_value.values()
    assert len(firsts) > 1                     # the seed changes the order


def test_query_table_closed_forms():
    """Q2, Q4 and Q8 of the query table against closed forms that share nothing
    with Generic Join: the 4-loop is the closed 4-walk count, the diamond sums
    2 t(e)^2 over the edges and the two-triangle query (2 t(v))^2 over the vertices,
    t the triangles on an edge or vertex (textbook.c)."""
    for g in (inputs.chung_lu(300, 2000, 3), inputs.rmat(9, 1500, 4), inputs.erdos_renyi(256, 1500, 5)):
        q4, q8 = oracle.textbook_diamond_twotriangle(g, threads=2)
        n, atoms = Q["loop4"]
        assert oracle.gj(n, atoms, [g] * len(atoms), threads=2).count == oracle.textbook_cycle4(g, threads=2)
        n, atoms = Q["diamond4"]
        assert oracle.gj(n, atoms, [g] * len(atoms), threads=2).count == q4
        n, atoms = Q["twotriangle"]
        assert oracle.gj(n, atoms, [g] * len(atoms), threads=2).count == q8
    # a planted mistake is caught: one edge fewer changes both closed forms
    g = inputs.chung_lu(300, 2000, 3)
    base = oracle.textbook_diamond_twotriangle(g, threads=2)
    u, v = int(g[0, 0]), int(g[0, 1])
    keep = ~(((g[:, 0] == u) & (g[:, 1] == v)) | ((g[:, 0] == v) & (g[:, 1] == u)))
    assert oracle.textbook_diamond_twotriangle(g[keep], threads=2) != base
