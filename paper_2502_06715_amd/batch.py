"""Batched execution of many small join queries.

The queries of one shape (triangle or 4-cycle) and size class are fused into a
single Generic Join: their graphs become one relation whose ids carry the query number above
the vertex bits (a segmented CoCo, see hc_build_coco_segmented), the first
variable's share is the query number, so every query is one HyperCube cell (or
2^extra cells), and the per-cell counts of hc_join_count_cells are the per-query
counts.  The deepest level of all queries of a shape then runs as one persistent
launch whose per-XCD queues sweep the queries in order.

`run_sequential` is the one-query-per-launch baseline: build, decide shares and
count each query on its own.
"""

from __future__ import annotations

import time

import numpy as np

from . import hc, inputs


def union_relation(graphs, mix_bits: int):
    """Concatenate graphs with query i's ids shifted to i * 2^mix_bits."""
    seg_bits = max(1, int(len(graphs) - 1).bit_length())
    assert mix_bits + seg_bits <= 31, "batch too large for int32 ids"
    parts = []
    for i, g in enumerate(graphs):
        if g.shape[0]:
            assert int(g.max()) < (1 << mix_bits)
        parts.append(g.astype(np.int64) + (np.int64(i) << np.int64(mix_bits)))
    rel = np.concatenate(parts).astype(np.int32) if parts else np.zeros((0, 2), np.int32)
    return rel, seg_bits


# Size classes of the batched queries: class c holds the queries whose edge count is
# below 2^SIZE_CLASSES[c] (and at least the previous bound); the last class the rest.
SIZE_CLASSES = (12, 14, 16)


def size_class(m: int) -> int:
    """Size class of a query with m undirected edges."""
    for c, lg in enumerate(SIZE_CLASSES):
        if m < (1 << lg):
            return c
    return len(SIZE_CLASSES)


def id_bits(graphs) -> int:
    mx = max((int(g.max()) for g in graphs if g.shape[0]), default=1)
    return max(1, mx.bit_length())


class Autotune:
    """Measured choice of a batch's launch parameters, cached per batch signature
    (a shape and size class of queries): the extra split of every query's first
    variable (its share: 2^extra cells per query) and the search method of the
    intersections (the LDS windows or one of Section 5's per-element methods).
    Coordinate descent: the split is timed with the default method, then the
    methods with the chosen split."""

    def __init__(self, splits=(0, 1, 2, 3), methods=("window", "exponential", "by_size")):
        self.splits = tuple(splits)
        self.methods = tuple(methods)
        self.choice = {}
        self.timings = {}

    def _best(self, key, cands, run):
        best, best_t = None, None
        for c in cands:
            t0 = time.perf_counter()
            run(c)
            dt = time.perf_counter() - t0
            self.timings[(key, c)] = dt
            if best_t is None or dt < best_t:
                best, best_t = c, dt
        return best

    def pick(self, key, run):
        """run(extra_bits, method) executes the batch once; returns (extra_bits, method)."""
        if key in self.choice:
            return self.choice[key]
        x = self._best(key, [(s, self.methods[0]) for s in self.splits], lambda c: run(*c))[0]
        best = self._best(key, [(x, m) for m in self.methods], lambda c: run(*c))
        self.choice[key] = best
        return best


def count_batched(ctx: hc.Context, shape: str, rel_dev, n_queries: int, mix_bits: int, seg_bits: int,
                  extra_bits: int = 0, coco=None, method: str = "window"):
    """Per-query counts (uint64 array) of one fused join over a segmented relation."""
    n, atoms = inputs.QUERIES[shape]
    own = coco is None
    if own:
        coco = hc.build_coco(ctx, rel_dev, [0, 1], key_bits=mix_bits, segment_bits=seg_bits, symmetric=True)
    # one segment per query: the library sums each query's 2^extra_bits cells
    per_query, _ = hc.join_count_segments(ctx, hc.Query(n, atoms), [coco] * len(atoms), list(range(n)),
                                          extra_bits, flags=hc.SEARCH_METHODS[method])
    if own:
        coco.free()
    return per_query[:n_queries]


def graph_caps(shape: str, graphs, limit: int = 1 << 28):
    """Exact frontier and element capacities of a fused batch's captured join (order
    0..n-1, only the first variable split, so no frontier entry is replicated), from
    the degrees: the triangle's frontiers and materialised levels hold at most the
    directed edges; the 4-cycle's third frontier holds every 2-path (a, b, c), the
    sum of the squared degrees (the edge lists hold both directions).  None when that exceeds `limit` (the batch then runs
    eagerly)."""
    need = sum(int(g.shape[0]) for g in graphs)   # directed edges: the lists hold both directions
    if shape == "cycle4":
        paths = 0
        for g in graphs:
            if g.shape[0]:
                deg = np.bincount(g[:, 0].astype(np.int64))
                paths += int((deg ** 2).sum())
        need = max(need, paths)
    if need > limit:
        return None
    return max(need, 1 << 12), max(need, 1 << 12)


class BatchGraph:
    """A fused batch's count per query as a captured join (hc_join_graph) over its
    resident segmented CoCo: replayed per step, with the per-query counts summed over
    each query's 2^extra cells on the device."""

    def __init__(self, ctx: hc.Context, shape: str, coco, n_queries: int, extra_bits: int, caps):
        n, atoms = inputs.QUERIES[shape]
        seg = int(coco.info.key_bits - coco.info.mix_bits)
        shares = [0] * n
        shares[0] = seg + extra_bits
        self.n_queries = n_queries
        self.g = hc.JoinGraph(ctx, hc.Query(n, atoms), [coco] * len(atoms), list(range(n)), shares,
                              mode="cells", cell_group=extra_bits, frontier_cap=caps[0], item_cap=caps[1])

    def launch(self):
        self.g.launch()

    def result(self):
        """(per-query counts, replayed)."""
        _, per, rep = self.g.result()
        return per[: self.n_queries], rep

    def free(self):
        self.g.free()


def count_sequential(ctx: hc.Context, shape: str, graphs_dev, log2_cells: int = 6):
    """One query per launch: build, choose shares by the cost model, count."""
    n, atoms = inputs.QUERIES[shape]
    q = hc.Query(n, atoms)
    out = np.zeros(len(graphs_dev), dtype=np.uint64)
    for i, t in enumerate(graphs_dev):
        c = hc.build_coco(ctx, t, [0, 1], symmetric=True)
        order, shares = hc.compute_shares(ctx, q, [c] * len(atoms), log2_cells)
        out[i] = hc.join_count(ctx, q, [c] * len(atoms), order, shares)
        c.free()
    return out
