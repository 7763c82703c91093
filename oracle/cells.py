"""HyperCube cells by definition -- TEST INFRASTRUCTURE ONLY.

Section 2 ("HyperCube Algorithm") gives every variable v a share P_v and a hash
h_v into [0, P_v); a cell is a coordinate vector (s_1..s_n), and an atom's tuple
is sent to every cell whose coordinates agree with the hashes of the tuple's
values on the atom's variables.  Section 5 (Executor) runs one Generic Join
per cell on those fragments and concatenates the outputs: a result tuple t is
produced by the one cell (h_1(t_1), .., h_n(t_n)), so the cells' outputs are
pairwise disjoint and their union is Q(D).

Reading of the open hash (the same as the CoCo oracle's): shares are powers of
two, P_v = 2^k_v, and h_v(x) is the top k_v bits of the b-bit bijective mixer
H_b of ``oracle.coco`` (one mixer for every variable).

``cells`` filters every relation per cell, runs the Generic Join oracle on each
cell's fragments, checks that every emitted tuple lies in the cell that
emitted it, that no tuple is emitted by two cells, and that the union equals
the unpartitioned result, and returns the per-cell counts.  Small inputs only
(one oracle call per cell).
"""

from __future__ import annotations

import itertools

import numpy as np

from . import coco, oracle


def coords(x, k: int, b: int, seed: int = 0) -> np.ndarray:
    """Coordinate of each value under a share 2^k: the top k bits of H_b(x)."""
    x = np.asarray(x, dtype=np.int64)
    if k == 0:
        return np.zeros(x.shape, dtype=np.int64)
    return (coco.mix(x, b, seed) >> np.uint64(b - k)).astype(np.int64)


def cell_index(coord_by_var, log2_shares, order) -> int:
    """Cell id of a coordinate vector in the library's packing: the variables in
    order, the first variable of the order in the lowest bits, variable v taking
    log2_shares[v] bits."""
    cid, shift = 0, 0
    for v in order:
        cid |= int(coord_by_var[v]) << shift
        shift += int(log2_shares[v])
    return cid


def cells(n_vars: int, atoms, relations, log2_shares, b: int, seed: int = 0, order=None, check: bool = True):
    """Per-cell Generic Join.  Returns (counts, rows): counts[c] is the number of
    result tuples of cell c (library packing, see ``cell_index``), rows[c] the
    sorted head-order tuples of cell c.  With check, asserts the partition
    properties of Section 5 against the unpartitioned oracle."""
    order = list(range(n_vars)) if order is None else list(order)
    ks = [int(k) for k in log2_shares]
    rels = [np.asarray(r, dtype=np.int64).reshape(-1, len(a)) for r, a in zip(relations, atoms)]
    # coordinate of every value of every atom column
    col_coord = [[coords(r[:, c], ks[a[c]], b, seed) for c in range(len(a))] for r, a in zip(rels, atoms)]
    n_cells = 1 << sum(ks)
    counts = np.zeros(n_cells, dtype=np.uint64)
    rows = [None] * n_cells
    for s in itertools.product(*[range(1 << k) for k in ks]):
        frags = []
        for r, a, cc in zip(rels, atoms, col_coord):
            keep = np.ones(r.shape[0], dtype=bool)
            for c, v in enumerate(a):
                keep &= cc[c] == s[v]
            frags.append(r[keep])
        res = oracle.gj(n_vars, atoms, frags, order=order, emit=True)
        cid = cell_index(s, ks, order)
        counts[cid] = res.count
        rows[cid] = res.rows
        if check and res.count:
            for v in range(n_vars):
                assert np.all(coords(res.rows[:, v], ks[v], b, seed) == s[v]), \
                    "cell %s emitted a tuple outside its coordinates" % (s,)
    if check:
        nonempty = [r for r in rows if r is not None and r.shape[0]]
        union = np.concatenate(nonempty) if nonempty else np.zeros((0, n_vars), np.int64)
        if union.shape[0]:
            union = union[np.lexsort(union.T[::-1])]
            assert not np.any(np.all(union[1:] == union[:-1], axis=1)), "two cells emitted the same tuple"
        full = oracle.gj(n_vars, atoms, rels, order=order, emit=True)
        assert union.shape[0] == full.count and np.array_equal(union, full.rows), \
            "the union of the cells differs from the unpartitioned result"
    return counts, rows
