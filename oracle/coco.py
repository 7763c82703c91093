"""The CoCo index and HyperCube partition ids by definition -- TEST INFRASTRUCTURE ONLY.

CoCo (Section 4, "Compressed Column layout"): for a k-ary relation sorted
lexicographically in the variable order, level r holds V_r, the values of
column r listed once per distinct prefix of length r, and O_r, where the
children of entry e of level r are entries O_r[e] .. O_r[e+1]-1 of level r+1
(O_r has l_r + 1 entries).  The relation is a set, so the last level keeps no
offsets (the build drops O_k).

Partition ids (Section 4): tuple (x_1..x_k) of an atom gets the ids
s_c = h(x_c) mod P_c.  The hash is left open by the paper; the reading used
here is the b-bit bijective mixer H_b below, and shares are powers of two, so
s_c is the top log2(P_c) bits of H_b(x_c).  The CoCo stores the mixed keys
H_b(x): sorted order is mixed-key order, and every partition of every level is
a contiguous range.

Partition sizes B and start positions B^pref (Section 4): B counts tuples per
partition id vector; B^pref is the *exclusive* prefix sum of B in
lexicographic order of the id vectors (the start of each partition in the
partitioned array), the reading forced by the worked example of Section 4.

H_b: Wellons' "lowbias32" integer hash (hash-prospector; xorshift 16,
multiply 0x7feb352d, xorshift 15, multiply 0x846ca68b, xorshift 16),
restricted to b-bit words: every step is taken modulo 2^b, and the shifts
become ceil(b/2), max(1, ceil(b/2)-1), ceil(b/2).  The seed is xor-ed in
first.  Each step is a bijection of b-bit words (xorshift-right, and
multiplication by an odd constant), so H_b is a bijection of [0, 2^b).
This is an independent implementation of that definition.
"""

from __future__ import annotations

import numpy as np

C1 = 0x7FEB352D
C2 = 0x846CA68B


def mix_params(b: int):
    h = (b + 1) // 2
    return h, max(1, h - 1), h


def mix_segmented(x, b: int, seed: int = 0):
    """Segmented keys (batched relations): H_b on the low b bits, the bits above them
    (the segment number) unchanged."""
    x = np.asarray(x).astype(np.uint64)
    hi = (x >> np.uint64(b)) << np.uint64(b)
    return hi | mix(x & np.uint64((1 << b) - 1), b, seed)


def mix(x, b: int, seed: int = 0):
    """H_b on an array of non-negative ids < 2^b (uint64 arithmetic)."""
    x = np.asarray(x).astype(np.uint64)
    mask = np.uint64((1 << b) - 1)
    s1, s2, s3 = (np.uint64(s) for s in mix_params(b))
    x = (x ^ np.uint64(seed & ((1 << b) - 1))) & mask
    x = x ^ (x >> s1)
    x = (x * np.uint64(C1)) & mask
    x = x ^ (x >> s2)
    x = (x * np.uint64(C2)) & mask
    x = x ^ (x >> s3)
    return x


def mix_scalar(x: int, b: int, seed: int = 0) -> int:
    mask = (1 << b) - 1
    s1, s2, s3 = mix_params(b)
    x = (x ^ (seed & mask)) & mask
    x ^= x >> s1
    x = (x * C1) & mask
    x ^= x >> s2
    x = (x * C2) & mask
    x ^= x >> s3
    return x


def key_bits_for(tuples) -> int:
    """Smallest b with every id < 2^b (at least 1)."""
    t = np.asarray(tuples)
    mx = int(t.max()) if t.size else 0
    return max(1, mx.bit_length())


def coco_levels(tuples, col_order, b, seed: int = 0, segmented: bool = False):
    """CoCo of a relation: returns dict with V (list of arrays: uint32 mixed keys, or the
    raw int64 values when b is None), O (list of int64 arrays, one per level except
    the last), n_unique, n_dup.  segmented: only the low b bits are mixed."""
    t = np.asarray(tuples, dtype=np.int64)
    k = t.shape[1]
    if b is None:
        cols = [t[:, c].copy() for c in col_order]
    elif segmented:
        cols = [mix_segmented(t[:, c], b, seed) for c in col_order]
    else:
        cols = [mix(t[:, c], b, seed) for c in col_order]
    if t.shape[0] == 0:
        return dict(V=[np.zeros(0, np.uint32) for _ in range(k)],
                    O=[np.zeros(1, np.int64) for _ in range(k - 1)], n_unique=0, n_dup=0)
    order = np.lexsort(cols[::-1])
    cols = [c[order] for c in cols]
    # set semantics: keep the first row of each run of equal rows
    keep = np.ones(t.shape[0], dtype=bool)
    same = np.ones(t.shape[0] - 1, dtype=bool)
    for c in cols:
        same &= c[1:] == c[:-1]
    keep[1:] = ~same
    cols = [c[keep] for c in cols]
    nu = cols[0].size
    V, O = [], []
    # new[r][i]: row i starts a new distinct prefix of length r+1
    new_prefix = np.zeros(nu, dtype=bool)
    new_prefix[0] = True
    starts = []
    for r in range(k):
        diff = np.zeros(nu, dtype=bool)
        diff[0] = True
        diff[1:] = cols[r][1:] != cols[r][:-1]
        new_prefix = new_prefix | diff
        idx = np.flatnonzero(new_prefix)
        starts.append(idx)
        V.append(cols[r][idx].astype(np.uint32) if b is not None else cols[r][idx])
    for r in range(k - 1):
        # entry e of level r spans rows starts[r][e] .. starts[r][e+1]-1; its children are
        # the level-(r+1) entries whose start rows fall in that span
        child = np.searchsorted(starts[r + 1], starts[r])
        O.append(np.concatenate([child, [starts[r + 1].size]]).astype(np.int64))
    return dict(V=V, O=O, n_unique=nu, n_dup=int(t.shape[0] - nu))


def partition_ids(tuples, log2_shares, b: int, seed: int = 0):
    """Partition id vector per tuple: s_c = top log2_shares[c] bits of H_b(x_c)."""
    t = np.asarray(tuples, dtype=np.int64)
    ids = []
    for c, k in enumerate(log2_shares):
        h = mix(t[:, c], b, seed)
        ids.append((h >> np.uint64(b - k)).astype(np.int64) if k > 0 else np.zeros(t.shape[0], np.int64))
    return ids


def partition_sizes(tuples, log2_shares, b: int, seed: int = 0):
    """B (partition sizes, flattened lexicographically) and B^pref (exclusive prefix)."""
    ids = partition_ids(tuples, log2_shares, b, seed)
    flat = np.zeros(len(ids[0]) if ids else 0, dtype=np.int64)
    for c, k in enumerate(log2_shares):
        flat = (flat << k) | ids[c]
    B = np.bincount(flat, minlength=1 << sum(log2_shares)).astype(np.int64)
    Bpref = np.concatenate([[0], np.cumsum(B)[:-1]]).astype(np.int64)
    return B, Bpref


def partition_sizes_by_ids(ids, shares):
    """B and exclusive B^pref from explicit partition ids (shares = P_c, any positive ints)."""
    ids = [np.asarray(i, dtype=np.int64) for i in ids]
    flat = np.zeros(ids[0].size, dtype=np.int64)
    for c, p in enumerate(shares):
        flat = flat * p + ids[c]
    total = int(np.prod(shares))
    B = np.bincount(flat, minlength=total).astype(np.int64)
    Bpref = np.concatenate([[0], np.cumsum(B)[:-1]]).astype(np.int64)
    return B.reshape(shares), Bpref.reshape(shares)
