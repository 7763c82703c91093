"""Brute-force enumeration of a full conjunctive query -- TEST INFRASTRUCTURE ONLY.

Straight from the definition of Section 2, Eq. (1): a tuple t over the active
domain belongs to Q(D) iff for every atom R_j(X_j) the projection of t on X_j
is a row of R_j.  Enumerates Dom^n, so only for tiny inputs (|Dom|^n <= ~1e6).
"""

from __future__ import annotations

import itertools

import numpy as np


def brute(n_vars: int, atoms, relations, lo=None, hi=None):
    """Sorted list of head-order tuples of Q(D)."""
    sets = [set(map(tuple, np.asarray(r).reshape(-1, len(a)).tolist())) for r, a in zip(relations, atoms)]
    dom = sorted({x for s in sets for row in s for x in row})
    if len(dom) ** n_vars > 2_000_000:
        raise ValueError("instance too large for brute force")
    out = []
    for t in itertools.product(dom, repeat=n_vars):
        if lo is not None and any(not (lo[v] <= t[v] < hi[v]) for v in range(n_vars)):
            continue
        if all(tuple(t[v] for v in a) in s for a, s in zip(atoms, sets)):
            out.append(t)
    return out
