"""ctypes wrapper of the C oracle (gj.c, textbook.c) -- TEST INFRASTRUCTURE ONLY.

``gj`` computes the full conjunctive query of Section 2, Eq. (1), under set
semantics, by Generic Join over sorted tuple arrays.  Rows come back in head
order; ``emit=True`` returns them sorted lexicographically.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["gj.c", "textbook.c"]
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (plain gcc, -O2, OpenMP)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.oracle_gj.restype = ctypes.c_int64
        L.oracle_gj.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P, P,
                                ctypes.c_int64, P, P, ctypes.c_int]
        L.oracle_gj_timed.restype = ctypes.c_int64
        L.oracle_gj_timed.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, ctypes.c_uint64,
                                      ctypes.c_double, P, P, P, P, P, ctypes.c_int]
        L.oracle_digest_rows.restype = None
        L.oracle_digest_rows.argtypes = [P, ctypes.c_int64, ctypes.c_int, P]
        L.textbook_triangles.restype = ctypes.c_int64
        L.textbook_triangles.argtypes = [P, ctypes.c_int64, ctypes.c_int]
        L.textbook_4cliques.restype = ctypes.c_int64
        L.textbook_4cliques.argtypes = [P, ctypes.c_int64, ctypes.c_int]
        L.textbook_4clique_digest.restype = ctypes.c_int64
        L.textbook_4clique_digest.argtypes = [P, ctypes.c_int64, ctypes.c_int, P]
        L.textbook_closed_4walks.restype = ctypes.c_int64
        L.textbook_closed_4walks.argtypes = [P, ctypes.c_int64, ctypes.c_int]
        L.textbook_triangle_stats.restype = ctypes.c_int64
        L.textbook_triangle_stats.argtypes = [P, ctypes.c_int64, ctypes.c_int, P]
        _lib = L
    return _lib


def _as_int64(relations, atoms):
    """int64 row-major copies of the relations; an object given for several atoms of
    the same arity is converted once (the C side then sorts it once per column order)."""
    seen = {}
    out = []
    for r, a in zip(relations, atoms):
        key = (id(r), len(a))
        if key not in seen:
            seen[key] = np.ascontiguousarray(np.asarray(r, dtype=np.int64).reshape(-1, len(a)))
        out.append(seen[key])
    return out


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Result:
    def __init__(self, count, rows=None, digest=None, work=None):
        self.count = count
        self.rows = rows
        self.digest = digest
        self.work = work


def gj(n_vars: int, atoms, relations, order=None, lo=None, hi=None, emit=False,
       digest=False, work=False, threads: int = 0, capacity: int = None) -> Result:
    """Generic Join.

    atoms: list of variable tuples, one per atom (head-order variable ids).
    relations: list of int arrays [rows, arity], one per atom (may repeat objects).
    order: variable order (default 0..n-1).  lo/hi: optional per-variable range
    predicate lo[v] <= x_v < hi[v] on raw ids.  capacity: with emit, the expected
    number of rows if known (one pass instead of a counting pass first; a larger
    result falls back to the two passes).
    """
    L = lib()
    order = list(range(n_vars)) if order is None else list(order)
    arity = np.array([len(a) for a in atoms], dtype=np.int32)
    avars = np.array([v for a in atoms for v in a], dtype=np.int32)
    rels = _as_int64(relations, atoms)
    rows = np.array([r.shape[0] for r in rels], dtype=np.int64)
    ptrs = (ctypes.c_void_p * len(rels))(*[r.ctypes.data for r in rels])
    ordr = np.array(order, dtype=np.int32)
    lo_a = hi_a = None
    if lo is not None:
        lo_a = np.array(lo, dtype=np.int64)
        hi_a = np.array(hi, dtype=np.int64)
    out = None
    cap = 0
    if emit and capacity is not None:
        cap = max(int(capacity), 1)
        out = np.zeros((cap, n_vars), dtype=np.int64)
    elif emit:
        # first pass: count, to size the buffer exactly
        c0 = L.oracle_gj(n_vars, len(atoms), _ptr(arity), _ptr(avars), ptrs, _ptr(rows), _ptr(ordr),
                         _ptr(lo_a) if lo_a is not None else None,
                         _ptr(hi_a) if hi_a is not None else None,
                         None, 0, None, None, threads)
        if c0 < 0:
            raise ValueError("invalid query")
        cap = max(int(c0), 1)
        out = np.zeros((cap, n_vars), dtype=np.int64)
    dg = np.zeros(2, dtype=np.uint64) if digest else None
    wk = np.zeros(n_vars, dtype=np.uint64) if work else None
    c = L.oracle_gj(n_vars, len(atoms), _ptr(arity), _ptr(avars), ptrs, _ptr(rows), _ptr(ordr),
                    _ptr(lo_a) if lo_a is not None else None,
                    _ptr(hi_a) if hi_a is not None else None,
                    _ptr(out) if out is not None else None, cap,
                    _ptr(dg) if dg is not None else None,
                    _ptr(wk) if wk is not None else None, threads)
    if c < 0:
        raise ValueError("invalid query")
    if emit and c > cap:
        return gj(n_vars, atoms, relations, order, lo, hi, emit, digest, work, threads)
    res_rows = None
    if emit:
        res_rows = out[:c]
        if c:
            res_rows = res_rows[np.lexsort(res_rows.T[::-1])]
    return Result(int(c), res_rows,
                  (int(dg[0]), int(dg[1])) if dg is not None else None,
                  [int(x) for x in wk] if wk is not None else None)


def gj_timed(n_vars: int, atoms, relations, budget_s: float, seed: int = 1, order=None, threads: int = 0):
    """Sort once, then run Generic Join over the first variable's values in a seeded
    random order as one parallel loop that takes no new value once budget_s seconds
    have passed.  Returns a dict with sort_s, count (of the values done), wall, busy
    (thread-seconds), runs_done and runs."""
    L = lib()
    order = list(range(n_vars)) if order is None else list(order)
    arity = np.array([len(a) for a in atoms], dtype=np.int32)
    avars = np.array([v for a in atoms for v in a], dtype=np.int32)
    rels = _as_int64(relations, atoms)
    rows = np.array([r.shape[0] for r in rels], dtype=np.int64)
    ptrs = (ctypes.c_void_p * len(rels))(*[r.ctypes.data for r in rels])
    ordr = np.array(order, dtype=np.int32)
    count = np.zeros(1, dtype=np.uint64)
    f = np.zeros(3, dtype=np.float64)            # wall, busy, sort
    done = np.zeros(1, dtype=np.int64)
    n = L.oracle_gj_timed(n_vars, len(atoms), _ptr(arity), _ptr(avars), ptrs, _ptr(rows), _ptr(ordr), seed,
                          budget_s, _ptr(count), _ptr(f[0:1]), _ptr(f[1:2]), _ptr(done), _ptr(f[2:3]), threads)
    if n < 0:
        raise ValueError("invalid query")
    return {"sort_s": float(f[2]), "count": int(count[0]), "wall": float(f[0]), "busy": float(f[1]),
            "runs_done": int(done[0]), "runs": int(n)}


def digest_rows(rows: np.ndarray) -> tuple:
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    n = rows.shape[1] if rows.ndim == 2 else 1
    d = np.zeros(2, dtype=np.uint64)
    lib().oracle_digest_rows(_ptr(rows), rows.shape[0], n, _ptr(d))
    return int(d[0]), int(d[1])


def textbook_triangles(edges, threads: int = 0) -> int:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64))
    return int(lib().textbook_triangles(_ptr(e), e.shape[0], threads))


def textbook_4cliques(edges, threads: int = 0) -> int:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64))
    return int(lib().textbook_4cliques(_ptr(e), e.shape[0], threads))


def textbook_4clique_digest(edges, threads: int = 0):
    """(number of K4, digest of the ordered 4-clique query output) by oriented enumeration."""
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64))
    d = np.zeros(2, dtype=np.uint64)
    k = int(lib().textbook_4clique_digest(_ptr(e), e.shape[0], threads, _ptr(d)))
    return k, (int(d[0]), int(d[1]))


def textbook_cycle4(edges, threads: int = 0) -> int:
    """Ordered 4-cycle query count on a symmetric loop-free relation: the closed
    4-walks, trace(A^4) = sum over (u, w) of c(u, w)^2, c = common neighbours
    (wedge counting in textbook.c)."""
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64))
    if e.shape[0] == 0:
        return 0
    return int(lib().textbook_closed_4walks(_ptr(e), e.shape[0], threads))



def textbook_diamond_twotriangle(edges, threads: int = 0):
    """(ordered diamond count, ordered two-triangle count) on a symmetric loop-free
    relation, in closed form from the triangles on every edge and vertex:
    sum_e 2 t(e)^2 and sum_v (2 t(v))^2 (textbook.c)."""
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64))
    if e.shape[0] == 0:
        return 0, 0
    out = np.zeros(2, dtype=np.uint64)
    if lib().textbook_triangle_stats(_ptr(e), e.shape[0], threads, _ptr(out)) != 0:
        raise ValueError("negative id")
    return int(out[0]), int(out[1])
