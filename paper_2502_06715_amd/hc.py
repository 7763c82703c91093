"""Python binding of libhc.so (the gfx950 Generic Join library).

Argument marshalling only: every step of the join runs in the library's HIP
kernels.  PyTorch supplies device memory (its caching allocator, through the
library's allocator callbacks) and the stream the library orders its work on.
The names follow the C-ABI in include/hc.h.
"""

from __future__ import annotations

import ctypes
import json
import os
import weakref
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhc.so")

HC_OK, HC_ERR_INVALID, HC_ERR_OOM, HC_ERR_OVERFLOW, HC_ERR_DEVICE, HC_ERR_UNSUPPORTED, HC_ERR_CANCELLED = range(7)
HC_I32, HC_I64 = 0, 1
HC_BUILD_SYMMETRIC = 0x1
HC_NO_REWRITE = 0x1
HC_FORCE_MERGE = 0x2
HC_FORCE_GALLOP = 0x4
HC_KEEP_ORDER = 0x8
HC_JOINT_SEARCH = 0x10
HC_PESSIMISTIC = 0x20
HC_CACHE_SHARES = 0x40
HC_EMIT_SORTED = 0x80
HC_SEARCH_WINDOW = 0x000
HC_SEARCH_EXPONENTIAL = 0x100
HC_SEARCH_QUADRATIC = 0x200
HC_SEARCH_LINEAR = 0x300
HC_SEARCH_BY_SIZE = 0x400
SEARCH_METHODS = {"window": HC_SEARCH_WINDOW, "exponential": HC_SEARCH_EXPONENTIAL,
                  "quadratic": HC_SEARCH_QUADRATIC, "linear": HC_SEARCH_LINEAR, "by_size": HC_SEARCH_BY_SIZE}

_STATUS = {1: "HC_ERR_INVALID", 2: "HC_ERR_OOM", 3: "HC_ERR_OVERFLOW", 4: "HC_ERR_DEVICE", 5: "HC_ERR_UNSUPPORTED",
           6: "HC_ERR_CANCELLED"}


class HCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_STATUS.get(status, str(status)), msg))
        self.status = status


class _Query(ctypes.Structure):
    _fields_ = [("n_vars", ctypes.c_int32), ("n_atoms", ctypes.c_int32),
                ("atom_arity", ctypes.c_void_p), ("atom_vars", ctypes.c_void_p),
                ("var_lo", ctypes.c_void_p), ("var_hi", ctypes.c_void_p)]


class CocoInfo(ctypes.Structure):
    _fields_ = [("n_input", ctypes.c_int64), ("n_unique", ctypes.c_int64), ("arity", ctypes.c_int32),
                ("key_bits", ctypes.c_int32), ("mix_seed", ctypes.c_uint64), ("col_order", ctypes.c_int32 * 4),
                ("level_len", ctypes.c_int64 * 4), ("max_children", ctypes.c_int64 * 4),
                ("distinct", ctypes.c_int64 * 4), ("symmetric", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("bytes", ctypes.c_int64), ("mix_bits", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Timing(ctypes.Structure):
    _fields_ = [("leaf_ms", ctypes.c_double), ("leaf_launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("leaf_items", ctypes.c_uint64)]


_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

# exported symbols and their signatures
P, I32, I64, U32, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
SIGNATURES = {
    "hc_ctx_create": (ctypes.c_int, [ctypes.c_int, P, _ALLOC, _FREE, P, P]),
    "hc_ctx_destroy": (None, [P]),
    "hc_last_error": (ctypes.c_char_p, [P]),
    "hc_build_coco": (ctypes.c_int, [P, P, I64, I32, ctypes.c_int, P, I32, U64, U32, P]),
    "hc_build_coco_segmented": (ctypes.c_int, [P, P, I64, I32, ctypes.c_int, P, I32, I32, U64, U32, P]),
    "hc_coco_free": (None, [P]),
    "hc_coco_get_info": (ctypes.c_int, [P, P]),
    "hc_coco_copy_level": (ctypes.c_int, [P, P, I32, P, P]),
    "hc_partition_sizes": (ctypes.c_int, [P, P, P, P, P]),
    "hc_compute_shares": (ctypes.c_int, [P, P, P, I32, U32, P, P]),
    "hc_compute_shares_from_info": (ctypes.c_int, [P, P, I32, U32, P, P]),
    "hc_join_count": (ctypes.c_int, [P, P, P, P, P, U32, P, P]),
    "hc_join_emit": (ctypes.c_int, [P, P, P, P, P, U32, P, I64, P]),
    "hc_join_count_cells": (ctypes.c_int, [P, P, P, P, P, U32, P, P]),
    "hc_join_count_noalloc": (ctypes.c_int, [P, P, P, P, P, U32, P, P, P]),
    "hc_join_count_segments": (ctypes.c_int, [P, P, P, P, I32, U32, P, P]),
    "hc_join_workspace_bound": (ctypes.c_int, [P, P, P, P, P, U32, I64, I64, P]),
    "hc_join_count_multi": (ctypes.c_int, [P, P, P, P, U32, I64, P, P]),
    "hc_join_graph_create": (ctypes.c_int, [P, P, P, P, P, U32, I32, P, I64, I64, I64, P]),
    "hc_join_graph_launch": (ctypes.c_int, [P]),
    "hc_join_graph_result": (ctypes.c_int, [P, P, P, P, P]),
    "hc_join_graph_destroy": (None, [P]),
    "hc_plan_describe": (ctypes.c_int, [P, P, U32, P, ctypes.c_size_t]),
    "hc_plan_cost_from_info": (ctypes.c_int, [P, P, P, P, U32, P, P]),
    "hc_ctx_set_profiling": (ctypes.c_int, [P, ctypes.c_int]),
    "hc_ctx_set_grid_limit": (ctypes.c_int, [P, I32]),
    "hc_ctx_cancel": (ctypes.c_int, [P, I32]),
    "hc_ctx_get_timing": (ctypes.c_int, [P, P]),
}

_lib = None


def lib():
    """Load libhc.so.  Raises if it has not been built: there is no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libhc.so is not built; run `python -m paper_2502_06715_amd.build_lib`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


@dataclass
class Query:
    """Full conjunctive query: variables 0..n_vars-1 (head order), atoms as variable tuples."""
    n_vars: int
    atoms: Sequence[Sequence[int]]
    var_lo: Optional[Sequence[int]] = None
    var_hi: Optional[Sequence[int]] = None

    def c(self) -> _Query:
        ar = np.array([len(a) for a in self.atoms], dtype=np.int32)
        av = np.array([v for a in self.atoms for v in a], dtype=np.int32)
        q = _Query(self.n_vars, len(self.atoms), ar.ctypes.data, av.ctypes.data, None, None)
        keep = [ar, av]
        if self.var_lo is not None:
            lo = np.array(self.var_lo, dtype=np.int64)
            hi = np.array(self.var_hi, dtype=np.int64)
            q.var_lo, q.var_hi = lo.ctypes.data, hi.ctypes.data
            keep += [lo, hi]
        q._keep = keep   # the arrays live as long as the struct (thread-safe for shared queries)
        return q


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


class Context:
    """hc_ctx on a torch device and stream, allocating through torch's caching allocator."""

    def __init__(self, device: int = 0, stream=None, use_torch_allocator: bool = True, max_bytes: int = 0):
        """max_bytes > 0 caps the device memory this context's calls may hold at once
        (through torch's allocator): a request beyond it is refused, and the call
        fails with HC_ERR_OOM."""
        import torch
        self._torch = torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        sptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        self._sptr = sptr
        self.max_bytes = int(max_bytes)
        self.live = {}
        self._graphs = weakref.WeakSet()   # captured joins on this context, released before it
        self.alloc_error = None   # why the allocator last refused a request
        self.n_allocs = 0         # requests the library made through this context's allocator
        if use_torch_allocator:
            def _alloc(nbytes, user):
                self.n_allocs += 1
                if self.max_bytes and sum(self.live.values()) + int(nbytes) > self.max_bytes:
                    self.alloc_error = "context cap of %d bytes" % self.max_bytes
                    return None
                try:
                    p = torch.cuda.caching_allocator_alloc(int(nbytes), device, sptr)
                except Exception as e:
                    self.alloc_error = "%s: %s" % (type(e).__name__, str(e).splitlines()[0] if str(e) else "")
                    return None
                if self.max_bytes:
                    self.live[p] = int(nbytes)
                return p

            def _free(ptr, user):
                self.live.pop(ptr, None)
                cuda = getattr(torch, "cuda", None)
                if cuda is None:   # interpreter shutdown: torch is gone, the process ends
                    return
                cuda.caching_allocator_delete(ptr)

            self._cb = (_ALLOC(_alloc), _FREE(_free))
        else:
            self._cb = (_ALLOC(), _FREE())
        h = ctypes.c_void_p()
        st = lib().hc_ctx_create(device, ctypes.c_void_p(sptr), self._cb[0], self._cb[1], None, ctypes.byref(h))
        if st != HC_OK:
            raise HCError(st, "hc_ctx_create failed")
        self.h = h

    def check(self, st: int):
        if st != HC_OK:
            msg = lib().hc_last_error(self.h).decode()
            if st == HC_ERR_OOM and self.alloc_error:
                msg += " (%s)" % self.alloc_error
                self.alloc_error = None
            raise HCError(st, msg)

    def cancel(self, on: bool = True):
        """Raise (or withdraw) the context's cancel request; safe from another thread."""
        st = lib().hc_ctx_cancel(self.h, 1 if on else 0)
        if st != HC_OK:
            raise HCError(st, "hc_ctx_cancel failed")

    def set_grid_limit(self, max_workgroups: int):
        """Persistent kernels of this context launch at most max_workgroups workgroups
        (0: the default, 8 per compute unit)."""
        self.check(lib().hc_ctx_set_grid_limit(self.h, int(max_workgroups)))

    def set_profiling(self, on: bool):
        lib().hc_ctx_set_profiling(self.h, 1 if on else 0)

    def timing(self) -> Timing:
        t = Timing()
        lib().hc_ctx_get_timing(self.h, ctypes.byref(t))
        return t

    def close(self):
        if getattr(self, "h", None):
            for g in list(getattr(self, "_graphs", ())):
                g.free()   # a graph uses the context's stream and allocator
            lib().hc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Coco:
    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self.h = handle
        info = CocoInfo()
        lib().hc_coco_get_info(self.h, ctypes.byref(info))
        self.info = info

    def free(self):
        if self.h:
            lib().hc_coco_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_coco(ctx: Context, tuples, col_order=None, key_bits: int = 0, seed: int = 0,
               symmetric: bool = False, segment_bits: int = 0) -> Coco:
    """hc_build_coco on a CUDA tensor [n, arity] of int32/int64.  With segment_bits > 0
    (hc_build_coco_segmented) key_bits is the number of mixed low bits and the ids
    carry a segment number above them."""
    torch = ctx._torch
    t = tuples
    assert t.is_cuda and t.dim() == 2, "tuples must be a 2-D CUDA tensor"
    t = t.contiguous()
    dt = {torch.int32: HC_I32, torch.int64: HC_I64}[t.dtype]
    arity = t.shape[1]
    co = _i32(list(range(arity)) if col_order is None else col_order)
    h = ctypes.c_void_p()
    flags = HC_BUILD_SYMMETRIC if symmetric else 0
    if segment_bits:
        st = lib().hc_build_coco_segmented(ctx.h, ctypes.c_void_p(t.data_ptr()), t.shape[0], arity, dt,
                                           co.ctypes.data, key_bits, segment_bits, seed & 0xFFFFFFFFFFFFFFFF,
                                           flags, ctypes.byref(h))
    else:
        st = lib().hc_build_coco(ctx.h, ctypes.c_void_p(t.data_ptr()), t.shape[0], arity, dt, co.ctypes.data,
                                 key_bits, seed & 0xFFFFFFFFFFFFFFFF, flags, ctypes.byref(h))
    ctx.check(st)
    return Coco(ctx, h)


def coco_level(ctx: Context, coco: Coco, level: int):
    n = coco.info.level_len[level]
    vals = np.zeros(max(n, 1), dtype=np.uint32)
    offs = np.zeros(n + 1, dtype=np.int32) if level + 1 < coco.info.arity else None
    ctx.check(lib().hc_coco_copy_level(ctx.h, coco.h, level, vals.ctypes.data,
                                       offs.ctypes.data if offs is not None else None))
    return vals[:n], offs


def partition_sizes(ctx: Context, coco: Coco, log2_shares):
    ls = _i32(log2_shares)
    total = 1 << int(ls.sum())
    B = np.zeros(total, dtype=np.int64)
    Bp = np.zeros(total, dtype=np.int64)
    ctx.check(lib().hc_partition_sizes(ctx.h, coco.h, ls.ctypes.data, B.ctypes.data, Bp.ctypes.data))
    return B, Bp


def _handles(cocos):
    return (ctypes.c_void_p * len(cocos))(*[c.h for c in cocos])


def compute_shares(ctx: Context, q: Query, cocos, log2_total_P: int, flags: int = 0, order=None):
    order_a = _i32(order if order is not None else list(range(q.n_vars)))
    shares = np.zeros(q.n_vars, dtype=np.int32)
    if order is not None:
        flags |= HC_KEEP_ORDER
    qc = q.c()
    ctx.check(lib().hc_compute_shares(ctx.h, ctypes.byref(qc), _handles(cocos), log2_total_P, flags,
                                      order_a.ctypes.data, shares.ctypes.data))
    return order_a.tolist(), shares.tolist()


def compute_shares_from_info(q: Query, infos, log2_total_P: int, flags: int = 0, order=None):
    """Host-only share decision from CocoInfo structs (no GPU needed)."""
    order_a = _i32(order if order is not None else list(range(q.n_vars)))
    shares = np.zeros(q.n_vars, dtype=np.int32)
    if order is not None:
        flags |= HC_KEEP_ORDER
    arr = (CocoInfo * len(infos))(*infos)
    qc = q.c()
    st = lib().hc_compute_shares_from_info(ctypes.byref(qc), arr, log2_total_P, flags, order_a.ctypes.data,
                                           shares.ctypes.data)
    if st != HC_OK:
        raise HCError(st, "hc_compute_shares_from_info failed")
    return order_a.tolist(), shares.tolist()


def join_count(ctx: Context, q: Query, cocos, order, log2_shares=None, flags: int = 0, digest: bool = False):
    order_a = _i32(order)
    sh = _i32(log2_shares) if log2_shares is not None else None
    cnt = ctypes.c_uint64(0)
    dg = (ctypes.c_uint64 * 2)()
    qc = q.c()
    ctx.check(lib().hc_join_count(ctx.h, ctypes.byref(qc), _handles(cocos), order_a.ctypes.data,
                                  sh.ctypes.data if sh is not None else None, flags, ctypes.byref(cnt),
                                  dg if digest else None))
    if digest:
        return int(cnt.value), (int(dg[0]), int(dg[1]))
    return int(cnt.value)


def join_count_noalloc(ctx: Context, q: Query, cocos, order, log2_shares=None, flags: int = 0,
                       digest: bool = False):
    """hc_join_count_noalloc: the count (and digest) with every device buffer taken from
    the library's fixed per-GPU scratch array.  Returns (count, digest or None, bytes of
    scratch used)."""
    order_a = _i32(order)
    sh = _i32(log2_shares) if log2_shares is not None else None
    cnt = ctypes.c_uint64(0)
    used = ctypes.c_uint64(0)
    dg = (ctypes.c_uint64 * 2)()
    qc = q.c()
    ctx.check(lib().hc_join_count_noalloc(ctx.h, ctypes.byref(qc), _handles(cocos), order_a.ctypes.data,
                                          sh.ctypes.data if sh is not None else None, flags, ctypes.byref(cnt),
                                          dg if digest else None, ctypes.byref(used)))
    return int(cnt.value), ((int(dg[0]), int(dg[1])) if digest else None), int(used.value)


def join_count_cells(ctx: Context, q: Query, cocos, order, log2_shares, flags: int = 0):
    """Per-cell counts (numpy uint64, 2^sum(shares) entries) and the total."""
    order_a = _i32(order)
    sh = _i32(log2_shares)
    cells = np.zeros(1 << int(sh.sum()), dtype=np.uint64)
    cnt = ctypes.c_uint64(0)
    qc = q.c()
    ctx.check(lib().hc_join_count_cells(ctx.h, ctypes.byref(qc), _handles(cocos), order_a.ctypes.data,
                                        sh.ctypes.data, flags, cells.ctypes.data, ctypes.byref(cnt)))
    return cells, int(cnt.value)


def join_count_segments(ctx: Context, q: Query, cocos, order, log2_extra: int = 0, flags: int = 0):
    """Per-segment counts (numpy uint64, 2^segment_bits entries) of segmented CoCos, and
    the total; the first variable of the order is split into 2^log2_extra cells per
    segment."""
    order_a = _i32(order)
    seg = int(cocos[0].info.key_bits - cocos[0].info.mix_bits)
    counts = np.zeros(1 << seg, dtype=np.uint64)
    cnt = ctypes.c_uint64(0)
    qc = q.c()
    ctx.check(lib().hc_join_count_segments(ctx.h, ctypes.byref(qc), _handles(cocos), order_a.ctypes.data,
                                           int(log2_extra), flags, counts.ctypes.data, ctypes.byref(cnt)))
    return counts, int(cnt.value)


def join_workspace_bound(ctx: Context, q: Query, cocos, order, log2_shares=None, flags: int = 0,
                         n_queries: int = 0, first_width: int = 0) -> int:
    """Upper bound (bytes) of the device memory of one count call (n_queries = 0) or
    of one join_count_multi call over n_queries ranges at most first_width wide."""
    order_a = _i32(order)
    sh = _i32(log2_shares) if log2_shares is not None else None
    out = ctypes.c_uint64(0)
    qc = q.c()
    ctx.check(lib().hc_join_workspace_bound(ctx.h, ctypes.byref(qc), _handles(cocos), order_a.ctypes.data,
                                            sh.ctypes.data if sh is not None else None, flags, int(n_queries),
                                            int(first_width), ctypes.byref(out)))
    return int(out.value)


def join_count_multi(ctx: Context, q: Query, cocos, order, ranges, flags: int = 0) -> np.ndarray:
    """Counts of q with its first variable restricted to each [lo, hi) of ranges,
    in one pass (numpy uint64 array)."""
    order_a = _i32(order)
    r = np.ascontiguousarray(np.asarray(ranges, dtype=np.int64).reshape(-1, 2))
    counts = np.zeros(max(r.shape[0], 1), dtype=np.uint64)
    qc = q.c()
    ctx.check(lib().hc_join_count_multi(ctx.h, ctypes.byref(qc), _handles(cocos), order_a.ctypes.data, flags,
                                        r.shape[0], r.ctypes.data, counts.ctypes.data))
    return counts[: r.shape[0]]


def join_emit(ctx: Context, q: Query, cocos, order, log2_shares=None, flags: int = 0, capacity: int = None,
              out=None):
    """Returns (rows tensor [n_out, n_vars] view, n_out).  Raises HCError(HC_ERR_OVERFLOW)
    (with .n_out set) when the result exceeds the capacity."""
    torch = ctx._torch
    dt = torch.int64 if cocos[0].info.dtype == HC_I64 else torch.int32
    if out is None:
        cap = capacity if capacity is not None else 0
        out = torch.empty((max(cap, 1), q.n_vars), dtype=dt, device="cuda:%d" % ctx.device)
    else:
        cap = out.shape[0] if capacity is None else capacity
    order_a = _i32(order)
    sh = _i32(log2_shares) if log2_shares is not None else None
    n_out = ctypes.c_int64(0)
    qc = q.c()
    st = lib().hc_join_emit(ctx.h, ctypes.byref(qc), _handles(cocos), order_a.ctypes.data,
                            sh.ctypes.data if sh is not None else None, flags, ctypes.c_void_p(out.data_ptr()),
                            cap, ctypes.byref(n_out))
    if st == HC_ERR_OVERFLOW:
        e = HCError(st, lib().hc_last_error(ctx.h).decode())
        e.n_out = int(n_out.value)
        raise e
    ctx.check(st)
    return out[: n_out.value], int(n_out.value)


class JoinGraph:
    """hc_join_graph_*: a join recorded once as a fixed launch sequence in a HIP graph
    (frontier sizes stay on the device) and replayed.  mode "count", "cells" (per-cell
    counts in groups of 2^cell_group cells) or "emit" (rows into `out`, a device tensor
    [capacity, n_vars] that the graph keeps writing to)."""

    def __init__(self, ctx: Context, q: Query, cocos, order, log2_shares=None, flags: int = 0, mode: str = "count",
                 cell_group: int = 0, out=None, frontier_cap: int = 0, item_cap: int = 0):
        assert mode in ("count", "cells", "emit")
        self.ctx = ctx
        self.mode = mode
        self._keep = (list(cocos), out)
        order_a = _i32(order)
        sh = _i32(log2_shares) if log2_shares is not None else np.zeros(q.n_vars, np.int32)
        self.n_cells = (1 << int(sh.sum())) >> (cell_group if mode == "cells" else 0)
        self.out = out
        cap = int(out.shape[0]) if (mode == "emit" and out is not None) else 0
        h = ctypes.c_void_p()
        qc = q.c()
        ctx.check(lib().hc_join_graph_create(ctx.h, ctypes.byref(qc), _handles(cocos), order_a.ctypes.data,
                                             sh.ctypes.data, flags, cell_group if mode == "cells" else -1,
                                             ctypes.c_void_p(out.data_ptr()) if mode == "emit" else None, cap,
                                             int(frontier_cap), int(item_cap), ctypes.byref(h)))
        self.h = h
        ctx._graphs.add(self)

    def launch(self):
        """Enqueue one replay on the context's stream."""
        self.ctx.check(lib().hc_join_graph_launch(self.h))

    def result(self):
        """Wait for the last replay: (count, per-cell counts or emitted rows or None,
        replayed) -- replayed is False when a capacity was exceeded and the eager path
        computed the result."""
        cnt = ctypes.c_uint64(0)
        n_out = ctypes.c_int64(0)
        rep = ctypes.c_int32(0)
        cells = np.zeros(self.n_cells, dtype=np.uint64) if self.mode == "cells" else None
        st = lib().hc_join_graph_result(self.h, ctypes.byref(cnt), cells.ctypes.data if cells is not None else None,
                                        ctypes.byref(n_out), ctypes.byref(rep))
        if st == HC_ERR_OVERFLOW:
            e = HCError(st, lib().hc_last_error(self.ctx.h).decode())
            e.n_out = int(n_out.value)
            raise e
        self.ctx.check(st)
        extra = cells if self.mode == "cells" else (self.out[: n_out.value] if self.mode == "emit" else None)
        return int(cnt.value), extra, bool(rep.value)

    def run(self):
        self.launch()
        return self.result()

    def free(self):
        # (a closed context has released the graph already)
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            lib().hc_join_graph_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def plan_cost_from_info(q: Query, infos, order, log2_shares=None, flags: int = 0):
    """(total, per-level costs) of one plan under the cost model (host-only)."""
    arr = (CocoInfo * len(infos))(*infos)
    order_a = _i32(order)
    sh = _i32(log2_shares) if log2_shares is not None else None
    per = np.zeros(q.n_vars, dtype=np.float64)
    tot = ctypes.c_double(0)
    qc = q.c()
    st = lib().hc_plan_cost_from_info(ctypes.byref(qc), arr, order_a.ctypes.data,
                                      sh.ctypes.data if sh is not None else None, flags, per.ctypes.data,
                                      ctypes.byref(tot))
    if st != HC_OK:
        raise HCError(st, "hc_plan_cost_from_info failed")
    return float(tot.value), per


def plan_describe(q: Query, order, flags: int = 0) -> dict:
    buf = ctypes.create_string_buffer(1 << 16)
    order_a = _i32(order)
    qc = q.c()
    st = lib().hc_plan_describe(ctypes.byref(qc), order_a.ctypes.data, flags, buf, len(buf))
    if st != HC_OK:
        raise HCError(st, "hc_plan_describe failed")
    return json.loads(buf.value.decode())
