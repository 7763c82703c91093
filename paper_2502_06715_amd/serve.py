"""Serving join queries over resident CoCo indexes, with continuous batching.

A request asks for the count of one query shape (triangle, 4-cycle, 4-clique)
over one resident graph, either restricted to a block of ids of the query's
first variable or whole (a full query: the id block is the graph's whole id
range).  The server:

* keeps one symmetric CoCo per graph resident in HBM (built once, reused by
  every request and every atom of every shape);
* runs ``n_slots`` slot threads; each owns a HIP stream and a library context,
  so the passes of different slots overlap on the device;
* whenever a slot is free it takes the oldest waiting request together with the
  other waiting requests of the same (graph, shape), up to ``max_batch``, and
  counts them all in one hc_join_count_multi pass, one frontier entry per
  request (requests that arrived while earlier passes ran join the next pass:
  continuous batching rather than fixed batches);
* with ``max_weight``, packs a pass only up to that much work (the engine's proxy:
  the bindings of the first level, scaled for the deeper shapes), so that one
  request on a hub vertex does not hold a whole pass of light ones;
* admits a pass only while its memory estimate fits: the budget minus the
  resident indexes is the free memory, and a pass reserves
  hc_join_workspace_bound of its batch until it ends.  A batch that does not
  fit is halved until it does or is one request; a single request that can
  never fit (larger than the whole free budget) is failed.

With ``fuse=False`` every request is its own hc_join_count call (one query per
launch); with ``n_slots=1`` nothing overlaps.  The scheduling logic does not
depend on the device: the engine that estimates and runs passes is injected,
so the admission and batching rules are testable on the CPU.
"""

from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

from . import inputs

Key = Tuple[int, str]   # (graph, shape)


@dataclass
class Request:
    id: int
    graph: int
    query: str
    lo: int
    hi: int
    t_arrival: float = 0.0        # scheduled arrival (seconds from the stream start)
    t_admit: float = 0.0
    t_done: float = 0.0
    count: Optional[int] = None
    error: Optional[str] = None
    batch: int = 0                # size of the pass that answered it
    full: bool = False            # the whole query on its graph (not an id block)
    done: threading.Event = field(default_factory=threading.Event, repr=False)



class GpuEngine:
    """Resident CoCos and one library context (own stream) per slot.

    With ``shared_index`` all graphs live in one segmented CoCo (graph g's ids carry
    g above the vertex bits), so the waiting requests of one shape over every graph
    fuse into one pass; otherwise each graph has its own CoCo and a pass covers one
    (graph, shape)."""

    def __init__(self, graphs: List[np.ndarray], n_slots: int, device: int = 0, shared_index: bool = False,
                 grid_share: float = 0.0):
        """grid_share in (0, 1]: each slot's persistent kernels use at most that share of
        the default grid, leaving compute units free for the passes of other slots."""
        import torch
        from . import batch, hc
        self.hc = hc
        self.torch = torch
        self.dev = torch.device("cuda:%d" % device)
        # default-priority streams, one per slot
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(max(1, n_slots))]
        self.ctxs = [hc.Context(device, stream=s) for s in self.streams]
        if grid_share > 0:
            n_cu = torch.cuda.get_device_properties(self.dev).multi_processor_count
            for c in self.ctxs:
                c.set_grid_limit(max(8, int(8 * n_cu * grid_share)))
        self.est_ctx = hc.Context(device, stream=self.streams[0])   # estimates run under the scheduler lock
        self.cocos = []
        self.index_bytes = 0
        self.shared = shared_index
        self.mix_bits = 0
        with torch.cuda.stream(self.streams[0]):
            if shared_index:
                self.mix_bits = batch.id_bits(graphs)
                rel, seg = batch.union_relation(graphs, self.mix_bits)
                t = torch.from_numpy(rel).to(self.dev)
                self.cocos.append(hc.build_coco(self.ctxs[0], t, [0, 1], key_bits=self.mix_bits, segment_bits=seg,
                                                symmetric=True))
                self.streams[0].synchronize()
                del t
            else:
                for g in graphs:
                    t = torch.from_numpy(np.ascontiguousarray(g)).to(self.dev)
                    self.cocos.append(hc.build_coco(self.ctxs[0], t, [0, 1], symmetric=True))
                    self.streams[0].synchronize()
                    del t
        self.index_bytes = sum(int(c.info.bytes) for c in self.cocos)
        self._q = {name: hc.Query(*inputs.QUERIES[name]) for name in inputs.QUERIES}
        # host-side work proxies: degree prefix sums per graph, and the degree-biased
        # mean degree of a neighbour (sum deg^2 / sum deg) for the deeper levels
        self.deg_prefix = []
        self.kappa = []
        for g in graphs:
            deg = np.bincount(g[:, 0], minlength=int(g.max()) + 1 if g.shape[0] else 1).astype(np.float64)
            self.deg_prefix.append(np.concatenate([[0.0], np.cumsum(deg)]))
            self.kappa.append(float((deg * deg).sum() / max(deg.sum(), 1.0)))

    def weight(self, r: "Request") -> float:
        """Work proxy of a request: the bindings of its first level (sum of the degrees
        of its id block), times the mean degree of a neighbour for the shapes with a
        fourth variable."""
        dp = self.deg_prefix[r.graph]
        lo, hi = min(r.lo, dp.size - 1), min(r.hi, dp.size - 1)
        e1 = dp[hi] - dp[lo] if hi > lo else 0.0
        return max(1.0, e1 * (self.kappa[r.graph] if inputs.QUERIES[r.query][0] > 3 else 1.0))

    def group_key(self, r: "Request"):
        return r.query if self.shared else (r.graph, r.query)

    def _range(self, r: "Request") -> Tuple[int, int]:
        off = (r.graph << self.mix_bits) if self.shared else 0
        return off + r.lo, off + r.hi

    def _args(self, key):
        shape = key if self.shared else key[1]
        coco = self.cocos[0] if self.shared else self.cocos[key[0]]
        n, atoms = inputs.QUERIES[shape]
        return self._q[shape], [coco] * len(atoms), list(range(n))

    def estimate(self, key, n: int, width: int) -> int:
        q, cs, order = self._args(key)
        return self.hc.join_workspace_bound(self.est_ctx, q, cs, order, None, 0, n_queries=n, first_width=width)

    def run(self, slot: int, key, reqs: List["Request"], fused: bool) -> List[int]:
        q, cs, order = self._args(key)
        ctx = self.ctxs[slot]
        ranges = [self._range(r) for r in reqs]
        if fused:
            return [int(c) for c in self.hc.join_count_multi(ctx, q, cs, order, ranges)]
        out = []
        big = 1 << 40
        for lo, hi in ranges:
            n = q.n_vars
            qr = self.hc.Query(n, q.atoms, var_lo=[lo] + [0] * (n - 1), var_hi=[hi] + [big] * (n - 1))
            out.append(self.hc.join_count(ctx, qr, cs, order))
        return out

    def close(self):
        for c in self.cocos:
            c.free()
        self.cocos = []


class Server:
    def __init__(self, engine, budget_bytes: int, n_slots: int = 4, max_batch: int = 256, fuse: bool = True,
                 clock: Callable[[], float] = time.perf_counter, max_weight: Optional[float] = None):
        self.engine = engine
        self.max_weight = max_weight
        self.n_slots = n_slots
        self.max_batch = max_batch if fuse else 1
        self.fuse = fuse
        self.clock = clock
        self.free = int(budget_bytes) - int(getattr(engine, "index_bytes", 0))
        if self.free <= 0:
            raise ValueError("the resident indexes alone exceed the memory budget")
        self.free0 = self.free
        self.peak_reserved = 0
        self.pending: List[Request] = []
        self.cv = threading.Condition()
        self.stop = False
        self.in_flight = 0
        self.passes = 0
        self.t0 = 0.0
        self.threads: List[threading.Thread] = []
        self.errors: List[str] = []

    # ---------------------------------------------------------------- lifecycle
    def start(self, t0: Optional[float] = None):
        self.t0 = self.clock() if t0 is None else t0
        for i in range(self.n_slots):
            th = threading.Thread(target=self._slot, args=(i,), daemon=True)
            th.start()
            self.threads.append(th)

    def close(self):
        with self.cv:
            self.stop = True
            self.cv.notify_all()
        for th in self.threads:
            th.join()

    def submit(self, r: Request):
        with self.cv:
            self.pending.append(r)
            self.cv.notify()

    # ---------------------------------------------------------------- scheduling
    def _take(self):
        """Under the lock: the next pass (key, batch, reserved bytes), or None."""
        while self.pending:
            head = self.pending[0]
            key = self.engine.group_key(head)
            batch = [r for r in self.pending if self.engine.group_key(r) == key][: self.max_batch]
            if self.max_weight is not None and len(batch) > 1:
                # a pass carries at most max_weight of work (its first request always):
                # a heavy request does not hold a whole pass of light ones
                w, keep = 0.0, []
                for r in batch:
                    wr = self.engine.weight(r)
                    if keep and w + wr > self.max_weight:
                        continue
                    keep.append(r)
                    w += wr
                batch = keep
            while True:
                width = max(r.hi - r.lo for r in batch)
                est = int(self.engine.estimate(key, len(batch), max(width, 1)))
                if est <= self.free or len(batch) == 1:
                    break
                batch = batch[: len(batch) // 2]
            if est <= self.free:
                ids = {id(r) for r in batch}
                self.pending = [r for r in self.pending if id(r) not in ids]
                self.free -= est
                self.peak_reserved = max(self.peak_reserved, self.free0 - self.free)
                self.in_flight += 1
                return key, batch, est
            if est > self.free0:
                # can never be admitted: fail it and look at the next request
                self.pending.pop(0)
                head.error = "memory estimate %d bytes exceeds the free budget %d" % (est, self.free0)
                head.t_done = self.clock() - self.t0
                head.done.set()
                continue
            return None   # wait for memory to free up
        return None

    def _slot(self, slot: int):
        while True:
            with self.cv:
                task = self._take()
                while task is None:
                    if self.stop and not self.pending:
                        return
                    self.cv.wait(0.05)
                    task = self._take()
            key, batch, est = task
            t_admit = self.clock() - self.t0
            err = None
            try:
                counts = self.engine.run(slot, key, batch, self.fuse)
            except Exception as e:   # reported per request; the slot keeps serving
                counts, err = [None] * len(batch), "%s: %s" % (type(e).__name__, e)
            t_done = self.clock() - self.t0
            with self.cv:
                self.free += est
                self.in_flight -= 1
                self.passes += 1
                if err:
                    self.errors.append(err)
                self.cv.notify_all()
            for r, c in zip(batch, counts):
                r.t_admit, r.t_done, r.count, r.error, r.batch = t_admit, t_done, c, err, len(batch)
                r.done.set()


def replay(server: Server, requests: List[Request], time_scale: float = 1.0):
    """Open-loop load: submit each request at its scheduled arrival time, wait for
    all answers.  Returns the wall time from the stream start to the last answer."""
    t0 = server.clock()
    server.start(t0)
    for r in requests:
        wait = t0 + r.t_arrival * time_scale - server.clock()
        if wait > 0:
            time.sleep(wait)
        server.submit(r)
    for r in requests:
        r.done.wait()
    end = server.clock() - t0
    server.close()
    return end


def summarize(requests: List[Request], wall_s: float) -> Dict:
    lat = np.array([(r.t_done - r.t_arrival) * 1e3 for r in requests if r.error is None])
    ok = int(lat.size)
    errors: Dict[str, int] = {}
    for r in requests:
        if r.error is not None:
            errors[r.error] = errors.get(r.error, 0) + 1
    return {
        "errors": errors,
        "requests": len(requests),
        "answered": ok,
        "failed": len(requests) - ok,
        "queries_per_s": ok / wall_s if wall_s > 0 else 0.0,
        "p50_ms": float(np.percentile(lat, 50)) if ok else None,
        "p99_ms": float(np.percentile(lat, 99)) if ok else None,
        "mean_batch": float(np.mean([r.batch for r in requests if r.error is None])) if ok else 0.0,
        "wall_s": wall_s,
    }


def requests_from_stream(stream) -> List[Request]:
    return [Request(id=s["id"], graph=s["graph"], query=s["query"], lo=s["lo"], hi=s["hi"], t_arrival=s["t"],
                    full=bool(s.get("full", False)))
            for s in stream]
