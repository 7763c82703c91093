"""Seeded synthetic inputs shared by the tests, the oracle runs and the bench.

This module holds only input generation: a counter-based random stream and
graph generators shaped like the graph workloads of the paper's experiments
(Section 7.1: sparse/skewed, dense/skewed and sparse/uniform graphs).  It
contains none of the join method's arithmetic (no key mixing, no sorting into
a variable order, no intersections), so the GPU path and the CPU oracle can
both consume its arrays without sharing any of the method's code.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used counter-style: the i-th
draw of stream ``seed`` is ``finalize(seed + (i + 1) * GAMMA)`` with the
published golden-ratio increment and finaliser constants.

Every generator returns the *directed, symmetric* tuple array of an
undirected simple graph: each kept undirected edge {u, v} (u != v) appears as
(u, v) and (v, u), rows shuffled so that a consumer really has to sort.
"""

from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1

# Seed conventions: one stream family per workload.
SEED_CONFIG = 0x4843_0000            # + config number (1, 2, 3)
SEED_BATCH = 0x4843_1000_0000        # + query index (batched workload)
SEED_SERVE = 0x4843_2000_0000        # + graph index (served workload)
SHUFFLE_SALT = 0x5348_5546_464C_4521  # separates the shuffle stream


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Draws ``start .. start+count-1`` of the SplitMix64 stream ``seed``."""
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK64) + idx * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_scalar(seed: int, i: int) -> int:
    """Pure-Python single draw, used to pin the vectorised stream."""
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def _unit_double(r: np.ndarray) -> np.ndarray:
    """Top 53 bits of each draw as a double in [0, 1)."""
    return (r >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _bits(x: int) -> int:
    return max(1, int(x).bit_length())


def _draw_until(m: int, seed: int, id_bits: int, draw_batch) -> np.ndarray:
    """Draw candidate edges in generation order until ``m`` unique undirected edges
    (self-loops rejected, {u, v} canonicalised to (min, max)) have been kept; the
    first occurrence of each edge in generation order is the one kept."""
    key_bits = 2 * id_bits
    batch_bits = min(23, 64 - key_bits)
    assert batch_bits >= 10, "ids too wide for the packed dedup"
    # candidates are drawn in batches of 2^k (k <= batch_bits); the batch size never
    # changes which edges are kept, only how many draws are taken at a time
    batch_bits = min(batch_bits, max(10, int(2 * m).bit_length()))
    batch = 1 << batch_bits
    accepted = np.zeros(0, dtype=np.uint64)          # sorted kept keys
    kept = []                                        # kept keys in generation order
    n_kept = 0
    start = 0
    while n_kept < m:
        u, v = draw_batch(start, batch)
        start += batch
        lo = np.minimum(u, v).astype(np.uint64)
        hi = np.maximum(u, v).astype(np.uint64)
        local = np.arange(batch, dtype=np.uint64)
        ok = lo != hi
        key = (lo[ok] << np.uint64(id_bits)) | hi[ok]
        packed = np.sort((key << np.uint64(batch_bits)) | local[ok])
        k_sorted = packed >> np.uint64(batch_bits)
        first = np.ones(k_sorted.size, dtype=bool)
        first[1:] = k_sorted[1:] != k_sorted[:-1]
        cand = packed[first]                          # first occurrence per key
        ck = cand >> np.uint64(batch_bits)
        if accepted.size:
            pos = np.searchsorted(accepted, ck)
            pos = np.minimum(pos, accepted.size - 1)
            cand = cand[accepted[pos] != ck]
        # back to generation order: repack as (local index, key) and sort
        gen = np.sort(((cand & np.uint64(batch - 1)) << np.uint64(key_bits))
                      | (cand >> np.uint64(batch_bits)))
        take = gen[: m - n_kept] & np.uint64((1 << key_bits) - 1)
        kept.append(take)
        n_kept += take.size
        accepted = np.sort(np.concatenate([accepted, take]))
    chosen = np.concatenate(kept)
    u = (chosen >> np.uint64(id_bits)).astype(np.int64)
    v = (chosen & np.uint64((1 << id_bits) - 1)).astype(np.int64)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    nrow = src.size
    idx_bits = _bits(nrow - 1)
    rnd = splitmix64(seed ^ SHUFFLE_SALT, 0, nrow) >> np.uint64(idx_bits)
    order = (np.sort((rnd << np.uint64(idx_bits)) | np.arange(nrow, dtype=np.uint64))
             & np.uint64((1 << idx_bits) - 1)).astype(np.int64)
    return np.stack([src[order], dst[order]], axis=1).astype(np.int32)


def erdos_renyi(n: int, m: int, seed: int) -> np.ndarray:
    """Uniform endpoints; ``n`` must be a power of two.  Candidate i uses draws 2i, 2i+1."""
    assert n & (n - 1) == 0 and n >= 2
    shift = np.uint64(64 - (n.bit_length() - 1))

    def draw(start, count):
        r = splitmix64(seed, 2 * start, 2 * count)
        return (r[0::2] >> shift).astype(np.int64), (r[1::2] >> shift).astype(np.int64)

    return _draw_until(m, seed, _bits(n - 1), draw)


def rmat(scale: int, m: int, seed: int, a=0.57, b=0.19, c=0.19) -> np.ndarray:
    """R-MAT (Chakrabarti, Zhan, Faloutsos 2004): ``scale`` recursive quadrant draws
    per edge, most significant bit first, no noise and no vertex permutation.
    Candidate i uses the 64-bit draws d = ceil(scale/2)*i ..; level l takes the
    high 32 bits of draw l//2 when l is even and the low 32 bits when l is odd,
    and compares them with the cumulative quadrant thresholds (a, a+b, a+b+c)*2^32."""
    ta = np.uint32(int(round(a * 2**32)))
    tb = np.uint32(int(round((a + b) * 2**32)))
    tc = np.uint32(int(round((a + b + c) * 2**32)))
    nd = (scale + 1) // 2

    def draw(start, count):
        r = np.ascontiguousarray(splitmix64(seed, nd * start, nd * count).reshape(count, nd).T)
        u = np.zeros(count, dtype=np.uint32)
        v = np.zeros(count, dtype=np.uint32)
        for lvl in range(scale):
            w = r[lvl // 2]
            q = (w >> np.uint64(32)).astype(np.uint32) if lvl % 2 == 0 else w.astype(np.uint32)
            ubit = q >= tb
            vbit = ((q >= ta) & ~ubit) | (q >= tc)
            u = (u << np.uint32(1)) | ubit
            v = (v << np.uint32(1)) | vbit
        return u.astype(np.int64), v.astype(np.int64)

    return _draw_until(m, seed, scale, draw)


def chung_lu(n: int, m: int, seed: int, beta: float = 2.1) -> np.ndarray:
    """Chung-Lu power-law graph: weights w_i = (i+1)^(-1/(beta-1)); each endpoint
    is drawn with probability proportional to w by inverse CDF in double.
    Candidate i uses draws 2i, 2i+1."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (beta - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]

    def draw(start, count):
        r = splitmix64(seed, 2 * start, 2 * count)
        uu = _unit_double(r)
        idx = np.searchsorted(cdf, uu, side="right")
        np.minimum(idx, n - 1, out=idx)
        return idx[0::2].astype(np.int64), idx[1::2].astype(np.int64)

    return _draw_until(m, seed, _bits(n - 1), draw)


def complete_graph(n: int) -> np.ndarray:
    """Symmetric edge set of K_n without self-loops (unshuffled)."""
    u, v = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = u != v
    return np.stack([u[keep], v[keep]], axis=1).astype(np.int32)


def complete_bipartite(s: int, t: int) -> np.ndarray:
    """Symmetric edge set of K_{s,t}: left ids 0..s-1, right ids s..s+t-1."""
    u, v = np.meshgrid(np.arange(s), np.arange(s, s + t), indexing="ij")
    u, v = u.ravel(), v.ravel()
    return np.stack([np.concatenate([u, v]), np.concatenate([v, u])], axis=1).astype(np.int32)


def random_relation(n_rows: int, domain: int, seed: int, arity: int = 2) -> np.ndarray:
    """Tiny random relation with possible duplicates (for set-semantics tests)."""
    r = splitmix64(seed, 0, n_rows * arity)
    return ((r >> np.uint64(33)) % np.uint64(domain)).astype(np.int32).reshape(n_rows, arity)


# The three single-GPU workloads (sizes from the workload table).
CONFIGS = {
    1: dict(kind="er", n=1 << 12, m=1 << 15, query="triangle"),
    2: dict(kind="rmat", scale=20, m=1 << 24, query="triangle"),
    3: dict(kind="chung_lu", n=1 << 18, m=1 << 22, query="clique4"),
}


def config_graph(cfg: int, scale_down: int = 0) -> np.ndarray:
    """Directed symmetric tuples of workload ``cfg``.  ``scale_down`` divides the
    vertex and edge counts by 2**scale_down (same recipe, smaller instance)."""
    spec = CONFIGS[cfg]
    seed = SEED_CONFIG + cfg
    if spec["kind"] == "er":
        return erdos_renyi(spec["n"] >> scale_down, spec["m"] >> scale_down, seed)
    if spec["kind"] == "rmat":
        return rmat(spec["scale"] - scale_down, spec["m"] >> scale_down, seed)
    return chung_lu(spec["n"] >> scale_down, spec["m"] >> scale_down, seed)


# Query shapes (head variables are 0..n_vars-1; each atom lists its variables).
# Names follow the query table of Section 7.1 (Q1, Q2, Q4, Q6, Q8) and the
# 4-cycle R(a,b), S(b,c), T(c,d), U(d,a) of the served workload.
QUERIES = {
    "triangle": (3, [(0, 1), (1, 2), (0, 2)]),                                  # Q1
    "loop4": (4, [(0, 1), (0, 2), (1, 3), (2, 3)]),                              # Q2
    "cycle4": (4, [(0, 1), (1, 2), (2, 3), (3, 0)]),
    "diamond4": (4, [(0, 1), (0, 2), (1, 3), (2, 3), (1, 2)]),                   # Q4
    "clique4": (4, [(0, 1), (0, 2), (1, 3), (2, 3), (1, 2), (0, 3)]),            # Q6
    "twotriangle": (5, [(0, 1), (0, 2), (1, 2), (2, 3), (2, 4), (3, 4)]),        # Q8
    # ternary atoms (the tensor-kernel queries of the query table)
    "lw": (4, [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]),                     # Loomis-Whitney
    "ct": (4, [(0, 1, 2), (0, 1, 3), (0, 2, 3)]),                                # clover-triangle
}

GRAPH_SALT = 0x4752_4150_4853_4544   # separates a query's graph stream from its spec draws


def _next_pow2(x: float) -> int:
    v = 2
    while v < x:
        v <<= 1
    return v


def batch_spec(n_queries: int = 4096, seed_base: int = SEED_BATCH, log2_lo: float = 10.0, log2_hi: float = 18.0):
    """The batched workload: query q draws 3 numbers from stream seed_base + q:
    shape (triangle or 4-cycle, top bit of draw 0), graph (Erdos-Renyi or R-MAT, top
    bit of draw 1) and m = round(2^U(log2_lo, log2_hi)) unique undirected edges (draw
    2); n = next_pow2(m/8) vertices for Erdos-Renyi, next_pow2(m/16) for R-MAT."""
    out = []
    for q in range(n_queries):
        r = splitmix64(seed_base + q, 0, 3)
        shape = "triangle" if int(r[0]) >> 63 == 0 else "cycle4"
        kind = "er" if int(r[1]) >> 63 == 0 else "rmat"
        u = float(_unit_double(r[2:3])[0])
        m = int(round(2.0 ** (log2_lo + (log2_hi - log2_lo) * u)))
        n = _next_pow2(m / 8.0) if kind == "er" else _next_pow2(m / 16.0)
        n = max(n, 64)
        out.append({"q": q, "query": shape, "kind": kind, "m": m, "n": n, "seed": (seed_base + q) ^ GRAPH_SALT})
    return out


def batch_graph(spec) -> np.ndarray:
    if spec["kind"] == "er":
        return erdos_renyi(spec["n"], spec["m"], spec["seed"])
    return rmat(spec["n"].bit_length() - 1, spec["m"], spec["seed"])


def parallel_graphs(fn, specs, workers: int = 0):
    """fn(spec) for every spec, in parallel processes (each graph is a pure function
    of its spec)."""
    import os
    from concurrent.futures import ProcessPoolExecutor
    if workers <= 0:
        try:
            workers = min(16, len(os.sched_getaffinity(0)))
        except AttributeError:
            workers = min(16, os.cpu_count() or 1)
    if workers == 1 or len(specs) < 2:
        return [fn(s) for s in specs]
    with ProcessPoolExecutor(max_workers=min(workers, len(specs))) as ex:
        return list(ex.map(fn, specs, chunksize=max(1, len(specs) // (4 * workers))))


def batch_graphs(specs, workers: int = 0):
    """Graphs of a batch, generated in parallel processes."""
    return parallel_graphs(batch_graph, specs, workers)


# ---------------------------------------------------------------- served workload
STREAM_SALT = 0x5354_5245_414D_5121   # separates the request stream from the graph streams
SERVE_MIX = (("triangle", 0.5), ("cycle4", 0.3), ("clique4", 0.2))


def serve_graph_specs(n_graphs: int = 16, log2_lo: float = 16.0, log2_hi: float = 24.0):
    """The resident graphs of the served workload: R-MAT graph g has
    m_g = round(2^(log2_lo + (log2_hi - log2_lo) g / (n_graphs - 1))) undirected
    edges and 2^scale vertices with 2^scale = next_pow2(m_g / 16) (edge factor 16)."""
    out = []
    for g in range(n_graphs):
        t = g / (n_graphs - 1) if n_graphs > 1 else 0.0
        m = int(round(2.0 ** (log2_lo + (log2_hi - log2_lo) * t)))
        n = _next_pow2(m / 16.0)
        out.append({"g": g, "kind": "rmat", "m": m, "n": n, "seed": SEED_SERVE + g})
    return out


def serve_graph(spec) -> np.ndarray:
    return rmat(spec["n"].bit_length() - 1, spec["m"], spec["seed"])


def serve_stream(graph_specs, n_requests: int = 20000, qps: float = 2000.0, seed: int = SEED_SERVE,
                 max_log2_width: int = 4):
    """Requests of the served workload, in arrival order.  Request i draws 4 numbers
    from stream seed ^ STREAM_SALT (draws 4i .. 4i+3): the inter-arrival gap
    -ln(1 - U)/qps (a Poisson process), the shape (50% triangle, 30% 4-cycle, 20%
    4-clique), the graph (uniform), and the block of first-variable ids it asks
    about: width 2^u (u uniform in 0..max_log2_width, from the top 24 bits of draw 3),
    start uniform over the graph's vertex ids (from its low 40 bits).  Each request counts the query's tuples whose first
    variable lies in [lo, lo + width)."""
    r = splitmix64(seed ^ STREAM_SALT, 0, 4 * n_requests).reshape(n_requests, 4)
    u = _unit_double(r.reshape(-1)).reshape(n_requests, 4)
    t = np.cumsum(-np.log1p(-u[:, 0]) / qps)
    cum = np.cumsum([p for _, p in SERVE_MIX])
    out = []
    for i in range(n_requests):
        k = int(np.searchsorted(cum, u[i, 1], side="right"))
        shape = SERVE_MIX[min(k, len(SERVE_MIX) - 1)][0]
        g = min(int(u[i, 2] * len(graph_specs)), len(graph_specs) - 1)
        n = graph_specs[g]["n"]
        w = 1 << (((int(r[i, 3]) >> 40) * (max_log2_width + 1)) >> 24)
        lo = int(((int(r[i, 3]) & ((1 << 40) - 1)) * (n - w + 1)) >> 40) if n > w else 0
        out.append({"id": i, "t": float(t[i]), "query": shape, "graph": g, "lo": lo, "hi": lo + w})
    return out


FULL_SALT = 0x4655_4C4C_5155_4552   # separates the full-query stream from the id-block stream
FULL_MAX_EDGES = 150000             # 4-cycle and 4-clique full counts only on graphs this small


def serve_full_stream(graph_specs, n_requests: int = 400, qps: float = 50.0, seed: int = SEED_SERVE,
                      max_edges: int = FULL_MAX_EDGES):
    """Full-query requests over the resident graphs, in arrival order: request i draws
    3 numbers from stream seed ^ FULL_SALT (draws 3i .. 3i+2): the Poisson gap, the
    shape (50% triangle, 30% 4-cycle, 20% 4-clique) and the graph -- uniform over all
    graphs for triangles, over the graphs of at most max_edges undirected edges for
    the 4-variable shapes (their full outputs reach 10^9 and more tuples on the larger
    graphs).  Each request counts the query's whole output on its graph."""
    r = splitmix64(seed ^ FULL_SALT, 0, 3 * n_requests).reshape(n_requests, 3)
    u = _unit_double(r.reshape(-1)).reshape(n_requests, 3)
    t = np.cumsum(-np.log1p(-u[:, 0]) / qps)
    cum = np.cumsum([p for _, p in SERVE_MIX])
    small = [s["g"] for s in graph_specs if s["m"] <= max_edges]
    out = []
    for i in range(n_requests):
        k = int(np.searchsorted(cum, u[i, 1], side="right"))
        shape = SERVE_MIX[min(k, len(SERVE_MIX) - 1)][0]
        pool = list(range(len(graph_specs))) if shape == "triangle" else small
        g = pool[min(int(u[i, 2] * len(pool)), len(pool) - 1)]
        out.append({"id": i, "t": float(t[i]), "query": shape, "graph": g, "lo": 0,
                    "hi": graph_specs[g]["n"], "full": True})
    return out


# ---------------------------------------------------------------- tensor workloads
SEED_TENSOR = 0x4843_3000_0000
TENSOR_U = (0, 1)   # first-attribute domain of the clover-triangle relations (reading of a garbled passage)


def full_product(*sizes) -> np.ndarray:
    """Every tuple of [s_1] x ... x [s_k] (0-based ids), rows in lexicographic order."""
    g = np.stack(np.meshgrid(*[np.arange(s, dtype=np.int32) for s in sizes], indexing="ij"), -1)
    return g.reshape(-1, len(sizes))


def st_dense(n: int = 512, m: int = 4096):
    """ST-Dense: R1..R4 are the full cube [n]^3 (one array serves all four); R5..R7
    are the full U x [m] x [m] with U = TENSOR_U."""
    cube = full_product(n, n, n)
    ct = full_product(m, m)
    ct = np.concatenate([np.concatenate([np.full((ct.shape[0], 1), u, np.int32), ct], 1) for u in TENSOR_U])
    return {"lw": [cube] * 4, "ct": [ct] * 3}


def random_tuples(n_rows: int, sizes, seed: int) -> np.ndarray:
    """n_rows distinct tuples drawn uniformly from [s_1] x ... x [s_k]: candidate i
    takes draw i of stream `seed` and splits it into the k coordinates by
    multiply-shift of successive 21-bit fields; the first n_rows distinct
    candidates in draw order are kept, then rows are shuffled."""
    k = len(sizes)
    out = np.zeros((0, k), np.int64)
    seen = np.zeros(0, np.int64)
    start = 0
    mult = [int(np.prod(sizes[c + 1:])) for c in range(k)]
    while out.shape[0] < n_rows:
        cnt = max(1024, int((n_rows - out.shape[0]) * 1.3))
        r = splitmix64(seed, start, cnt)
        start += cnt
        cols = [(((r >> np.uint64(21 * c)) & np.uint64((1 << 21) - 1)) * np.uint64(sizes[c]) >> np.uint64(21))
                .astype(np.int64) for c in range(k)]
        key = sum(cols[c] * mult[c] for c in range(k))
        allk = np.concatenate([seen, key])
        _, first = np.unique(allk, return_index=True)
        keep = np.zeros(allk.size, bool)
        keep[first] = True
        new = keep[seen.size:]
        add = np.stack(cols, 1)[new]
        add = add[np.argsort(np.flatnonzero(new), kind="stable")]
        out = np.concatenate([out, add])[:n_rows]
        seen = np.concatenate([seen, key[new]])
    rnd = splitmix64(seed ^ SHUFFLE_SALT, 0, out.shape[0])
    return out[np.argsort(rnd, kind="stable")].astype(np.int32)


def st_sparse(n: int = 5120, rows: int = 512 ** 3, m: int = 40960, rows2: int = 4096 ** 2):
    """ST-Sparse: R1..R4 each `rows` distinct random tuples of [n]^3 (density
    rows / n^3 = 0.001 at full size); R5..R7 each `rows2` distinct random pairs of
    [m]^2 under every first-attribute value of TENSOR_U (density 0.01)."""
    lw = [random_tuples(rows, (n, n, n), SEED_TENSOR + j) for j in range(4)]
    ct = []
    for j in range(3):
        parts = []
        for u in TENSOR_U:
            p = random_tuples(rows2, (m, m), SEED_TENSOR + 16 + 4 * j + u)
            parts.append(np.concatenate([np.full((p.shape[0], 1), u, np.int32), p], 1))
        ct.append(np.concatenate(parts))
    return {"lw": lw, "ct": ct}
