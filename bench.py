"""Benchmark of the Generic Join hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2] [--no-cpu-baseline]

A step is one pass of the whole hot path over the workload, with the input
tuples already resident in HBM: CoCo build (key mix, radix sort, levels),
share/order decision, and the HyperCube-partitioned Generic Join count.
Default workload: triangle query Q(a,b,c) = R(a,b), S(b,c), T(a,c) with
R = S = T the symmetric edge set of an R-MAT graph (scale 20, a,b,c,d =
0.57, 0.19, 0.19, 0.05, 2^24 undirected edges -> 2^25 int32 tuples), shares
over all three variables from the cost model with P = 2^12 cells.

Prints one JSON line: output tuples/s (the count divided by the step time),
the roofline of the dominant kernel (the deepest Generic Join level, timed
with HIP events on the library's stream), and the CPU oracle timed on a
bounded sample of the same workload on this host's cores.
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CLOCK_HZ = 2.4e9


def _source_hash():
    """Hash of the sources that decide the leaf kernel's work: its code and the share
    decision (a different share vector changes the kernel's traffic)."""
    h = hashlib.sha256()
    for f in ["join.hip", "prim_dev.h", "hc_internal.h", "plan.cpp"]:
        h.update(open(os.path.join(ROOT, "paper_2502_06715_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_threads():
    try:
        return min(16, len(os.sched_getaffinity(0)))
    except AttributeError:
        return min(16, os.cpu_count() or 1)


def _workload(cfg):
    from paper_2502_06715_amd import inputs
    spec = inputs.CONFIGS[cfg]
    if spec["kind"] == "rmat":
        desc = ("triangle query, R=S=T symmetric edge set of R-MAT scale %d (a,b,c,d = 0.57,0.19,0.19,0.05), "
                "2^%d undirected edges (2^%d int32 tuples), HyperCube shares over all 3 variables, count"
                % (spec["scale"], spec["m"].bit_length() - 1, spec["m"].bit_length()))
        return desc, spec["scale"], "triangle"
    if spec["kind"] == "er":
        desc = ("triangle query, R=S=T symmetric edge set of an Erdos-Renyi graph, 2^%d vertices, 2^%d "
                "undirected edges, plain Generic Join (1 share per variable), full output + count"
                % (spec["n"].bit_length() - 1, spec["m"].bit_length() - 1))
        return desc, spec["n"].bit_length() - 1, "triangle"
    desc = ("4-clique query over 6 atoms on one Chung-Lu graph (beta 2.1), 2^%d vertices, 2^%d undirected "
            "edges, count" % (spec["n"].bit_length() - 1, spec["m"].bit_length() - 1))
    return desc, spec["n"].bit_length() - 1, "clique4"


def cpu_baseline(E, n_vars, atoms, full_count, budget_s=15.0, budget_1t=5.0, seed=1):
    """The oracle on this host's cores (its OpenMP threads = the host threads this
    process may use, at most 16), on a bounded sample of the workload: sort once, then
    Generic Join over the first variable's values in a seeded random order (so the
    sample is a uniform one of the values, with the whole job's mix of light and heavy
    ones) as one parallel loop that takes no new value after budget_s seconds.  The
    job's time is the sort plus the loop's busy thread-seconds over the thread count,
    scaled by the sample's share of the output (a thread still in a heavy value at the
    deadline finishes it alone; its busy time counts that value, the wall time would
    count it for every thread).  A one-thread sample is timed beside it.
    (`bench.py --cpu-full` times the whole job at the same thread count: about a
    minute.)"""
    from oracle import oracle
    threads = _host_threads()
    r = oracle.gj_timed(n_vars, atoms, [E] * len(atoms), budget_s, seed=seed, threads=threads)
    frac = r["count"] / full_count if full_count else 0.0
    t_job = r["sort_s"] + (r["busy"] / threads / frac if frac > 0 else float("inf"))
    r1 = oracle.gj_timed(n_vars, atoms, [E] * len(atoms), budget_1t, seed=seed, threads=1)
    f1 = r1["count"] / full_count if full_count else 0.0
    t1 = r1["sort_s"] + (r1["busy"] / f1 if f1 > 0 else float("inf"))
    return {
        "value": full_count / t_job if t_job > 0 else 0.0,
        "unit": "tuples/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": _cpu_model(),
        "one_thread_value": full_count / t1 if t1 > 0 else 0.0,
        "sample": ("oracle (C, OpenMP, %d threads) sort+dedup of every atom (%.1f s), then Generic Join over "
                   "%d of %d first-variable values in seeded random order (%.1f s wall, %.1f busy thread-seconds, "
                   "%.2f%% of the output): %.1f s per full job; one thread: %d values, %.2f%% of the output, "
                   "%.1f s per full job" % (threads, r["sort_s"], r["runs_done"], r["runs"], r["wall"],
                                            r["busy"], 100 * frac, t_job, r1["runs_done"], 100 * f1, t1)),
    }


def bench_batch(args):
    """Batched workload: 4096 independent triangle / 4-cycle queries, each on its own
    ER or R-MAT graph with log-uniform 2^10..2^18 edges.  The queries are grouped by
    shape and size class (batch.size_class: the log2 of their edge count); a step
    builds one segmented CoCo per group over the union of its graphs and runs one
    fused count per group, with the extra split and the search method the autotuner
    picked for that group; the per-query counts are checked against the oracle's.
    The one-query-per-launch baseline (build, shares, count per query) runs on the
    same queries and device."""
    import torch
    from paper_2502_06715_amd import batch, hc, inputs

    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "batch_config4.json")))
    specs = inputs.batch_spec(gold["n_queries"])
    expect = np.array([int(c) for c in gold["counts"]], dtype=np.uint64)
    t0 = time.time()
    graphs = inputs.batch_graphs(specs)
    print("# generated %d graphs in %.1f s" % (len(graphs), time.time() - t0), file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    ctx = hc.Context(0)
    shapes = ["triangle", "cycle4"]
    groups = {}
    for shape in shapes:
        for cls in range(len(batch.SIZE_CLASSES) + 1):
            idx = np.array([i for i, s in enumerate(specs)
                            if s["query"] == shape and batch.size_class(s["m"]) == cls], dtype=np.int64)
            if idx.size == 0:
                continue
            gs = [graphs[i] for i in idx]
            mb = batch.id_bits(gs)
            rel, seg = batch.union_relation(gs, mb)
            groups[(shape, cls)] = dict(idx=idx, mb=mb, seg=seg, rel=torch.from_numpy(rel).to(dev), n=len(gs))
    torch.cuda.synchronize()
    # the autotuner times its candidates on every 8th query of each group
    tune = batch.Autotune()
    for key, g in groups.items():
        shape = key[0]
        sub = [graphs[i] for i in g["idx"][::8]]
        srel, sseg = batch.union_relation(sub, g["mb"])
        sdev = torch.from_numpy(srel).to(dev)
        c = hc.build_coco(ctx, sdev, [0, 1], key_bits=g["mb"], segment_bits=sseg, symmetric=True)
        tune.pick(key, lambda x, m: batch.count_batched(ctx, shape, sdev, len(sub), g["mb"], sseg,
                                                        extra_bits=x, coco=c, method=m))
        c.free()
        del sdev
        g["extra"], g["method"] = tune.choice[key]
        print("# autotune %s class %d (%d queries): extra split bits %d, search %s (timings %s)"
              % (shape, key[1], g["n"], g["extra"], g["method"],
                 {"%d/%s" % k[1]: round(v, 4) for k, v in tune.timings.items() if k[0] == key}),
              file=sys.stderr, flush=True)

    def step():
        got = np.zeros(len(specs), dtype=np.uint64)
        for (shape, _), g in groups.items():
            got[g["idx"]] = batch.count_batched(ctx, shape, g["rel"], g["n"], g["mb"], g["seg"],
                                                extra_bits=g["extra"], method=g["method"])
        return got

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    ms_batched = 1000.0 * (time.perf_counter() - t1) / args.steps
    for r in res:
        bad = np.flatnonzero(r != expect)
        if bad.size:
            print("batched count mismatch at queries %s" % bad[:8].tolist(), file=sys.stderr)
            sys.exit(1)

    # one query per launch: build + shares + count of every query on its own
    per_dev = [torch.from_numpy(np.ascontiguousarray(g)).to(dev) for g in graphs]
    torch.cuda.synchronize()
    seq = np.zeros(len(specs), dtype=np.uint64)
    t2 = time.perf_counter()
    for (shape, _), g in groups.items():
        seq[g["idx"]] = batch.count_sequential(ctx, shape, [per_dev[i] for i in g["idx"]])
    torch.cuda.synchronize()
    ms_seq = 1000.0 * (time.perf_counter() - t2)
    if np.any(seq != expect):
        print("one-query-per-launch count mismatch", file=sys.stderr)
        sys.exit(1)
    nq = len(specs)
    out = {
        "metric": "queries/s (batched triangle / 4-cycle workload)",
        "value": nq / (ms_batched / 1000.0),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_batched, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "4096 independent triangle / 4-cycle queries, each on its own Erdos-Renyi or "
                               "R-MAT graph, undirected edges log-uniform in [2^10, 2^18], int32 ids",
                   "size_classes_log2_edges": list(batch.SIZE_CLASSES),
                   "queries": {"%s/%d" % k: int(g["n"]) for k, g in groups.items()},
                   "tuples": int(sum(g["rel"].shape[0] for g in groups.values())),
                   "extra_split_bits": {"%s/%d" % k: int(g["extra"]) for k, g in groups.items()},
                   "search": {"%s/%d" % k: g["method"] for k, g in groups.items()}},
        "one_query_per_launch": {"value": nq / (ms_seq / 1000.0), "unit": "queries/s",
                                 "ms_total": round(ms_seq, 3)},
        "speedup_vs_one_query_per_launch": round(ms_seq / ms_batched, 3),
        "roofline": None,
        "resident": _batch_resident(ctx, groups, graphs, expect, max(args.steps, 2)),
    }
    print(json.dumps(out), flush=True)


def _batch_resident(ctx, groups, graphs, expect, steps):
    """The batched joins over segmented CoCos built once (resident indexes): a step
    of eager fused counts against a step where each group runs as the autotuner
    chose it: a captured join (hc_join_graph_*) when its frontier capacities
    (batch.graph_caps) fit and a replay beats the eager count, else eager; per-query
    counts checked on every step."""
    import torch
    from paper_2502_06715_amd import batch, hc
    cocos, graphs_of, choice = {}, {}, {}
    for key, g in groups.items():
        cocos[key] = hc.build_coco(ctx, g["rel"], [0, 1], key_bits=g["mb"], segment_bits=g["seg"], symmetric=True)
        caps = batch.graph_caps(key[0], [graphs[i] for i in g["idx"]])
        choice["%s/%d" % key] = "eager (capacities)"
        if caps is None:
            continue
        bg = batch.BatchGraph(ctx, key[0], cocos[key], g["n"], g["extra"], caps)
        # the autotuner's choice for the class: the captured join when a replay is the
        # faster of the two (both timed once after a warm-up call)
        tm = {}
        for name in ("eager", "captured"):
            for rep in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if name == "eager":
                    batch.count_batched(ctx, key[0], g["rel"], g["n"], g["mb"], g["seg"], extra_bits=g["extra"],
                                        coco=cocos[key], method=g["method"])
                else:
                    bg.launch()
                    bg.result()
                tm[name] = time.perf_counter() - t0
        choice["%s/%d" % key] = "captured" if tm["captured"] < tm["eager"] else "eager"
        choice["%s/%d" % key] += " (%.2f / %.2f ms)" % (1e3 * tm["captured"], 1e3 * tm["eager"])
        if tm["captured"] < tm["eager"]:
            graphs_of[key] = bg
        else:
            bg.free()

    def eager_step():
        got = np.zeros(expect.shape[0], dtype=np.uint64)
        for key, g in groups.items():
            got[g["idx"]] = batch.count_batched(ctx, key[0], g["rel"], g["n"], g["mb"], g["seg"],
                                                extra_bits=g["extra"], coco=cocos[key], method=g["method"])
        return got

    def graph_step():
        got = np.zeros(expect.shape[0], dtype=np.uint64)
        for bg in graphs_of.values():
            bg.launch()
        for key, g in groups.items():
            if key in graphs_of:
                per, rep = graphs_of[key].result()
                if not rep:
                    raise RuntimeError("captured batch %s/%d exceeded its capacities" % key)
                got[g["idx"]] = per
            else:
                got[g["idx"]] = batch.count_batched(ctx, key[0], g["rel"], g["n"], g["mb"], g["seg"],
                                                    extra_bits=g["extra"], coco=cocos[key], method=g["method"])
        return got

    out = {"captured_groups": ["%s/%d" % k for k in graphs_of], "choice_captured_over_eager_ms": choice}
    for name, fn in (("eager", eager_step), ("captured", graph_step)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            if np.any(fn() != expect):
                raise RuntimeError("resident %s batch: per-query counts differ from the oracle's" % name)
        torch.cuda.synchronize()
        out[name + "_ms_per_step"] = round(1000.0 * (time.perf_counter() - t0) / steps, 3)
        # the small groups alone (what the capture changes)
        keys = list(graphs_of)
        if keys:
            t0 = time.perf_counter()
            for _ in range(steps):
                if name == "eager":
                    for key in keys:
                        g = groups[key]
                        batch.count_batched(ctx, key[0], g["rel"], g["n"], g["mb"], g["seg"], extra_bits=g["extra"],
                                            coco=cocos[key], method=g["method"])
                else:
                    for key in keys:
                        graphs_of[key].launch()
                    for key in keys:
                        graphs_of[key].result()
            torch.cuda.synchronize()
            out[name + "_captured_groups_ms"] = round(1000.0 * (time.perf_counter() - t0) / steps, 3)
    for bg in graphs_of.values():
        bg.free()
    for c in cocos.values():
        c.free()
    return out


def bench_serve(args):
    """Served workload: a Poisson stream of requests (50% triangle, 30% 4-cycle, 20%
    4-clique) over 16 resident R-MAT graphs with 2^16 .. 2^24 undirected edges, each
    request counting one query's tuples whose first variable lies in a block of 1 ..
    16 vertex ids.  Two servers answer it: one query per launch (one slot, one
    hc_join_count per request, one CoCo per graph) and the serving loop (continuous
    batching of all waiting requests of a shape into one pass over a shared
    segmented CoCo of all graphs, concurrent slots on their own streams, admission
    under the HBM budget).  Saturation throughput of each comes from a closed-loop
    run (every request waiting at the start); latency from open-loop replays at
    0.8x and 0.5x of the one-query-per-launch saturation rate.  Every request gets
    the same count from both."""
    import torch
    from paper_2502_06715_amd import inputs, serve

    specs = inputs.serve_graph_specs()
    t0 = time.time()
    graphs = inputs.parallel_graphs(inputs.serve_graph, specs)
    print("# generated %d graphs (%d tuples) in %.1f s" % (len(graphs), sum(g.shape[0] for g in graphs),
                                                        time.time() - t0), file=sys.stderr, flush=True)
    base_eng = serve.GpuEngine(graphs, n_slots=1)
    eng = serve.GpuEngine(graphs, n_slots=args.slots, shared_index=True, grid_share=args.grid_share)
    torch.cuda.synchronize()
    print("# resident CoCos: %.2f GB per graph, %.2f GB shared" % (base_eng.index_bytes / 1e9, eng.index_bytes / 1e9),
          file=sys.stderr, flush=True)
    budget = int(args.budget_gb * 1e9)

    def run(e, slots, fuse, stream, closed):
        reqs = serve.requests_from_stream(stream)
        if closed:
            for r in reqs:
                r.t_arrival = 0.0
        srv = serve.Server(e, budget, n_slots=slots, fuse=fuse,
                           max_weight=(args.max_weight or None) if fuse else None)
        wall = serve.replay(srv, reqs)
        summ = serve.summarize(reqs, wall)
        summ["passes"] = srv.passes
        summ["peak_reserved_gb"] = round(srv.peak_reserved / 1e9, 3)
        return summ, [r.count for r in reqs]

    n_sat = min(args.requests, 4000)
    probe = inputs.serve_stream(specs, n_sat, qps=1.0)
    for _ in range(args.warmup):
        run(eng, args.slots, True, probe[:500], True)
        run(base_eng, 1, False, probe[:200], True)
    sat_base, c_base = run(base_eng, 1, False, probe, True)
    print("# saturation, one query per launch: %s" % json.dumps(sat_base), file=sys.stderr, flush=True)
    sat_srv, c_srv = run(eng, args.slots, True, probe, True)
    print("# saturation, serving loop: %s" % json.dumps(sat_srv), file=sys.stderr, flush=True)
    if c_base != c_srv or any(c is None for c in c_srv):
        bad = [i for i, (a, b) in enumerate(zip(c_base, c_srv)) if a != b]
        print("served counts differ from one-query-per-launch counts at %d requests (first %s); errors: %s"
              % (len(bad), bad[:8], json.dumps(sat_srv["errors"])), file=sys.stderr)
        sys.exit(1)
    if args.saturation_only:
        print(json.dumps({"saturation": {"serving_loop": sat_srv, "one_query_per_launch": sat_base}}), flush=True)
        eng.close()
        base_eng.close()
        return
    qps_sat = sat_base["queries_per_s"]
    open_runs = {}
    for frac in (0.8, 0.5):
        qps = frac * qps_sat
        stream = inputs.serve_stream(specs, args.requests, qps=qps)
        s_srv, cs = run(eng, args.slots, True, stream, False)
        open_runs["serving_loop_at_%.1fx" % frac] = s_srv
        print("# open loop %.0f/s, serving loop: %s" % (qps, json.dumps(s_srv)), file=sys.stderr, flush=True)
        if frac == 0.8:
            s_b, cb = run(base_eng, 1, False, stream, False)
            open_runs["one_query_per_launch_at_%.1fx" % frac] = s_b
            print("# open loop %.0f/s, one query per launch: %s" % (qps, json.dumps(s_b)), file=sys.stderr, flush=True)
            if cb != cs:
                print("served counts differ from one-query-per-launch counts", file=sys.stderr)
                sys.exit(1)
    # full queries: the whole query on a resident graph (triangles on every graph,
    # 4-cycles and 4-cliques on the graphs of at most inputs.FULL_MAX_EDGES edges)
    full = {}
    if args.full_requests > 0:
        fprobe = inputs.serve_full_stream(specs, args.full_requests, qps=1.0)
        fsat_base, fc_base = run(base_eng, 1, False, fprobe, True)
        print("# full queries, saturation, one query per launch: %s" % json.dumps(fsat_base), file=sys.stderr,
              flush=True)
        fsat_srv, fc_srv = run(eng, args.slots, True, fprobe, True)
        print("# full queries, saturation, serving loop: %s" % json.dumps(fsat_srv), file=sys.stderr, flush=True)
        if fc_base != fc_srv or any(c is None for c in fc_srv):
            print("full-query counts differ between the serving loop and one query per launch", file=sys.stderr)
            sys.exit(1)
        fqps = 0.8 * fsat_base["queries_per_s"]
        fstream = inputs.serve_full_stream(specs, args.full_requests, qps=fqps)
        fo_srv, fcs = run(eng, args.slots, True, fstream, False)
        fo_base, fcb = run(base_eng, 1, False, fstream, False)
        print("# full queries, open loop %.1f/s: serving loop %s; one query per launch %s"
              % (fqps, json.dumps(fo_srv), json.dumps(fo_base)), file=sys.stderr, flush=True)
        if fcs != fcb or any(c is None for c in fcs):
            print("full-query counts differ between the serving loop and one query per launch", file=sys.stderr)
            sys.exit(1)
        full = {"requests": args.full_requests, "max_edges_4var": inputs.FULL_MAX_EDGES,
                "saturation": {"serving_loop": fsat_srv, "one_query_per_launch": fsat_base,
                               "speedup": round(fsat_srv["queries_per_s"] / max(fsat_base["queries_per_s"], 1e-9), 3)},
                "open_loop_at_0.8x": {"serving_loop": fo_srv, "one_query_per_launch": fo_base}}
    main_run = open_runs["serving_loop_at_0.8x"]
    out = {
        "metric": "served queries/s (saturation) with p50/p99 latency at 0.8x the one-query-per-launch "
                  "saturation rate (Poisson stream, triangle / 4-cycle / 4-clique mix)",
        "value": sat_srv["queries_per_s"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * sat_srv["wall_s"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "p50_ms": main_run["p50_ms"],
        "p99_ms": main_run["p99_ms"],
        "config": {"workload": "Poisson stream of %d requests, 50%% triangle / 30%% 4-cycle / 20%% 4-clique, over "
                               "16 resident R-MAT graphs with 2^16..2^24 undirected edges (int32), first-variable "
                               "blocks of 1..16 ids, HBM admission budget %.0f GB" % (args.requests, args.budget_gb),
                   "slots": args.slots, "grid_share": args.grid_share,
                   "resident_index_gb": round(eng.index_bytes / 1e9, 3),
                   "max_weight": args.max_weight,
                   "saturation_requests": n_sat},
        "saturation": {"serving_loop": sat_srv, "one_query_per_launch": sat_base,
                       "speedup": round(sat_srv["queries_per_s"] / max(qps_sat, 1e-9), 3)},
        "open_loop": open_runs,
        "full_queries": full,
        "roofline": None,
    }
    eng.close()
    base_eng.close()
    print(json.dumps(out), flush=True)


def bench_tensor(args):
    """Tensor kernels (ternary atoms): the Loomis-Whitney query over R1..R4 and the
    clover-triangle query over R5..R7, on ST-Dense (full cubes [512]^3 and full
    {0,1} x [4096]^2 relations; counts checked against the closed forms 512^4 and
    2 * 4096^3) and on ST-Sparse (random tuples at densities 0.001 and 0.01, domain
    sizes divided by 2^tensor_scale; counts checked for equality with and without
    the rewriting and across two variable orders).  A step is CoCo build of every
    distinct relation + share decision + join count, inputs resident in HBM."""
    import torch
    from paper_2502_06715_amd import hc, inputs

    sc = args.tensor_scale
    t0 = time.time()
    dense = inputs.st_dense()
    n = 5120 >> sc
    m = 40960 >> sc
    sparse = inputs.st_sparse(n=n, rows=(512 >> sc) ** 3, m=m, rows2=(4096 >> sc) ** 2)
    print("# generated tensor relations in %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)
    ctx = hc.Context(0)
    dev = torch.device("cuda:0")
    results = {}
    closed = {("st_dense", "lw"): 512 ** 4, ("st_dense", "ct"): len(inputs.TENSOR_U) * 4096 ** 3}
    for ds_name, ds in [("st_dense", dense), ("st_sparse", sparse)]:
        for qn in ["lw", "ct"]:
            nv, atoms = inputs.QUERIES[qn]
            q = hc.Query(nv, atoms)
            rels = ds[qn]
            uniq = {}
            for r in rels:
                if id(r) not in uniq:
                    uniq[id(r)] = torch.from_numpy(np.ascontiguousarray(r)).to(dev)
            torch.cuda.synchronize()
            order = list(range(nv))

            def step(flags=0, order=order):
                cs = {}
                for key, t in uniq.items():
                    cs[key] = hc.build_coco(ctx, t, [0, 1, 2])
                cocos = [cs[id(r)] for r in rels]
                rule = hc.HC_CACHE_SHARES if args.share_rule == "cache" else 0
                o2, shares = hc.compute_shares(ctx, q, cocos, args.log2_cells, flags=hc.HC_KEEP_ORDER | rule,
                                               order=order)
                cnt = hc.join_count(ctx, q, cocos, order, shares, flags=flags)
                for c in cs.values():
                    c.free()
                return cnt, shares

            for _ in range(args.warmup):
                step()
            torch.cuda.synchronize()
            ts = time.perf_counter()
            outs = [step() for _ in range(args.steps)]
            torch.cuda.synchronize()
            ms = 1000.0 * (time.perf_counter() - ts) / args.steps
            cnt, shares = outs[-1]
            ok = all(o[0] == cnt for o in outs)
            check = "closed form"
            if (ds_name, qn) in closed:
                ok = ok and cnt == closed[(ds_name, qn)]
            else:
                check = "rewrite on/off agree"
                ok = ok and step(flags=hc.HC_NO_REWRITE)[0] == cnt
            if not ok:
                print("tensor count mismatch: %s %s %d" % (ds_name, qn, cnt), file=sys.stderr)
                sys.exit(1)
            results["%s/%s" % (ds_name, qn)] = {"count": cnt, "ms_per_step": round(ms, 3),
                                                "tuples_per_s": cnt / (ms / 1000.0), "log2_shares": shares,
                                                "rows_per_relation": [int(r.shape[0]) for r in rels],
                                                "check": check}
            print("# %s %s: %s" % (ds_name, qn, json.dumps(results["%s/%s" % (ds_name, qn)])), file=sys.stderr,
                  flush=True)
    main = results["st_dense/lw"]
    out = {
        "metric": "output tuples/s on tensor-kernel queries (Loomis-Whitney, clover-triangle)",
        "value": main["tuples_per_s"],
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "LW and CT over ST-Dense ([512]^3 cubes; {0,1} x [4096]^2) and ST-Sparse "
                               "(densities 0.001 / 0.01, domains / 2^%d), int32, count" % sc,
                   "log2_cells": args.log2_cells},
        "results": results,
        "roofline": None,
    }
    print(json.dumps(out), flush=True)


def bench_query_table(args):
    """The query table of Section 7.1 (Q1 triangle, Q2 4-loop, Q4 diamond, Q6
    4-clique, Q8 two triangles sharing a vertex) on the workload-3 recipe scaled
    down (2^16 vertices / 2^20 edges; Q8, whose output grows with the square of the
    triangles per vertex, at 2^14 / 2^18).  A step per query is CoCo build + order
    and share decision (the cost model's joint search, cache rule) + join count,
    the graph resident in HBM; every count is checked against the stored values
    (textbook counters and closed forms, written by tests/golden/make_golden.py)."""
    import torch
    from paper_2502_06715_amd import hc, inputs

    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "workloads.json")))["9"]
    ctx = hc.Context(0)
    dev = torch.device("cuda:0")
    graphs = {}
    results = {}
    tot_cnt, tot_ms = 0, 0.0
    for rec in gold["queries"]:
        qn, sd, want = rec["query"], rec["scale_down"], int(rec["count"])
        print("# query table: %s (scale_down %d)" % (qn, sd), file=sys.stderr, flush=True)
        if sd not in graphs:
            graphs[sd] = torch.from_numpy(inputs.config_graph(3, scale_down=sd)).to(dev)
        E = graphs[sd]
        nv, atoms = inputs.QUERIES[qn]
        q = hc.Query(nv, atoms)
        rule = hc.HC_CACHE_SHARES if args.share_rule == "cache" else 0

        def step():
            c = hc.build_coco(ctx, E, [0, 1], symmetric=True)
            order, shares = hc.compute_shares(ctx, q, [c] * len(atoms), args.log2_cells, flags=rule)
            cnt = hc.join_count(ctx, q, [c] * len(atoms), order, shares)
            c.free()
            return cnt, order, shares

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        outs = [step() for _ in range(args.steps)]
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - ts) / args.steps
        cnt, order, shares = outs[-1]
        if any(o[0] != want for o in outs):
            print("query table: %s count %d differs from the stored %d" % (qn, cnt, want), file=sys.stderr)
            sys.exit(1)
        results[qn] = {"count": cnt, "ms_per_step": round(ms, 3), "tuples_per_s": cnt / (ms / 1000.0),
                       "order": order, "log2_shares": shares, "tuples_in": int(E.shape[0]),
                       "graph": "2^%d vertices, 2^%d edges" % (18 - sd, 22 - sd), "check": rec["count_source"]}
        tot_cnt += cnt
        tot_ms += ms
        print("# %s: %s" % (qn, json.dumps(results[qn])), file=sys.stderr, flush=True)
    out = {
        "metric": "output tuples/s over the query table (Q1, Q2, Q4, Q6, Q8)",
        "value": tot_cnt / (tot_ms / 1000.0),
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(tot_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "query table Q1/Q2/Q4/Q6 on a Chung-Lu graph (beta 2.1, 2^16 vertices, 2^20 "
                               "undirected edges) and Q8 on one of 2^14 / 2^18, int32, count; a step runs every "
                               "query once",
                   "log2_cells": args.log2_cells, "share_rule": args.share_rule},
        "results": results,
        "roofline": None,
    }
    print(json.dumps(out), flush=True)


def _spearman(a, b):
    ra = np.argsort(np.argsort(a)).astype(np.float64)
    rb = np.argsort(np.argsort(b)).astype(np.float64)
    if ra.std() == 0 or rb.std() == 0:
        return None
    return float(np.corrcoef(ra, rb)[0, 1])


def bench_order_sweep(args):
    """Every variable order of the 4-clique query Q6 on a directed graph (the
    workload-3 Chung-Lu graph with every edge oriented from the smaller to the larger
    id), shares from the model for each order (P = 2^log2_cells): measured join
    time against the cost model's Eq. (total cost), with the optimizer's own pick
    (default and joint search) marked."""
    import itertools
    import torch
    from paper_2502_06715_amd import hc, inputs

    E = inputs.config_graph(3)
    E = np.ascontiguousarray(E[E[:, 0] < E[:, 1]])
    n, atoms = inputs.QUERIES["clique4"]
    q = hc.Query(n, atoms)
    ctx = hc.Context(0)
    t = torch.from_numpy(E).to("cuda:0")
    fwd = hc.build_coco(ctx, t, [0, 1])
    bwd = hc.build_coco(ctx, t, [1, 0])
    torch.cuda.synchronize()

    def cocos_for(order):
        pos = {v: i for i, v in enumerate(order)}
        return [fwd if pos[a[0]] < pos[a[1]] else bwd for a in atoms]

    rows = []
    for order in itertools.permutations(range(n)):
        order = list(order)
        cs = cocos_for(order)
        _, shares = hc.compute_shares(ctx, q, cs, args.log2_cells, order=order)
        cost, _ = hc.plan_cost_from_info(q, [c.info for c in cs], order, shares)
        hc.join_count(ctx, q, cs, order, shares)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cnt = hc.join_count(ctx, q, cs, order, shares)
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - t0)
        rows.append({"order": order, "log2_shares": shares, "count": cnt, "join_ms": round(ms, 3),
                     "model_cost": cost})
        print("# order %s shares %s: %.1f ms, model %.3g" % (order, shares, ms, cost), file=sys.stderr, flush=True)
    if len({r["count"] for r in rows}) != 1:
        print("counts differ across orders", file=sys.stderr)
        sys.exit(1)
    picks = {}
    for name, flags in [("default", 0), ("joint_search", hc.HC_JOINT_SEARCH),
                        ("pessimistic", hc.HC_PESSIMISTIC)]:
        o, sh = hc.compute_shares(ctx, q, cocos_for(list(range(n))), args.log2_cells, flags=flags)
        picks[name] = {"order": o, "log2_shares": sh}
    ms = [r["join_ms"] for r in rows]
    best = min(ms)
    for name, pk in picks.items():
        hit = [r for r in rows if r["order"] == pk["order"]]
        pk["order_join_ms"] = hit[0]["join_ms"] if hit else None
        pk["order_rank"] = sorted(ms).index(hit[0]["join_ms"]) + 1 if hit else None
    out = {"metric": "variable-order sweep of the 4-clique query (Q6) on a directed graph",
           "value": best, "unit": "ms (fastest order)", "n_gpus": 1, "higher_is_better": False,
           "data": "synthetic", "dtype": "u32", "vs_baseline": None,
           "config": {"workload": "Q6 over the workload-3 Chung-Lu graph oriented small id -> large id (%d edges)"
                                  % E.shape[0], "log2_cells": args.log2_cells},
           "count": rows[0]["count"], "orders": rows, "optimizer": picks,
           "spearman_model_vs_time": _spearman([r["model_cost"] for r in rows], ms), "roofline": None}
    fwd.free()
    bwd.free()
    print(json.dumps(out), flush=True)


def bench_share_sweep(args):
    """Every power-of-two factorisation P_a x P_b x P_c = 2^K (K = --log2-cells) of the
    triangle query on the R-MAT scale-20 graph (order a,b,c, CoCo built once):
    measured join time against the model, with the optimizer's picks marked."""
    import torch
    from paper_2502_06715_amd import hc, inputs

    E = inputs.config_graph(2)
    n, atoms = inputs.QUERIES["triangle"]
    q = hc.Query(n, atoms)
    ctx = hc.Context(0)
    c = hc.build_coco(ctx, torch.from_numpy(E).to("cuda:0"), [0, 1], key_bits=20)
    torch.cuda.synchronize()
    K = args.log2_cells
    rows = []
    for ka in range(K + 1):
        for kb in range(K + 1 - ka):
            sh = [ka, kb, K - ka - kb]
            cost, _ = hc.plan_cost_from_info(q, [c.info] * 3, [0, 1, 2], sh)
            hc.join_count(ctx, q, [c] * 3, [0, 1, 2], sh)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cnt = hc.join_count(ctx, q, [c] * 3, [0, 1, 2], sh)
            torch.cuda.synchronize()
            ms = 1000.0 * (time.perf_counter() - t0)
            rows.append({"log2_shares": sh, "count": cnt, "join_ms": round(ms, 3), "model_cost": cost})
            print("# shares %s: %.1f ms, model %.3g" % (sh, ms, cost), file=sys.stderr, flush=True)
    if len({r["count"] for r in rows}) != 1:
        print("counts differ across share vectors", file=sys.stderr)
        sys.exit(1)
    ms = [r["join_ms"] for r in rows]
    picks = {}
    for name, flags in [("default", 0), ("joint_search", hc.HC_JOINT_SEARCH), ("pessimistic", hc.HC_PESSIMISTIC),
                        ("cache", hc.HC_CACHE_SHARES)]:
        o, sh = hc.compute_shares(ctx, q, [c] * 3, K, flags=flags | hc.HC_KEEP_ORDER, order=[0, 1, 2])
        hit = [r for r in rows if r["log2_shares"] == sh]
        picks[name] = {"log2_shares": sh, "join_ms": hit[0]["join_ms"],
                       "rank": sorted(ms).index(hit[0]["join_ms"]) + 1}
    best = min(rows, key=lambda r: r["join_ms"])
    out = {"metric": "share sweep (all factorisations of 2^%d) of the triangle query on R-MAT scale 20" % K,
           "value": best["join_ms"], "unit": "ms (fastest share vector)", "n_gpus": 1, "higher_is_better": False,
           "data": "synthetic", "dtype": "u32", "vs_baseline": None,
           "config": {"workload": "triangle, R-MAT scale 20, 2^24 edges, order a,b,c, P = 2^%d" % K},
           "count": rows[0]["count"], "fastest": best, "optimizer": picks, "shares": rows,
           "spearman_model_vs_time": _spearman([r["model_cost"] for r in rows], ms), "roofline": None}
    c.free()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--log2-cells", type=int, default=12)
    ap.add_argument("--share-rule", choices=["cache", "paper"], default="cache",
                    help="share decision: cheapest vector whose cells fit an XCD's L2 (HC_CACHE_SHARES), "
                         "or the paper's evenness rule")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--requests", type=int, default=20000, help="served workload: requests in the stream")
    ap.add_argument("--slots", type=int, default=4, help="served workload: concurrent passes (streams)")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="served workload: HBM admission budget")
    ap.add_argument("--max-weight", type=float, default=2e6,
                    help="served workload: work proxy a fused pass may carry (0: unlimited)")
    ap.add_argument("--grid-share", type=float, default=0.5,
                    help="served workload: share of the default persistent grid each slot may use (0: all)")
    ap.add_argument("--full-requests", type=int, default=400,
                    help="served workload: requests of the full-query stream (0: none)")
    ap.add_argument("--saturation-only", action="store_true",
                    help="served workload: only the closed-loop saturation runs")
    ap.add_argument("--tensor-scale", type=int, default=1,
                    help="tensor workloads: divide ST-Sparse's domain sizes by 2^s (densities kept)")
    ap.add_argument("--cpu-full", action="store_true",
                    help="only time the CPU oracle on the whole workload (sort + Generic Join), no GPU")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = 1 << 28                                    # 2^28 int32 = 1 GiB read + 1 GiB written
        a = torch.ones(n, dtype=torch.int32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}), flush=True)
        return
    if args.cpu_full:
        from paper_2502_06715_amd import inputs
        from oracle import oracle
        desc, _, qname = _workload(args.config)
        n_vars, atoms = inputs.QUERIES[qname]
        E = inputs.config_graph(args.config)
        gold = json.load(open(os.path.join(ROOT, "tests", "golden", "workloads.json")))
        threads = _host_threads()
        t0 = time.perf_counter()
        cnt = oracle.gj(n_vars, atoms, [E] * len(atoms), threads=threads).count
        sec = time.perf_counter() - t0
        if cnt != gold[str(args.config)]["count"]:
            print("oracle count %d differs from the stored count" % cnt, file=sys.stderr)
            sys.exit(1)
        print(json.dumps({"workload": desc, "cpu_full_s": round(sec, 2), "tuples_per_s": cnt / sec,
                          "threads": threads, "cpu_model": _cpu_model(), "count": cnt}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs the join on a single device "
              "(cells would be sharded across GPUs by contiguous cell-id ranges); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    if args.config == 4:
        return bench_batch(args)
    if args.config == 5:
        return bench_serve(args)
    if args.config == 6:
        return bench_tensor(args)
    if args.config == 7:
        return bench_order_sweep(args)
    if args.config == 8:
        return bench_share_sweep(args)
    if args.config == 9:
        return bench_query_table(args)

    import torch
    from paper_2502_06715_amd import hc, inputs

    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "workloads.json")))
    desc, b, qname = _workload(args.config)
    n_vars, atoms = inputs.QUERIES[qname]
    t0 = time.time()
    E = inputs.config_graph(args.config)
    print("# generated workload %d: %d tuples in %.1f s" % (args.config, E.shape[0], time.time() - t0),
          file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    E_dev = torch.from_numpy(E).to(dev)
    ctx = hc.Context(0)
    ctx.set_profiling(True)
    q = hc.Query(n_vars, atoms)
    stream = torch.cuda.current_stream()
    # the small Erdos-Renyi workload is plain Generic Join (one share per variable)
    # with the full output materialised besides the count
    share_flags = hc.HC_CACHE_SHARES if args.share_rule == "cache" else 0
    emit = inputs.CONFIGS[args.config].get("kind") == "er"
    log2_cells = 0 if emit else args.log2_cells
    expect_rows = int(gold[str(args.config)]["count"])
    rows_buf = torch.empty((max(expect_rows, 1), n_vars), dtype=torch.int32, device=dev) if emit else None

    def step():
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        coco = hc.build_coco(ctx, E_dev, [0, 1], key_bits=b)
        ev[1].record(stream)
        order, shares = hc.compute_shares(ctx, q, [coco] * len(atoms), log2_cells, flags=share_flags)
        ev[2].record(stream)
        cnt = hc.join_count(ctx, q, [coco] * len(atoms), order, shares)
        if emit:
            _, n_out = hc.join_emit(ctx, q, [coco] * len(atoms), order, shares, out=rows_buf)
            if n_out != cnt:
                raise RuntimeError("emitted %d rows for a count of %d" % (n_out, cnt))
        ev[3].record(stream)
        ev[3].synchronize()
        t = ctx.timing()
        coco.free()
        return dict(count=cnt, order=order, shares=shares, build_ms=ev[0].elapsed_time(ev[1]),
                    shares_ms=ev[1].elapsed_time(ev[2]), join_ms=ev[2].elapsed_time(ev[3]),
                    leaf_ms=t.leaf_ms, leaf_launches=t.leaf_launches, leaf_items=t.leaf_items)

    for _ in range(args.warmup):
        r = step()
        print("# warmup step: %s" % json.dumps(r), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    res = []
    for _ in range(args.steps):
        res.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    for r in res:
        print("# step: %s" % json.dumps(r), file=sys.stderr, flush=True)
    ms_per_step = 1000.0 * elapsed / args.steps
    count = res[-1]["count"]
    expect = gold[str(args.config)]["count"]
    if any(r["count"] != expect for r in res):
        print("count mismatch: %s vs oracle %d" % ([r["count"] for r in res], expect), file=sys.stderr)
        sys.exit(1)

    # roofline of the dominant kernel: the deepest level of Generic Join
    leaf_ms = sum(r["leaf_ms"] for r in res)
    shares_now = res[-1]["shares"]
    launches = sum(r["leaf_launches"] for r in res)
    wk = gold[str(args.config)].get("work_gallop_per_level")
    roof = None
    if wk and launches:
        alg_bytes_step = 4.0 * wk[-1] + 8.0          # elements touched x 4 B + the count
        per_launch = alg_bytes_step * args.steps / launches
        avg_ms = leaf_ms / launches
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        traffic = None
        issue = None
        hbm_measured = None
        limiter = None
        tf = os.path.join(ROOT, "profiles", "leaf_traffic_config%d.json" % args.config)
        if os.path.exists(tf):
            t = json.load(open(tf))
            # the counters hold for this kernel source, share rule and share vector only
            if t.get("source_hash") == _source_hash() and t.get("log2_shares") == shares_now:
                traffic = t.get("bytes_per_launch")
                sec = avg_ms * 1e-3
                hbm_measured = {"gbs": round(traffic / sec / 1e9, 1),
                                "frac": round(traffic / sec / 1e9 / HBM_PEAK_GBS, 4)}
                # instruction issue: a wave64 vector instruction takes one of a CU's 4 SIMDs
                # for 4 cycles, a scalar one the CU's scalar unit for 1 (256 CUs at 2.4 GHz);
                # counts from the profile, time from this run
                if t.get("valu_insts_per_launch"):
                    issue = {"valu_frac": round(t["valu_insts_per_launch"] * 4 / (1024 * CLOCK_HZ * sec), 3),
                             "salu_frac": round(t["salu_insts_per_launch"] / (256 * CLOCK_HZ * sec), 3),
                             "source": t.get("summary")}
                # what the counters say limits the kernel: the busiest of HBM and the two
                # issue pipes (the rest of its time is spent waiting on L2 and LDS latency)
                fr = {"hbm": hbm_measured["frac"]}
                if issue:
                    fr.update({"vector issue": issue["valu_frac"], "scalar issue": issue["salu_frac"]})
                limiter = max(fr, key=fr.get)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_probe2<M_COUNT, 2> (deepest level)", "avg_launch_ms": round(avg_ms, 3),
                "launches_per_step": launches / args.steps,
                "algorithmic_bytes_per_launch": per_launch,
                "hbm_measured": hbm_measured, "issue": issue, "limiter": limiter}
    out = {
        "metric": "output tuples/s on triangle query" if qname == "triangle" else "output tuples/s",
        "value": count / (ms_per_step / 1000.0),
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": desc, "tuples": int(E.shape[0]), "count": count, "order": res[-1]["order"],
                   "log2_shares": res[-1]["shares"], "log2_cells": log2_cells, "share_rule": args.share_rule,
                   "emit": emit},
        "phases_ms": {k: round(float(np.mean([r[k] for r in res])), 3)
                      for k in ["build_ms", "shares_ms", "join_ms", "leaf_ms"]},
        "roofline": roof,
    }
    if emit:
        out["captured"] = bench_captured_join(ctx, q, E_dev, b, atoms, res[-1]["order"], res[-1]["shares"],
                                              expect, rows_buf)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(E, n_vars, atoms, expect, args.cpu_budget)
    print(json.dumps(out), flush=True)


def bench_captured_join(ctx, q, E_dev, b, atoms, order, shares, expect, rows_buf, reps=50):
    """The join of the step (count and full output) over a resident CoCo: the
    library's count and emit calls (which run a join this small as the device-sized
    sequence, launched directly) against replays of the same sequences captured in
    HIP graphs (hc_join_graph_*); every result checked."""
    import torch
    from paper_2502_06715_amd import hc
    coco = hc.build_coco(ctx, E_dev, [0, 1], key_bits=b)
    cocos = [coco] * len(atoms)
    ctx.set_profiling(False)

    def calls():
        cnt = hc.join_count(ctx, q, cocos, order, shares)
        _, n_out = hc.join_emit(ctx, q, cocos, order, shares, out=rows_buf)
        return cnt, n_out

    gc = hc.JoinGraph(ctx, q, cocos, order, shares)
    ge = hc.JoinGraph(ctx, q, cocos, order, shares, mode="emit", out=rows_buf)

    def graph():
        gc.launch()
        ge.launch()
        c, _, r1 = gc.result()
        n, _, r2 = ge.result()
        if not (r1 and r2):
            raise RuntimeError("a captured join exceeded its capacities")
        return c, n

    out = {}
    for name, fn in (("calls", calls), ("graph", graph)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            c, n = fn()
            if c != expect or n != expect:
                raise RuntimeError("%s join: count %d, rows %d, expected %d" % (name, c, n, expect))
        torch.cuda.synchronize()
        out[name + "_join_ms"] = round(1000.0 * (time.perf_counter() - t0) / reps, 4)
    gc.free()
    ge.free()
    coco.free()
    ctx.set_profiling(True)
    return out


if __name__ == "__main__":
    main()
