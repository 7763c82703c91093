"""GPU parity of the batched path: many small triangle / 4-cycle queries fused into
one Generic Join over a segmented CoCo, per-query counts read from the per-cell
counts (Section 5: the cells partition the output, so a cell range per query
sums to that query's count).  Bit-exact against the oracle's per-query counts,
for every extra split of the first variable the autotuner may pick, and against
one-query-per-launch."""

import json
import os

import numpy as np
import pytest

from paper_2502_06715_amd import batch, hc, inputs
from oracle import coco as ococo
from oracle import oracle
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return hc.Context(0)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _expected(spec, g):
    if spec["query"] == "triangle":
        return 6 * oracle.textbook_triangles(g)
    return oracle.textbook_cycle4(g)


@pytest.fixture(scope="module")
def small_batch():
    specs = inputs.batch_spec(96, seed_base=inputs.SEED_BATCH + (1 << 20), log2_lo=6, log2_hi=12)
    graphs = [inputs.batch_graph(s) for s in specs]
    # an empty graph and a single-edge graph inside the batch
    graphs[5] = np.zeros((0, 2), np.int32)
    graphs[7] = np.array([[0, 1], [1, 0]], np.int32)
    return specs, graphs


def test_segmented_coco_bit_exact(ctx, small_batch):
    specs, graphs = small_batch
    gs = graphs[:20]
    mb = batch.id_bits(gs)
    rel, seg = batch.union_relation(gs, mb)
    log("segmented coco rows=%d mix_bits=%d seg_bits=%d" % (rel.shape[0], mb, seg))
    c = hc.build_coco(ctx, _dev(rel), [0, 1], key_bits=mb, seed=0x1234, segment_bits=seg, symmetric=True)
    exp = ococo.coco_levels(rel, [0, 1], mb, 0x1234, segmented=True)
    assert c.info.mix_bits == mb and c.info.key_bits == mb + seg
    assert c.info.n_unique == exp["n_unique"]
    for r in range(2):
        v, o = hc.coco_level(ctx, c, r)
        assert np.array_equal(v, exp["V"][r])
        if r == 0:
            assert np.array_equal(o.astype(np.int64), exp["O"][0])
    c.free()


@pytest.mark.parametrize("shape", ["triangle", "cycle4"])
@pytest.mark.parametrize("extra", [0, 1, 3])
def test_batched_counts_match_oracle(ctx, small_batch, shape, extra):
    specs, graphs = small_batch
    # every graph of the batch under this shape (the shapes of the specs are ignored here)
    mb = batch.id_bits(graphs)
    rel, seg = batch.union_relation(graphs, mb)
    log("batched %s extra=%d queries=%d rows=%d" % (shape, extra, len(graphs), rel.shape[0]))
    got = batch.count_batched(ctx, shape, _dev(rel), len(graphs), mb, seg, extra_bits=extra)
    exp = [_expected({"query": shape}, g) for g in graphs]
    assert [int(x) for x in got] == exp


def test_batched_ragged_segment_count(ctx, small_batch):
    """A batch whose size is not a power of two: the unused segments count zero."""
    specs, graphs = small_batch
    gs = graphs[:37]
    mb = batch.id_bits(gs)
    rel, seg = batch.union_relation(gs, mb)
    assert seg == 6
    got = batch.count_batched(ctx, "triangle", _dev(rel), len(gs), mb, seg)
    assert [int(x) for x in got] == [_expected({"query": "triangle"}, g) for g in gs]


def test_sequential_equals_batched(ctx, small_batch):
    specs, graphs = small_batch
    gs = [g for g in graphs[:24] if g.shape[0]]
    got = batch.count_sequential(ctx, "cycle4", [_dev(g) for g in gs])
    assert [int(x) for x in got] == [_expected({"query": "cycle4"}, g) for g in gs]


def test_segmented_share_rules_rejected(ctx, small_batch):
    """A share on a variable other than the first, or a first-variable share below
    the segment bits, would mix queries: the library refuses both."""
    specs, graphs = small_batch
    gs = graphs[:8]
    mb = batch.id_bits(gs)
    rel, seg = batch.union_relation(gs, mb)
    c = hc.build_coco(ctx, _dev(rel), [0, 1], key_bits=mb, segment_bits=seg, symmetric=True)
    n, atoms = inputs.QUERIES["triangle"]
    q = hc.Query(n, atoms)
    with pytest.raises(hc.HCError):
        hc.join_count_cells(ctx, q, [c] * 3, [0, 1, 2], [seg - 1, 0, 0])
    with pytest.raises(hc.HCError):
        hc.join_count_cells(ctx, q, [c] * 3, [0, 1, 2], [seg, 1, 0])
    c.free()


def test_full_batch_per_query_counts(ctx):
    """The full 4096-query workload (log-uniform 2^10..2^18 edges), both shapes, per
    query bit-exact against the stored oracle counts."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batch_config4.json")))
    specs = inputs.batch_spec(gold["n_queries"])
    log("generating %d graphs" % len(specs))
    graphs = inputs.batch_graphs(specs)
    exp = np.array([int(c) for c in gold["counts"]], dtype=np.uint64)
    for shape in ["triangle", "cycle4"]:
        idx = [i for i, s in enumerate(specs) if s["query"] == shape]
        gs = [graphs[i] for i in idx]
        mb = batch.id_bits(gs)
        rel, seg = batch.union_relation(gs, mb)
        log("full batch %s queries=%d rows=%d mix_bits=%d seg_bits=%d" % (shape, len(gs), rel.shape[0], mb, seg))
        got = batch.count_batched(ctx, shape, _dev(rel), len(gs), mb, seg, extra_bits=1)
        bad = np.flatnonzero(got != exp[idx])
        assert bad.size == 0, [(idx[i], int(got[i]), int(exp[idx[i]])) for i in bad[:5]]
