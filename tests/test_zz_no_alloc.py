"""The entry point that allocates nothing (hc_join_count_noalloc) against
hc_join_count on the same inputs: counts and digests equal, two calls in a row
with the second on a smaller input, no request through the context's allocator,
and a call too large for the fixed scratch array rejected with a clear error."""

import numpy as np
import pytest

from paper_2502_06715_amd import hc, inputs
from tests.gpu_util import config_graph, log

pytestmark = pytest.mark.gpu
SCRATCH = 256 << 20   # bytes of the library's per-GPU scratch array


def _coco(ctx, E, b):
    import torch
    return hc.build_coco(ctx, torch.from_numpy(np.ascontiguousarray(E)).to("cuda:0"), [0, 1], key_bits=b,
                         symmetric=True)


def test_noalloc_equals_join_count_two_calls():
    ctx = hc.Context(0)
    cases = [
        ("triangle", config_graph(1), 12, [0, 1, 2], [1, 2, 1]),
        ("triangle", inputs.erdos_renyi(1 << 9, 1 << 11, 0x4E41), 9, [2, 0, 1], [0, 0, 0]),
    ]
    for name, E, b, order, shares in cases:
        n, atoms = inputs.QUERIES[name]
        q = hc.Query(n, atoms)
        c = _coco(ctx, E, b)
        exp = hc.join_count(ctx, q, [c] * len(atoms), order, shares, digest=True)
        before = ctx.n_allocs
        cnt, dg, used = hc.join_count_noalloc(ctx, q, [c] * len(atoms), order, shares, digest=True)
        log("noalloc %s rows=%d shares=%s: count %d, scratch used %d" % (name, E.shape[0], shares, cnt, used))
        assert ctx.n_allocs == before, "the call allocated through the context"
        assert (cnt, dg) == exp
        assert 0 < used <= SCRATCH


def test_noalloc_lifted_pools_and_repeat():
    """The 4-clique query with the rewriting (lifted pools in the scratch array), twice
    in a row, then a smaller graph: every call equals hc_join_count."""
    ctx = hc.Context(0)
    n, atoms = inputs.QUERIES["clique4"]
    q = hc.Query(n, atoms)
    for E, b in [(inputs.chung_lu(2048, 12000, 77), 11), (inputs.chung_lu(2048, 12000, 77), 11),
                 (inputs.chung_lu(512, 2000, 78), 9)]:
        c = _coco(ctx, E, b)
        for flags in [0, hc.HC_NO_REWRITE]:
            exp = hc.join_count(ctx, q, [c] * 6, [0, 1, 2, 3], [1, 1, 0, 1], flags=flags, digest=True)
            before = ctx.n_allocs
            cnt, dg, used = hc.join_count_noalloc(ctx, q, [c] * 6, [0, 1, 2, 3], [1, 1, 0, 1], flags=flags,
                                                  digest=True)
            log("noalloc clique4 rows=%d flags=%d: count %d, scratch used %d" % (E.shape[0], flags, cnt, used))
            assert ctx.n_allocs == before
            assert (cnt, dg) == exp and 0 < used <= SCRATCH


def test_noalloc_rejects_calls_beyond_the_array():
    """2^24 HyperCube cells: the first frontier alone (one entry per cell, never
    split) exceeds the array, so the call is refused before anything runs, and a
    normal call afterwards still works."""
    ctx = hc.Context(0)
    E = inputs.rmat(16, 1 << 18, 0x4E42)
    n, atoms = inputs.QUERIES["triangle"]
    q = hc.Query(n, atoms)
    c = _coco(ctx, E, 16)
    with pytest.raises(hc.HCError) as ei:
        hc.join_count_noalloc(ctx, q, [c] * 3, [0, 1, 2], [8, 8, 8])
    assert ei.value.status == hc.HC_ERR_UNSUPPORTED
    assert "scratch" in str(ei.value)
    exp = hc.join_count(ctx, q, [c] * 3, [0, 1, 2], [2, 2, 0])
    assert hc.join_count_noalloc(ctx, q, [c] * 3, [0, 1, 2], [2, 2, 0])[0] == exp
