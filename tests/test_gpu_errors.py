"""Failure handling on the GPU path, every condition forced from the host: a cancel
request raised before or during a join (the kernels poll it and leave), and an
allocator that refuses requests (HC_ERR_OOM).  After each failure the context and
library keep working and give exact results."""

import threading
import time

import numpy as np
import pytest

from paper_2502_06715_amd import hc, inputs
from tests.gpu_util import config_graph, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return hc.Context(0)


def _coco(ctx, E, b):
    import torch
    return hc.build_coco(ctx, torch.from_numpy(E).to("cuda:0"), [0, 1], key_bits=b, symmetric=True)


def test_cancel_before_the_call(ctx):
    E = config_graph(1)
    c = _coco(ctx, E, 12)
    q = hc.Query(*inputs.QUERIES["triangle"])
    expect = hc.join_count(ctx, q, [c] * 3, [0, 1, 2])
    ctx.cancel(True)
    with pytest.raises(hc.HCError) as ei:
        hc.join_count(ctx, q, [c] * 3, [0, 1, 2])
    assert ei.value.status == hc.HC_ERR_CANCELLED
    ctx.cancel(False)
    assert hc.join_count(ctx, q, [c] * 3, [0, 1, 2]) == expect
    c.free()


def test_cancel_a_running_join():
    """A 4-clique count that takes over a second without the rewriting is cancelled
    from another thread 0.2 s in; it returns HC_ERR_CANCELLED well before it would
    have finished, and the context then counts exactly again."""
    ctx = hc.Context(0)
    E = config_graph(3)
    c = _coco(ctx, E, 18)
    n, atoms = inputs.QUERIES["clique4"]
    q = hc.Query(n, atoms)
    res = {}

    def run():
        t0 = time.perf_counter()
        try:
            res["count"] = hc.join_count(ctx, q, [c] * 6, [0, 1, 2, 3], [1, 1, 1, 1], flags=hc.HC_NO_REWRITE)
        except hc.HCError as e:
            res["status"] = e.status
        res["s"] = time.perf_counter() - t0

    th = threading.Thread(target=run)
    th.start()
    time.sleep(0.2)
    ctx.cancel(True)
    th.join(60)
    assert not th.is_alive()
    log("cancelled join returned after %.3f s: %s" % (res["s"], res))
    assert res.get("status") == hc.HC_ERR_CANCELLED and res["s"] < 1.5
    ctx.cancel(False)
    small = config_graph(1)
    c1 = _coco(ctx, small, 12)
    qt = hc.Query(*inputs.QUERIES["triangle"])
    from tests.test_gpu_join import GOLD
    assert hc.join_count(ctx, qt, [c1] * 3, [0, 1, 2]) == GOLD["1"]["count"]
    c1.free()
    c.free()


def test_allocator_refusal_is_oom(ctx):
    E = config_graph(1)
    c = _coco(ctx, E, 12)
    tight = hc.Context(0, max_bytes=64 << 10)
    q = hc.Query(*inputs.QUERIES["clique4"])
    with pytest.raises(hc.HCError) as ei:
        hc.join_count(tight, q, [c] * 6, [0, 1, 2, 3])
    assert ei.value.status == hc.HC_ERR_OOM
    assert not tight.live          # everything the failed call allocated was given back
    from oracle import oracle
    n, atoms = inputs.QUERIES["clique4"]
    assert hc.join_count(ctx, q, [c] * 6, [0, 1, 2, 3]) == oracle.gj(n, atoms, [E] * 6).count
    c.free()
