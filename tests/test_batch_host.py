"""Host logic of the batched path: union relation layout and the autotuner."""

import time

import numpy as np

from paper_2502_06715_amd import batch


def test_union_relation_segments():
    gs = [np.array([[0, 1], [1, 0]], np.int32), np.zeros((0, 2), np.int32), np.array([[2, 3], [3, 2]], np.int32)]
    mb = batch.id_bits(gs)
    rel, seg = batch.union_relation(gs, mb)
    assert mb == 2 and seg == 2
    assert rel.tolist() == [[0, 1], [1, 0], [2 + 8, 3 + 8], [3 + 8, 2 + 8]]


def test_autotune_picks_fastest_and_caches():
    calls = []

    def run(x, m):
        calls.append((x, m))
        time.sleep(0.001 * (abs(x - 2) + (0 if m == "by_size" else 3)))

    t = batch.Autotune(splits=(0, 1, 2, 3), methods=("window", "exponential", "by_size"))
    assert t.pick("cycle4", run) == (2, "by_size")
    n = len(calls)
    assert t.pick("cycle4", run) == (2, "by_size") and len(calls) == n   # cached
    assert n == 4 + 3


def test_size_classes_cover_the_batch():
    from paper_2502_06715_amd import batch, inputs
    specs = inputs.batch_spec(512)
    cls = [batch.size_class(s["m"]) for s in specs]
    assert set(cls) == set(range(len(batch.SIZE_CLASSES) + 1))
    for s, c in zip(specs, cls):
        lo = 0 if c == 0 else 1 << batch.SIZE_CLASSES[c - 1]
        hi = 1 << batch.SIZE_CLASSES[c] if c < len(batch.SIZE_CLASSES) else 1 << 62
        assert lo <= s["m"] < hi
