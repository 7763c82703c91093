"""GPU parity of the CoCo build (Section 4) against the oracle's CoCo by definition:
every level array must be bit-identical, at sizes spanning several 4096-key sort
tiles with a ragged tail, for arities 1-4, both id widths, and the full-size
workload graphs."""

import numpy as np
import pytest

from paper_2502_06715_amd import hc, inputs
from oracle import coco as ococo
from tests.gpu_util import config_graph, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return hc.Context(0)


def _check_coco(ctx, rel, col_order, b, seed, dtype="int32", symmetric=False):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(rel).astype(dtype)).to("cuda:0")
    c = hc.build_coco(ctx, t, col_order, key_bits=b, seed=seed, symmetric=symmetric)
    bb = b if b else ococo.key_bits_for(rel)
    exp = ococo.coco_levels(rel, col_order, bb, seed)
    k = rel.shape[1]
    assert c.info.key_bits == bb
    assert c.info.n_unique == exp["n_unique"]
    for r in range(k):
        v, o = hc.coco_level(ctx, c, r)
        assert np.array_equal(v, exp["V"][r]), "level %d values differ" % r
        if r + 1 < k:
            assert np.array_equal(o.astype(np.int64), exp["O"][r]), "level %d offsets differ" % r
            mc = int(np.diff(exp["O"][r]).max()) if exp["O"][r].size > 1 else 0
            assert c.info.max_children[r] == mc
    uniq = np.unique(rel, axis=0) if rel.shape[0] else rel
    for col in range(k):
        if bb <= 30:
            assert c.info.distinct[col] == np.unique(uniq[:, col]).size
    return c


@pytest.mark.parametrize("arity,n,domain,b,seed,order", [
    (2, 0, 10, 4, 0, [0, 1]),
    (2, 1, 10, 4, 0, [1, 0]),
    (2, 4096 * 3 + 17, 300, 9, 7, [0, 1]),
    (2, 100000, 50000, 16, 123456789, [1, 0]),
    (2, 70000, 1 << 20, 0, 5, [0, 1]),
    (1, 5000, 3000, 12, 1, [0]),
    (3, 20000, 40, 6, 3, [2, 0, 1]),
    (4, 30000, 16, 4, 9, [3, 1, 2, 0]),
    (2, 9000, 1 << 31, 32, 0xFFFF_FFFF_1234, [0, 1]),
])
def test_coco_bit_exact(ctx, arity, n, domain, b, seed, order):
    log("coco arity=%d n=%d domain=%d b=%d" % (arity, n, domain, b))
    rel = inputs.random_relation(n, domain, 1000 + n + arity, arity) if n else np.zeros((0, arity), np.int32)
    if domain == 1 << 31:
        rel = (inputs.splitmix64(5, 0, n * arity) >> np.uint64(33)).astype(np.int64).reshape(n, arity)
    _check_coco(ctx, rel, order, b, seed)


def test_coco_int64_ids(ctx):
    rel = (inputs.splitmix64(77, 0, 20000) >> np.uint64(34)).astype(np.int64).reshape(10000, 2)
    _check_coco(ctx, rel, [1, 0], 0, 42, dtype="int64")


def test_coco_config1_and_symmetric(ctx):
    E = config_graph(1)
    c = _check_coco(ctx, E, [0, 1], 12, 0, symmetric=True)
    assert c.info.symmetric == 1


def test_coco_config2_full_size(ctx):
    E = config_graph(2)
    log("config 2 CoCo: %d rows" % E.shape[0])
    _check_coco(ctx, E, [0, 1], 20, 0, symmetric=True)


def test_symmetric_claim_rejected(ctx):
    import torch
    t = torch.tensor([[0, 1], [1, 0], [2, 3]], dtype=torch.int32, device="cuda:0")
    with pytest.raises(hc.HCError) as ei:
        hc.build_coco(ctx, t, symmetric=True)
    assert ei.value.status == hc.HC_ERR_INVALID


@pytest.mark.parametrize("vals,b,status", [
    ([[0, -1]], 0, hc.HC_ERR_INVALID),
    ([[0, 16]], 4, hc.HC_ERR_INVALID),
])
def test_build_rejects_bad_ids(ctx, vals, b, status):
    import torch
    t = torch.tensor(vals, dtype=torch.int32, device="cuda:0")
    with pytest.raises(hc.HCError) as ei:
        hc.build_coco(ctx, t, key_bits=b)
    assert ei.value.status == status


def test_build_rejects_too_wide_keys(ctx):
    import torch
    t = torch.zeros((4, 3), dtype=torch.int32, device="cuda:0")
    with pytest.raises(hc.HCError) as ei:
        hc.build_coco(ctx, t, key_bits=22)
    assert ei.value.status == hc.HC_ERR_UNSUPPORTED


@pytest.mark.parametrize("shares", [[0, 0], [1, 2], [3, 0], [2, 2, 1]])
def test_partition_sizes_match_oracle(ctx, shares):
    import torch
    arity = len(shares)
    rel = inputs.random_relation(50000, 4000, 99 + arity, arity)
    b, seed = 12, 17
    t = torch.from_numpy(rel).to("cuda:0")
    c = hc.build_coco(ctx, t, list(range(arity))[::-1], key_bits=b, seed=seed)
    B, Bp = hc.partition_sizes(ctx, c, shares)
    uniq = np.unique(rel, axis=0)
    eB, eBp = ococo.partition_sizes(uniq, shares, b, seed)
    assert np.array_equal(B, eB) and np.array_equal(Bp, eBp)
    assert Bp[0] == 0 and Bp[-1] + B[-1] == uniq.shape[0]


@pytest.mark.parametrize("b", [1, 7, 16, 20, 24])
def test_mixer_is_a_bijection_on_the_gpu(ctx, b):
    """The build's key mix over every id of [0, 2^b): the top level of a unary CoCo
    holds 2^b distinct keys, i.e. every b-bit key exactly once (the mapping itself is
    pinned to the oracle's mixer by the bit-exact CoCo tests)."""
    import torch
    ids = np.arange(1 << b, dtype=np.int32).reshape(-1, 1)
    log("mixer bijection b=%d" % b)
    c = hc.build_coco(ctx, torch.from_numpy(ids).to("cuda:0"), [0], key_bits=b, seed=0xC0FFEE)
    v, _ = hc.coco_level(ctx, c, 0)
    assert v.size == 1 << b and np.array_equal(v, np.arange(1 << b, dtype=np.uint32))
    c.free()
