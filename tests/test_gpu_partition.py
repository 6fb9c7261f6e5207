"""The partition strategy (records sorted by bucket range, one workgroup per range) against
the oracle, bit for bit, in the cases its structure singles out: heavy Zipf skew (hot
tuples taken out of the record stream and summed), hot tuples whose Deltas cancel or
mix signs, a stream of one repeated tuple, segments cut short (n not a multiple of the
1024-tuple segment), several chunks, keys not 16-byte aligned, m not a power of two and
columns in several joins (the general hash), repetition groups of several shapes, the
counters after many calls, and hot-key hints carried across calls whose heavy keys
change."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.helpers import keys_u32, oracle_sketches, to_device_keys

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2402_15953_amd as csk


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check(graph, rels, weights, m, d, seed, unit, offset=0):
    info, co, ref = oracle_sketches(graph, rels, weights, m, d, seed)
    sk = csk.Sketch(graph, m, d, seed)
    for k, keys in enumerate(rels):
        kd = to_device_keys(keys)
        if offset:  # the same keys starting `offset` tuples into a larger buffer
            big = torch.zeros((keys.shape[0] + offset, keys.shape[1]), dtype=torch.int32, device="cuda")
            big[offset:] = kd
            kd = big[offset:]
        wd = None if weights is None else torch.from_numpy(weights[k]).cuda()
        sk.update(k, kd, wd, strategy=csk.UPDATE_PARTITION, unit_weights=unit)
    torch.cuda.synchronize()
    for k in range(graph.n_rel):
        got = sk.read_sketch(k)
        assert np.array_equal(got, ref[k]), (k, int(np.count_nonzero(got != ref[k])))
    sk.close()


CASES = [
    # graph, n, m, d, Zipf s, domain, weights (None / pm1 / pm50), key offset
    (W.chain(3), 300_000, 1 << 18, 15, 1.5, 10 ** 7, None, 0),
    (W.chain(3), 300_000, 1 << 18, 15, 1.5, 10 ** 7, "pm50", 0),
    (W.chain(5), 200_003, 1 << 18, 5, 1.0, 10 ** 7, "pm1", 1),
    (W.chain(3), 1, 1 << 17, 3, 1.1, 10 ** 6, None, 0),
    (W.chain(3), 1023, 1 << 20, 3, 1.1, 10 ** 6, None, 0),
    (W.chain(3), 1025, 1 << 19, 3, 1.1, 10 ** 6, "pm1", 3),
    (W.chain(3), (1 << 23) + 4097, 1 << 18, 3, 1.2, 10 ** 6, None, 0),
    (W.chain(3), (1 << 23) + 4097, 1 << 18, 3, 1.2, 10 ** 6, None, 1),
    (W.chain(3), 150_000, 300_007, 5, 1.1, 10 ** 6, "pm1", 0),
    (W.multiway_star(3), 100_000, 1 << 18, 3, 1.3, 1000, None, 0),
    (W.star(3), 100_000, 1 << 16, 5, 1.1, 10 ** 5, None, 0),
    (W.single_join(), 100_000, 1000, 5, 1.1, 10 ** 5, "pm1", 0),
    # repetition groups of other shapes: 129 blocks at d = 20, 300 blocks at d = 7
    (W.chain(3), 128 * 4096 + 5, 1 << 18, 20, 1.3, 10 ** 6, None, 0),
    (W.chain(3), 300 * 4096, 1 << 17, 7, 1.1, 10 ** 6, None, 0),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_partition_bit_exact(case):
    graph, n, m, d, s, D, wk, off = CASES[case]
    if max(len(graph.columns(k)) for k in range(graph.n_rel)) > 2:
        pytest.skip("partition strategy: at most two key columns")
    _say("partition", case, graph.name, n, m, d, s, wk, off)
    rels = [keys_u32(W.relation_keys(graph, k, n, "zipf", config=2100 + case, s=s, D=D)) for k in range(graph.n_rel)]
    weights = None
    if wk == "pm1":
        weights = [W.turnstile_weights(n, 0.3, seed=2100 + k).numpy() for k in range(graph.n_rel)]
    elif wk == "pm50":  # half the tuples deleted: hot tuples' Delta sums near zero
        weights = [W.turnstile_weights(n, 0.5, seed=2200 + k).numpy() for k in range(graph.n_rel)]
    _check(graph, rels, weights, m, d, 50 + case, wk is not None, off)


def test_partition_one_repeated_tuple():
    """Every tuple the same: all of them hot, no record emitted; then two alternating
    tuples, and a stream where the hot tuple's Deltas cancel exactly."""
    g, m, d = W.chain(3), 1 << 18, 7
    n = 50_000
    one = [np.full((n, len(g.columns(k))), 123457, dtype=np.uint32) for k in range(g.n_rel)]
    _check(g, one, None, m, d, 5, False)
    two = [np.where((np.arange(n) % 2)[:, None] == 0, 17, 99991).astype(np.uint32).repeat(len(g.columns(k)), axis=1)
           for k in range(g.n_rel)]
    _check(g, two, None, m, d, 6, False)
    w = [np.where(np.arange(n) % 2 == 0, 1, -1).astype(np.int64) for _ in range(g.n_rel)]
    _check(g, one, w, m, d, 7, True)


def test_partition_many_calls_equal_one():
    """96 calls of 2^14 tuples on one stream equal the oracle on the whole stream (the
    scratch buffer is reused call after call)."""
    g, m, d, seed = W.chain(5), 1 << 18, 15, 9
    n_call, calls = 1 << 14, 96
    rels = [keys_u32(W.relation_keys(g, k, n_call * calls, "zipf", config=2300, s=1.0, D=10 ** 7))
            for k in range(g.n_rel)]
    info, co, ref = oracle_sketches(g, rels, None, m, d, seed)
    sk = csk.Sketch(g, m, d, seed)
    dev = [to_device_keys(r) for r in rels]
    for c in range(calls):
        for k in range(g.n_rel):
            sk.update(k, dev[k][c * n_call:(c + 1) * n_call], strategy=csk.UPDATE_PARTITION)
    torch.cuda.synchronize()
    for k in range(g.n_rel):
        assert np.array_equal(sk.read_sketch(k), ref[k]), k
    sk.close()


def test_partition_hints_follow_the_stream():
    """Hot-key hints carried from call to call: a skewed stream, then one whose heavy
    keys are different tuples (stale hints), then spread keys (no hot tuple), then the
    first again; every relation's counters equal the oracle's on the whole stream."""
    g, m, d, seed = W.chain(3), 1 << 18, 7, 21
    n_call = 1 << 16
    parts = []
    for i, (s, shift) in enumerate(((1.5, 0), (1.5, 1000003), (0.5, 0), (1.5, 0))):
        keys = []
        for k in range(g.n_rel):
            x = keys_u32(W.relation_keys(g, k, 3 * n_call, "zipf", config=2400 + i, s=s, D=10 ** 6))
            keys.append((x.astype(np.uint64) + shift).astype(np.uint32))
        parts.append(keys)
    rels = [np.concatenate([p[k] for p in parts]) for k in range(g.n_rel)]
    info, co, ref = oracle_sketches(g, rels, None, m, d, seed)
    sk = csk.Sketch(g, m, d, seed)
    for p in parts:
        dev = [to_device_keys(x) for x in p]
        for c in range(3):
            for k in range(g.n_rel):
                sk.update(k, dev[k][c * n_call:(c + 1) * n_call], strategy=csk.UPDATE_PARTITION)
    torch.cuda.synchronize()
    for k in range(g.n_rel):
        assert np.array_equal(sk.read_sketch(k), ref[k]), k
    sk.close()
