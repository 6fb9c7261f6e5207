"""Filtered ingestion through the C ABI: the sketch of the tuples that pass a query's
filter predicates equals the oracle's sketch of the rows it keeps."""
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


CASES = [
    # graph, n, m, d, weights, predicates (column, lo, hi) over 3 attribute columns
    (W.chain(3), 200_000, 1 << 16, 9, None, [(0, 0, 2 ** 31)]),                   # 16-bit LDS
    (W.chain(3), 150_000, 1 << 12, 5, "pm1", [(1, 3, 6), (2, 0, 2 ** 32 - 1)]),    # 16-bit, +-1
    (W.star(4), 100_001, 1 << 14, 5, "big", [(0, 2 ** 30, 3 * 2 ** 30), (1, 0, 7), (2, 5, 5)]),  # atomics
    (W.single_join(), 5_000, 1024, 3, None, [(1, 9, 8)]),            # keeps nothing
    (W.chain(3), 3_000_000, 1 << 16, 9, None, [(1, 0, 9)]),           # keeps everything
    (W.chain(3), (1 << 23) + 777, 1 << 18, 7, "pm1", [(1, 0, 2)]),   # partition, 30%, two chunks
    (W.chain(3), 300_001, 1 << 20, 3, None, [(2, 1, 1), (1, 0, 8)]), # partition, one column kept in 8
    (W.multiway_star(3), 80_000, 1 << 17, 5, None, [(1, 0, 4)]),     # a column in two joins: atomics
    (W.chain(3), 90_000, 100_003, 5, "pm1", [(0, 0, 2 ** 30)]),      # m not a power of two: atomics
    (W.chain(3), 120_000, 1 << 16, 5, "pm1", [(0, 0, 2 ** 31), (1, 0, 6), (2, 1, 7)]),  # compacted, 3 predicates
    (W.chain(3), 70_000, 1 << 15, 5, None, [(1, 0, 4)]),             # m = 2^15: atomics
]


def _attrs(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.integers(0, 2 ** 32, size=(n, 3), dtype=np.uint64).astype(np.uint32)
    a[:, 1] = rng.integers(0, 10, size=n)
    a[:, 2] = rng.integers(0, 8, size=n)
    return a


@pytest.mark.parametrize("case", range(len(CASES)))
def test_filtered_update_matches_oracle(case):
    graph, n, m, d, wk, preds = CASES[case]
    seed = 500 + case
    _say("filtered", case, graph.name, n, m, d, wk, preds)
    rels = [keys_u32(W.relation_keys(graph, k, n, "zipf", config=600 + case, s=1.1, D=10 ** 5))
            for k in range(graph.n_rel)]
    weights = None
    if wk == "pm1":
        weights = [W.turnstile_weights(n, 0.1, seed=k).numpy() for k in range(graph.n_rel)]
    elif wk == "big":
        weights = [W.random_weights(n, -2 ** 40, 2 ** 40, seed=k).numpy() for k in range(graph.n_rel)]
    attrs = [_attrs(n, 77 + k) for k in range(graph.n_rel)]
    kept = [oracle.filter_rows(rels[k], None if weights is None else weights[k], attrs[k], preds)
            for k in range(graph.n_rel)]
    info, co, ref = oracle_sketches(graph, [kk for kk, _ in kept],
                                    None if weights is None else [ww for _, ww in kept], m, d, seed)
    sk = csk.Sketch(graph, m, d, seed)
    for k in range(graph.n_rel):
        w = None if weights is None else torch.from_numpy(weights[k]).cuda()
        got = sk.update_filtered(k, to_device_keys(rels[k]), torch.from_numpy(attrs[k].view(np.int32)).cuda(),
                                 preds, weights=w, unit_weights=(wk == "pm1"))
        assert got == len(kept[k][0]), (k, got, len(kept[k][0]))
    torch.cuda.synchronize()
    for k in range(graph.n_rel):
        assert np.array_equal(sk.read_sketch(k), ref[k]), k
    sk.close()


def test_filtered_update_rejects_bad_predicates():
    g = W.single_join()
    sk = csk.Sketch(g, 1024, 3, 1)
    keys = torch.zeros(10, 1, dtype=torch.int32, device="cuda")
    attrs = torch.zeros(10, 2, dtype=torch.int32, device="cuda")
    with pytest.raises(csk.CsError):
        sk.update_filtered(0, keys, attrs, [(2, 0, 1)])        # column beyond n_attrs
    with pytest.raises(csk.CsError):
        sk.update_filtered(0, keys, attrs, [(0, 0, 1)] * 9)    # more than 8 predicates
    assert sk.update_filtered(0, keys, attrs, []) == 10        # no predicate: every tuple
    sk.close()


def test_filtered_update_asynchronous_equals_counted():
    """Without a count the call only enqueues; the counters equal the counted call's."""
    g, n, m, d = W.chain(3), 400_000, 1 << 18, 5
    rels = [keys_u32(W.relation_keys(g, k, n, "zipf", config=650, s=1.2, D=10 ** 6)) for k in range(g.n_rel)]
    attrs = [_attrs(n, 90 + k) for k in range(g.n_rel)]
    preds = [(1, 2, 4)]
    a = csk.Sketch(g, m, d, 4)
    b = csk.Sketch(g, m, d, 4)
    for k in range(g.n_rel):
        kd = to_device_keys(rels[k])
        ad = torch.from_numpy(attrs[k].view(np.int32)).cuda()
        assert a.update_filtered(k, kd, ad, preds, count=False) is None
        b.update_filtered(k, kd, ad, preds)
    torch.cuda.synchronize()
    for k in range(g.n_rel):
        assert np.array_equal(a.read_sketch(k), b.read_sketch(k)), k
    a.close()
    b.close()
