"""Autotuner through the C ABI: every candidate it runs must give the reference counters,
the chosen variant then serves cs_update's automatic strategy, and the counters still
equal the oracle's."""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from tests.helpers import keys_u32, oracle_sketches, to_device_keys

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2402_15953_amd as csk


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    # graph, n, m, d, weights
    (W.chain(3), 400_000, 1 << 16, 9, None),
    (W.chain(3), 300_000, 1 << 12, 5, "pm1"),
    (W.star(4), 200_000, 1 << 18, 3, None),
    (W.chain(3), 100_000, 1 << 10, 5, "big"),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_tuned_update_matches_oracle(case):
    graph, n, m, d, wk = CASES[case]
    seed = 300 + case
    rels = [keys_u32(W.relation_keys(graph, k, n, "zipf", config=880 + case, s=1.1, D=10 ** 6))
            for k in range(graph.n_rel)]
    weights = None
    if wk == "pm1":
        weights = [W.turnstile_weights(n, 0.1, seed=k).numpy() for k in range(graph.n_rel)]
    elif wk == "big":
        weights = [W.random_weights(n, -2 ** 40, 2 ** 40, seed=k).numpy() for k in range(graph.n_rel)]
    info, co, ref = oracle_sketches(graph, rels, weights, m, d, seed)
    csk.tune_clear()
    sk = csk.Sketch(graph, m, d, seed)
    try:
        dev_keys = [to_device_keys(r) for r in rels]
        dev_w = None if weights is None else [torch.from_numpy(w).cuda() for w in weights]
        for k in range(graph.n_rel):
            rep = csk.tune_update(sk, k, dev_keys[k], None if dev_w is None else dev_w[k],
                                  unit_weights=(wk == "pm1"))
            ran = [c for c in rep["candidates"] if c["valid"] != 0]
            _say("case", case, "rel", k, "best", rep["best"], "ran", len(ran))
            assert rep["best"]["valid"] == 1
            assert all(c["valid"] == 1 for c in ran), rep["candidates"]   # every variant agrees
            assert len(ran) >= 3
        assert csk.tune_count() >= 1
        # tuning left the handle's counters untouched
        for k in range(graph.n_rel):
            assert not np.any(sk.read_sketch(k))
        for k in range(graph.n_rel):
            sk.update(k, dev_keys[k], None if dev_w is None else dev_w[k], unit_weights=(wk == "pm1"))
        torch.cuda.synchronize()
        for k in range(graph.n_rel):
            assert np.array_equal(sk.read_sketch(k), ref[k]), k
    finally:
        sk.close()
        csk.tune_clear()
