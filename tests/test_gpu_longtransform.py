"""Estimates whose transforms are 2^19 points or longer, against the oracle's exact
integers (Eq. 5 evaluated as Alg. 3 over the sketches' nonzero counters).

* spectral plan at m = 2^19 and 2^20: the two-pass FFT with 2048- and 4096-element
  tiles, and (large weights) its modular residue pass at those lengths;
* general plan at m = 10^6 (the paper's sketch size) and m = 999,983: Alg. 3's
  correlations as zero-padded number-theoretic transforms of length 2^21, then folded;
* general plan at m = 2^19 (a component of three attributes).

Sketches are bit-identical to the oracle's; every repetition and the median equal the
oracle's exact integers.  Inputs have few tuples so the oracle stays fast."""
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

INT128_EXACT = 2 ** 125


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    # graph, n per relation, m, d, Zipf s, domain, weights, plan
    (W.chain(3), 800, 1 << 19, 5, 1.1, 10 ** 6, None, "spectral"),
    (W.chain(3), 800, 1 << 20, 5, 1.1, 10 ** 6, None, "spectral"),
    (W.chain(5), 40, 1 << 20, 3, 1.0, 50, None, "spectral"),
    (W.star(4), 300, 1 << 19, 3, 1.2, 10 ** 6, None, "spectral"),
    (W.chain(3), 400, 1 << 20, 5, 1.1, 10 ** 6, "huge", "spectral"),
    (W.chain(3), 600, 10 ** 6, 5, 1.1, 10 ** 6, None, "general"),
    (W.chain(5), 40, 10 ** 6, 3, 1.0, 50, None, "general"),
    (W.chain(3), 500, 999_983, 3, 1.1, 10 ** 6, "pm1", "general"),
    (W.fig3_query(), 300, 1 << 19, 3, 1.1, 10 ** 5, None, "general"),
]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("case", range(len(CASES)))
def test_long_transform_estimate_exact(case):
    graph, n, m, d, s, D, wk, plan = CASES[case]
    _say("long transform", case, graph.name, n, m, d, s, wk, plan)
    rels = [keys_u32(W.relation_keys(graph, k, n, "zipf", config=1900 + case, s=s, D=D))
            for k in range(graph.n_rel)]
    weights = None
    if wk == "huge":
        weights = [W.random_weights(n, -2 ** 40, 2 ** 40, seed=1900 + k).numpy() for k in range(graph.n_rel)]
    elif wk == "pm1":
        weights = [W.turnstile_weights(n, 0.1, seed=1900 + k).numpy() for k in range(graph.n_rel)]
    seed = 70 + case
    info, co, ref = oracle_sketches(graph, rels, weights, m, d, seed)
    sk = csk.Sketch(graph, m, d, seed)
    assert sk.info()["plan"] == {"spectral": csk.PLAN_SPECTRAL, "general": csk.PLAN_GENERAL}[plan]
    for k in range(graph.n_rel):
        wd = None if weights is None else torch.from_numpy(weights[k]).cuda()
        sk.update(k, to_device_keys(rels[k]), wd, unit_weights=wk == "pm1")
    torch.cuda.synchronize()
    for k in range(graph.n_rel):
        assert np.array_equal(sk.read_sketch(k), ref[k]), k
    est = sk.estimate(reps=True)
    reps = []
    for t in range(d):
        exact = oracle.estimate_sparse(info, [ref[k][t] for k in range(graph.n_rel)], m)
        reps.append(exact)
        if abs(exact) < INT128_EXACT:
            assert est["rep_ints"][t] == exact, (t, est["rep_ints"][t], exact, est["rep_bounds"][t])
            assert est["rep_values"][t] == float(exact)
        else:
            assert abs(est["rep_values"][t] - exact) <= 1e-12 * abs(exact), (t, est["rep_values"][t], exact)
    med = oracle.median_lower(reps)
    assert est["exact"] and est["value"] == float(med)
    if -2 ** 63 <= med < 2 ** 63:
        assert est["value_i64"] == med
    _say("  median", med, "modular repetitions", est["n_modular"])
    sk.close()
