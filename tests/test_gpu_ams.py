"""AMS multi-join baseline (Eq. 1) on the GPU against the oracle, through the C ABI:
counters bit-identical, per-repetition numerators S_t = m X_t exact, median equal."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.helpers import keys_u32, to_device_keys

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2402_15953_amd as csk


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _weights(kind, graph, n):
    if kind is None:
        return None
    if kind == "pm1":
        return [W.turnstile_weights(n, 0.1, seed=k).numpy() for k in range(graph.n_rel)]
    return [W.random_weights(n, -2 ** 40, 2 ** 40, seed=30 + k).numpy() for k in range(graph.n_rel)]


CASES = [
    # graph, n, m, d, weights
    (W.chain(3), 3_000, 512, 3, None),
    (W.chain(3), 2_049, 1, 5, "pm1"),
    (W.single_join(), 1, 7, 2, None),
    (W.fig3_query(), 1_500, 300, 3, "big"),
    (W.star(4), 1_000, 1000, 2, None),
    (W.multiway_star(3), 777, 256, 3, "pm1"),
    (W.chain(5), 400, 4096, 1, None),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_ams_sketch_and_estimate_match_oracle(case):
    graph, n, m, d, wk = CASES[case]
    _say("ams", case, graph.name, n, m, d, wk)
    info = oracle.analyze(graph)
    rels = [keys_u32(W.relation_keys(graph, k, n, "zipf", config=300 + case, s=1.1, D=500))
            for k in range(graph.n_rel)]
    weights = _weights(wk, graph, n)
    seed = 70 + case
    coef = oracle.draw_ams_coefficients(seed, d, m, len(info.edges))
    sk = csk.AmsSketch(graph, m, d, seed)
    assert np.array_equal(sk.coefficients(), coef)
    ref = []
    for k in range(graph.n_rel):
        w = None if weights is None else weights[k]
        ref.append(oracle.create_ams_sketch(info, k, rels[k], w, m, coef))
        sk.update(k, to_device_keys(rels[k]), None if w is None else torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    for k in range(graph.n_rel):
        assert np.array_equal(sk.read_sketch(k), ref[k]), k
    nums, med = oracle.estimate_ams(ref)
    est = sk.estimate()
    for t in range(d):
        if abs(nums[t]) < 2 ** 120:
            assert est["rep_numerators"][t] == nums[t], t
    if all(abs(x) < 2 ** 120 for x in nums):
        assert est["exact"] and est["numerator"] == med
        assert est["value"] == pytest.approx(med / m, rel=1e-15, abs=1e-300)
    sk.close()


def test_ams_batches_reset_and_empty():
    graph = W.chain(3)
    info = oracle.analyze(graph)
    m, d, n = 128, 3, 5_000
    rels = [keys_u32(W.relation_keys(graph, k, n, "uniform", config=310, D=100)) for k in range(3)]
    coef = oracle.draw_ams_coefficients(3, d, m, len(info.edges))
    sk = csk.AmsSketch(graph, m, d, 3)
    est0 = sk.estimate()
    assert est0["exact"] and est0["numerator"] == 0 and est0["value"] == 0.0
    for k in range(3):
        kd = to_device_keys(rels[k])
        for a, b in ((0, 1), (1, 1000), (1000, 1000), (1000, 4321), (4321, n)):
            sk.update(k, kd[a:b])
    torch.cuda.synchronize()
    for k in range(3):
        assert np.array_equal(sk.read_sketch(k), oracle.create_ams_sketch(info, k, rels[k], None, m, coef))
    sk.reset()
    torch.cuda.synchronize()
    assert not any(sk.read_sketch(k).any() for k in range(3))
    sk.close()


def test_ams_full_size_sampled_counters():
    """The bench's AMS configuration (chain-3, 10^5 tuples per relation, m = 2^14, d = 5):
    64 sampled counters of every relation computed by the oracle one by one."""
    graph = W.chain(3)
    info = oracle.analyze(graph)
    m, d, n = 1 << 14, 5, 100_000
    rels = [keys_u32(W.relation_keys(graph, k, n, "zipf", config=2, s=1.1, D=10 ** 6)) for k in range(3)]
    sk = csk.AmsSketch(graph, m, d, 11)
    coef = sk.coefficients()
    for k in range(3):
        sk.update(k, to_device_keys(rels[k]))
    torch.cuda.synchronize()
    js = np.random.default_rng(5).choice(m, size=64, replace=False)
    sub = np.ascontiguousarray(coef[:, js])
    for k in range(3):
        got = sk.read_sketch(k)[:, js]
        ref = oracle.create_ams_sketch(info, k, rels[k], None, len(js), sub)
        assert np.array_equal(got, ref), k
    sk.close()


def test_ams_rejects_bad_arguments():
    with pytest.raises(csk.CsError) as e:
        csk.AmsSketch(W.chain(3), 0, 3, 1)
    assert e.value.status == csk.CS_EINVAL
    with pytest.raises(csk.CsError) as e:
        csk.AmsSketch(W.chain(3), 16, 65, 1)
    assert e.value.status == csk.CS_EINVAL
    sk = csk.AmsSketch(W.chain(3), 16, 2, 1)
    with pytest.raises(csk.CsError):
        sk.update(3, torch.zeros(4, 1, dtype=torch.int32, device="cuda"))
    sk.close()
