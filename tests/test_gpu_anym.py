"""Bucket counts m that are not powers of two, through the C ABI.

Sketches are reduced modulo m (Alg. 2's bin hash h(x) mod m) in every update kernel;
estimates go through Alg. 3's register program with zero-padded transforms (or the
exact inner product for two relations).  Sketches must equal the oracle's bit for bit
and estimates its exact integers."""
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


def _rels(graph, n, dist, D, config, s=1.1):
    return [keys_u32(W.relation_keys(graph, k, n, dist, config=config, s=s, D=D)) for k in range(graph.n_rel)]


def _weights(kind, graph, n):
    if kind is None:
        return None
    if kind == "pm1":
        return [W.turnstile_weights(n, 0.1, seed=k).numpy() for k in range(graph.n_rel)]
    return [W.random_weights(n, -2 ** 40, 2 ** 40, seed=70 + k).numpy() for k in range(graph.n_rel)]


def _run(graph, rels, weights, m, d, seed, strategy=0, unit=False, counters16=True):
    sk = csk.Sketch(graph, m, d, seed)
    for k, keys in enumerate(rels):
        wd = None if weights is None else torch.from_numpy(weights[k]).cuda()
        sk.update(k, to_device_keys(keys), wd, strategy=strategy, unit_weights=unit, counters16=counters16)
    torch.cuda.synchronize()
    return sk


SKETCH_CASES = [
    # graph, n, m, d, dist, D, weights
    (W.chain(3), 20_011, 1000, 5, "zipf", 10 ** 5, None),
    (W.chain(3), 70_000, 65_534, 9, "zipf", 10 ** 6, "pm1"),     # 16-bit counters, even m
    (W.chain(3), 70_000, 40_000, 3, "zipf", 10 ** 6, None),      # 16-bit counters, even m
    (W.chain(3), 30_000, 65_535, 3, "uniform", 10 ** 6, None),   # odd m: 32-bit counters
    (W.star(4), 50_000, 999_983, 2, "uniform", 10 ** 9, None),   # bucket-range segments
    (W.fig3_query(), 7_777, 300, 7, "uniform", 200, "big"),
    (W.multiway_star(4), 5_000, 3, 4, "zipf", 100, None),
    (W.chain(5), 30_000, 5_000, 15, "zipf", 10 ** 7, "pm1"),
    (W.single_join(), (1 << 21) + 77, 49_999, 2, "zipf", 10 ** 6, "pm1"),
    (W.chain(3), 300_000, 1_000_000, 5, "zipf", 10 ** 6, "pm1"),  # partition: partial last range
    (W.chain(3), 100_000, 99_991, 3, "uniform", 10 ** 6, None),
]


@pytest.mark.parametrize("case", range(len(SKETCH_CASES)))
@pytest.mark.parametrize("strategy", [0, 1, 2, 3, 4])
def test_sketch_bit_exact_any_m(case, strategy):
    graph, n, m, d, dist, D, wk = SKETCH_CASES[case]
    if strategy == 4 and (wk == "big" or max(len(graph.columns(k)) for k in range(graph.n_rel)) > 2):
        pytest.skip("partition strategy: +-1 weights and at most two key columns")
    _say("any-m sketch", case, graph.name, n, m, d, "strategy", strategy)
    rels = _rels(graph, n, dist, D, config=500 + case)
    weights = _weights(wk, graph, n)
    seed = 2000 + case
    info, co, ref = oracle_sketches(graph, rels, weights, m, d, seed)
    for c16 in ((True, False) if strategy == 2 else (True,)):
        sk = _run(graph, rels, weights, m, d, seed, strategy=strategy, unit=(wk == "pm1"), counters16=c16)
        for k in range(graph.n_rel):
            assert np.array_equal(sk.read_sketch(k), ref[k]), (k, c16)
        sk.close()


def test_invalid_m_rejected():
    for m in (0, 1, (1 << 20) + 1):
        with pytest.raises(csk.CsError) as e:
            csk.Sketch(W.chain(3), m, 3, 1)
        assert e.value.status == csk.CS_EINVAL


def _check_estimate(graph, sk, ref, m, d, info):
    est = sk.estimate(reps=True)
    reps = []
    for t in range(d):
        exact = oracle.estimate_alg3(info, [ref[k][t] for k in range(graph.n_rel)], m, method="ntt")
        reps.append(exact)
        if abs(exact) < INT128_EXACT:
            assert est["rep_ints"][t] == exact, (t, est["rep_ints"][t], exact)
        else:
            assert abs(est["rep_values"][t] - exact) <= 1e-12 * abs(exact)
    med = oracle.median_lower(reps)
    if abs(med) < INT128_EXACT:
        assert est["exact"] and est["value"] == float(med)
    return est


EST_CASES = [
    # graph, n, m, d, dist, D, s, weights
    (W.chain(3), 20_000, 1000, 5, "zipf", 10 ** 4, 1.1, None),
    (W.chain(3), 20_000, 2_500, 3, "zipf", 10 ** 5, 1.1, "pm1"),
    (W.chain(4), 5_000, 300, 5, "zipf", 10 ** 4, 1.2, "pm1"),
    (W.star(4), 8_000, 777, 3, "zipf", 1000, 1.2, None),
    (W.fig3_query(), 3_000, 300, 5, "zipf", 500, 1.1, "big"),
    (W.multiway_star(3), 2_000, 100, 3, "uniform", 50, 1.0, None),
    (W.chain(6), 3_000, 3, 4, "uniform", 30, 1.0, None),
    (W.single_join(), 100_000, 999_983, 5, "uniform", 10 ** 4, 1.0, None),
    (W.chain(3), 5_000, 1537, 5, "zipf", 10 ** 4, 1.1, "big"),
]


@pytest.mark.parametrize("case", range(len(EST_CASES)))
def test_estimate_exact_any_m(case):
    graph, n, m, d, dist, D, s, wk = EST_CASES[case]
    _say("any-m estimate", case, graph.name, n, m, d, wk)
    rels = _rels(graph, n, dist, D, config=600 + case, s=s)
    weights = _weights(wk, graph, n)
    seed = 40 + case
    info, co, ref = oracle_sketches(graph, rels, weights, m, d, seed)
    sk = _run(graph, rels, weights, m, d, seed)
    for k in range(graph.n_rel):
        assert np.array_equal(sk.read_sketch(k), ref[k])
    if graph.n_rel > 2:
        assert sk.info()["plan"] == csk.PLAN_GENERAL
    est = _check_estimate(graph, sk, ref, m, d, info)
    _say("  value", est["value"])
    sk.close()


def _chain3_eq5(info, c, m):
    """Eq. 5 for the 3-relation chain, summed over the nonzero counters of the two end
    relations only (every other term is zero): X = sum c_0[j0] c_1[(j0 + j1) mod m]
    c_2[j1], with the relations' bucket maps read from the join graph."""
    comps = [sorted(info.psi[u] for u in info.omega[k]) for k in range(3)]
    assert comps[0] == [0] and comps[2] == [1] and comps[1] == [0, 1], comps
    nz0 = np.nonzero(c[0])[0]
    nz2 = np.nonzero(c[2])[0]
    total = 0
    for a in range(0, len(nz0), 512):
        j0 = nz0[a:a + 512]
        idx = (j0[:, None] + nz2[None, :]) % m
        terms = c[0][j0][:, None] * c[1][idx] * c[2][nz2][None, :]
        total += int(terms.sum(dtype=np.int64))
    return total


@pytest.mark.parametrize("m", [65_534, 40_000, 65_535, 99_991])
def test_estimate_large_m_chain3(m):
    """Large m that are not powers of two (transforms of length 2^17 and 2^18): the
    exact per-repetition estimates against Eq. 5.  Unit weights on 3000 tuples keep
    every product of three counters and the sum exact in int64."""
    graph, n, d = W.chain(3), 3_000, 3
    _say("any-m large estimate", m)
    rels = _rels(graph, n, "zipf", 10 ** 5, config=700 + m % 97)
    weights = [W.turnstile_weights(n, 0.1, seed=k).numpy() for k in range(3)]
    seed = 77
    info, co, ref = oracle_sketches(graph, rels, weights, m, d, seed)
    sk = _run(graph, rels, weights, m, d, seed, unit=True)
    for k in range(3):
        assert np.array_equal(sk.read_sketch(k), ref[k])
    est = sk.estimate(reps=True)
    reps = []
    for t in range(d):
        c = [ref[k][t] for k in range(3)]
        assert max(int(np.abs(x).sum()) for x in c) ** 3 < 2 ** 63
        x = _chain3_eq5(info, c, m)
        reps.append(x)
        assert est["rep_ints"][t] == x, (t, est["rep_ints"][t], x)
    assert est["value"] == float(oracle.median_lower(reps))
    sk.close()


def test_batched_any_m():
    """The persistent batched update and the batched estimate with m not a power of two."""
    specs = [
        W.QuerySpec(W.chain(3), 1000, 5, (3000, 40_000, 500), 11),
        W.QuerySpec(W.star(4), 60_000, 3, (100_000, 7_000, 300, 90_000), 12),
        W.QuerySpec(W.chain(3), 65_534, 9, (200_000, 150_000, 100_000), 13),
        W.QuerySpec(W.single_join(), 12_345, 5, (50_000, 60_000), 14),
        W.QuerySpec(W.fig3_query(), 300, 5, (3000, 4000, 100, 2000), 15),
        W.QuerySpec(W.chain(4), 1 << 12, 5, (5000, 6000, 7000, 8000), 16),
    ]
    data = []
    for qi, sp in enumerate(specs):
        data.append([keys_u32(W.relation_keys(sp.graph, k, sp.n_per_rel[k], "zipf", config=800 + qi, s=1.2,
                                              D=10 ** 5)) for k in range(sp.graph.n_rel)])
    plain, batched, items = [], [], []
    for sp, rels in zip(specs, data):
        a = csk.Sketch(sp.graph, sp.m, sp.d, sp.sketch_seed)
        b = csk.Sketch(sp.graph, sp.m, sp.d, sp.sketch_seed)
        for k, keys in enumerate(rels):
            kd = to_device_keys(keys)
            a.update(k, kd)
            items.append((b, k, kd, None, False))
        plain.append(a)
        batched.append(b)
    bt = csk.Batch()
    bt.update(items)
    torch.cuda.synchronize()
    for qi, sp in enumerate(specs):
        info, co, ref = oracle_sketches(sp.graph, data[qi], None, sp.m, sp.d, sp.sketch_seed)
        for k in range(sp.graph.n_rel):
            assert np.array_equal(batched[qi].read_sketch(k), ref[k]), (qi, k)
            assert np.array_equal(plain[qi].read_sketch(k), ref[k]), (qi, k)
    got = bt.estimate(batched, reps=True)
    for qi, sk in enumerate(plain):
        assert got[qi] == sk.estimate(reps=True), qi
    for qi in (0, 3, 4):
        sp = specs[qi]
        info = oracle.analyze(sp.graph)
        reps, med = oracle.estimate(info, [plain[qi].read_sketch(k) for k in range(sp.graph.n_rel)], sp.m,
                                    method="ntt")
        assert got[qi]["rep_ints"] == reps, qi
    bt.close()
    for s in plain + batched:
        s.close()


def test_tuner_any_m():
    graph, n, m, d = W.chain(3), 200_000, 50_000, 5
    rels = _rels(graph, n, "zipf", 10 ** 6, config=901)
    info, co, ref = oracle_sketches(graph, rels, None, m, d, 5)
    csk.tune_clear()
    sk = csk.Sketch(graph, m, d, 5)
    for k in range(3):
        rep = csk.tune_update(sk, k, to_device_keys(rels[k]))
        ran = [c for c in rep["candidates"] if c["valid"] != 0]
        assert rep["best"]["valid"] == 1 and all(c["valid"] == 1 for c in ran), rep["candidates"]
    for k in range(3):
        sk.update(k, to_device_keys(rels[k]))
    torch.cuda.synchronize()
    for k in range(3):
        assert np.array_equal(sk.read_sketch(k), ref[k])
    sk.close()
    csk.tune_clear()
