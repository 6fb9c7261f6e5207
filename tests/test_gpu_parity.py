"""GPU path versus the CPU oracle, through the C ABI.

Sketches must be bit-identical; estimates must equal the oracle's exact integers for
every repetition (the library resolves every repetition exactly unless flagged).
"""
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


def _run_gpu(graph, rels, weights, m, d, seed, strategy=0, grid=0, unit=False, compact=True, counters16=True,
             extra_flags=0):
    sk = csk.Sketch(graph, m, d, seed)
    for k, keys in enumerate(rels):
        kd = to_device_keys(keys)
        wd = None if weights is None else torch.from_numpy(weights[k]).cuda()
        sk.update(k, kd, wd, strategy=strategy, grid=grid, unit_weights=unit, compact=compact,
                  counters16=counters16, extra_flags=extra_flags)
    torch.cuda.synchronize()
    return sk


def _rels(graph, n, dist, D, config, s=1.1):
    return [keys_u32(W.relation_keys(graph, k, n, dist, config=config, s=s, D=D)) for k in range(graph.n_rel)]


# --------------------------------------------------------------------------- setup checks

@pytest.mark.parametrize("graph", [W.single_join(), W.chain(3), W.chain(5), W.star(4), W.fig3_query(),
                                   W.multiway_star(3)])
def test_coefficients_and_components_match(graph):
    _say("coeffs", graph.name)
    info = oracle.analyze(graph)
    for seed in (0, 7, 2 ** 63 + 5):
        sk = csk.Sketch(graph, 1024, 5, seed)
        s, b = sk.coefficients()
        co = oracle.draw_coefficients(seed, 5, len(info.edges), info.n_comp)
        assert np.array_equal(s, co.sign_array())
        assert np.array_equal(b, co.bin_array())
        assert sk.components() == info.psi
        sk.close()


def test_partition_strategy_refuses_general_weights():
    sk = csk.Sketch(W.chain(3), 1 << 16, 3, 1)
    keys = torch.zeros(100, 1, dtype=torch.int32, device="cuda")
    w = torch.full((100,), 3, dtype=torch.int64, device="cuda")
    with pytest.raises(csk.CsError) as e:
        sk.update(0, keys, w, strategy=csk.UPDATE_PARTITION)
    assert e.value.status == csk.CS_EINVAL
    sk.update(0, keys, w)  # auto picks a strategy that handles any weights
    torch.cuda.synchronize()
    sk.close()


def test_invalid_arguments_rejected():
    with pytest.raises(csk.CsError) as e:
        csk.Sketch(W.chain(3), (1 << 20) + 1, 5, 1)   # m above 2^20
    assert e.value.status == csk.CS_EINVAL
    with pytest.raises(csk.CsError) as e:
        csk.Sketch(W.JoinGraph(3, (0, 1, 2), ((0, 1), (1, 2), (0, 2))), 1024, 5, 1)
    assert e.value.status == csk.CS_EGRAPH
    with pytest.raises(csk.CsError) as e:
        csk.Sketch(W.chain(3), 1024, 65, 1)
    assert e.value.status == csk.CS_EINVAL
    sk = csk.Sketch(W.chain(3), 1024, 5, 1)
    keys = torch.zeros(10, 1, dtype=torch.int32, device="cuda")
    with pytest.raises(csk.CsError):
        sk.update(3, keys)
    sk.update(0, keys[:0])  # n = 0 is a no-op
    assert not sk.read_sketch(0).any()


# --------------------------------------------------------------------------- sketch parity (Alg. 2)

SKETCH_CASES = [
    # graph, n, m, d, dist, D, weights
    (W.single_join(), 100_000, 1024, 5, "uniform", 10_000, None),
    (W.chain(3), 65, 2, 1, "uniform", 50, "pm1"),
    (W.chain(3), 1, 16, 3, "uniform", 50, None),
    (W.chain(3), 64, 1 << 16, 9, "zipf", 10 ** 6, None),
    (W.chain(3), 20_011, 1 << 16, 9, "zipf", 10 ** 6, "big"),
    (W.chain(5), 30_000, 1 << 13, 15, "zipf", 10 ** 7, "pm1"),
    (W.star(5), 12_345, 4096, 5, "zipf", 1000, None),
    (W.fig3_query(), 7_777, 512, 7, "uniform", 200, "big"),
    (W.multiway_star(4), 5_000, 256, 4, "zipf", 100, None),
    (W.chain(3), 50_000, 1 << 18, 3, "zipf", 10 ** 7, None),
    (W.chain(3), (1 << 21) + 12_345, 1 << 16, 2, "zipf", 10 ** 6, "pm1"),
    (W.star(4), 70_000, 1 << 20, 2, "uniform", 10 ** 9, None),
]


def _weights(kind, graph, n):
    if kind is None:
        return None
    if kind == "pm1":
        return [W.turnstile_weights(n, 0.1, seed=k).numpy() for k in range(graph.n_rel)]
    return [W.random_weights(n, -2 ** 62, 2 ** 62, seed=50 + k).numpy() for k in range(graph.n_rel)]


@pytest.mark.parametrize("case", range(len(SKETCH_CASES)))
@pytest.mark.parametrize("compact", [False, True])
def test_sketch_segmented_kernel_variants(case, compact):
    """The segmented strategy with 16-bit counters off, with and without the compacting
    kernel for bucket-range segments: every kernel variant must give the same counters."""
    graph, n, m, d, dist, D, wk = SKETCH_CASES[case]
    _say("sketch variant", case, graph.name, n, m, d, "compact", compact)
    rels = _rels(graph, n, dist, D, config=90 + case)
    weights = _weights(wk, graph, n)
    info, co, ref = oracle_sketches(graph, rels, weights, m, d, 1000 + case)
    sk = _run_gpu(graph, rels, weights, m, d, 1000 + case, strategy=2, unit=(wk == "pm1"), compact=compact,
                  counters16=False)
    for k in range(graph.n_rel):
        assert np.array_equal(sk.read_sketch(k), ref[k]), k
    sk.close()


@pytest.mark.parametrize("case", range(len(SKETCH_CASES)))
@pytest.mark.parametrize("strategy", [0, 2])
def test_sketch_full_reduction_path(case, strategy):
    """Hashes normally skip the full mod-p reduction (it changes a result only within 3 of
    a multiple of p); with the test flag most tuples take it: the counters must not change."""
    graph, n, m, d, dist, D, wk = SKETCH_CASES[case]
    _say("sketch full-reduction path", case, graph.name, n, m, d, "strategy", strategy)
    rels = _rels(graph, n, dist, D, config=90 + case)
    weights = _weights(wk, graph, n)
    info, co, ref = oracle_sketches(graph, rels, weights, m, d, 1000 + case)
    sk = _run_gpu(graph, rels, weights, m, d, 1000 + case, strategy=strategy, unit=(wk == "pm1"),
                  extra_flags=csk.UPDATE_TEST_FULL_REDUCTION)
    for k in range(graph.n_rel):
        assert np.array_equal(sk.read_sketch(k), ref[k]), k
    sk.close()


@pytest.mark.parametrize("m", [1 << 16, 1 << 17])
@pytest.mark.parametrize("kind", ["all_plus", "all_minus", "alternating", "two_hot"])
def test_counters16_spill(kind, m):
    """16-bit LDS counters hand multiples of 2^14 to the int64 sketch; counters driven far
    past +-2^15 in either direction, or swinging across the spill thresholds, stay exact."""
    graph = W.single_join()
    n, d, seed = 400_000, 5, 77
    rng = np.random.default_rng(9)
    if kind == "two_hot":
        k0 = rng.choice(np.array([3, 11], dtype=np.uint32), size=(n, 1))
    else:
        k0 = np.full((n, 1), 12345, dtype=np.uint32)
    k1 = rng.integers(0, 1000, size=(n, 1), dtype=np.uint32)
    if kind == "all_plus":
        w0 = np.ones(n, dtype=np.int64)
    elif kind == "all_minus":
        w0 = -np.ones(n, dtype=np.int64)
    elif kind == "alternating":
        # runs of 30 000 of one sign, then the other: the counter swings across both thresholds
        w0 = np.where((np.arange(n) // 30_000) % 2 == 0, 1, -1).astype(np.int64)
    else:
        w0 = np.where(rng.random(n) < 0.8, 1, -1).astype(np.int64)
    w1 = -np.ones(n, dtype=np.int64)
    rels, weights = [k0, k1], [w0, w1]
    _say("counters16", kind, n, m, d)
    info, co, ref = oracle_sketches(graph, rels, weights, m, d, seed)
    # grid=1: one chunk, so one workgroup per repetition sees every tuple
    for c16, grid in ((True, 1), (True, 3), (True, 0), (False, 1)):
        sk = _run_gpu(graph, rels, weights, m, d, seed, strategy=2, grid=grid, unit=True, counters16=c16)
        for k in range(2):
            assert np.array_equal(sk.read_sketch(k), ref[k]), (c16, grid, k)
        sk.close()


@pytest.mark.parametrize("m", [1 << 16, 1 << 18])
@pytest.mark.parametrize("offset", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [1, 3, 4, 4097, 100_003])
def test_counters16_alignment_and_tails(offset, n, m):
    """16-bit kernel: key and weight arrays starting at every 4-byte offset modulo 16 bytes
    (the quad loads need 16-byte alignment, the other form takes any), chunk lengths
    with 0-3 tuples after the last whole quad, one or several chunks, weights +1 (NULL)
    and +-1."""
    graph = W.chain(3)
    d, seed = 3, 5
    _say("counters16 alignment", offset, n, m)
    rels = _rels(graph, n + offset, "zipf", 10 ** 4, config=95)
    weights = [W.turnstile_weights(n + offset, 0.2, seed=k).numpy() for k in range(graph.n_rel)]
    refs = {}
    for use_w in (False, True):
        _, _, refs[use_w] = oracle_sketches(graph, [r[offset:] for r in rels],
                                            [w[offset:] for w in weights] if use_w else None, m, d, seed)
    for grid in (0, 3):
        for use_w in (False, True):
            sk = csk.Sketch(graph, m, d, seed)
            for k in range(graph.n_rel):
                kd = to_device_keys(rels[k])[offset:]
                wd = torch.from_numpy(weights[k]).cuda()[offset:] if use_w else None
                sk.update(k, kd, wd, strategy=2, grid=grid, unit_weights=True)
            torch.cuda.synchronize()
            for k in range(graph.n_rel):
                assert np.array_equal(sk.read_sketch(k), refs[use_w][k]), (grid, use_w, k)
            sk.close()


@pytest.mark.parametrize("case", range(len(SKETCH_CASES)))
@pytest.mark.parametrize("strategy", [0, 1, 2, 3, 4])
def test_sketch_bit_exact(case, strategy):
    graph, n, m, d, dist, D, wk = SKETCH_CASES[case]
    if strategy == 4 and (wk == "big" or max(len(graph.columns(k)) for k in range(graph.n_rel)) > 2):
        pytest.skip("partition strategy: +-1 weights and at most two key columns")
    if strategy in (1, 3) and n > 1_000_000:
        pytest.skip("global-atomic strategies: kept to the small cases")
    _say("sketch", case, graph.name, n, m, d, dist, wk, "strategy", strategy)
    rels = _rels(graph, n, dist, D, config=90 + case)
    weights = _weights(wk, graph, n)
    seed = 1000 + case
    info, co, ref = oracle_sketches(graph, rels, weights, m, d, seed)
    sk = _run_gpu(graph, rels, weights, m, d, seed, strategy=strategy, unit=(wk == "pm1"))
    for k in range(graph.n_rel):
        got = sk.read_sketch(k)
        assert np.array_equal(got, ref[k]), (k, np.argwhere(got != ref[k])[:5])
    sk.close()


def test_sketch_batches_and_misaligned_keys():
    """Streaming in uneven batches, including a two-column key buffer that is only
    4-byte aligned, gives the same counters as one batch (linearity, Sec. 2.2)."""
    graph = W.chain(3)
    n, m, d, seed = 10_001, 4096, 5, 3
    rels = _rels(graph, n, "zipf", 10 ** 5, config=77)
    info, co, ref = oracle_sketches(graph, rels, None, m, d, seed)
    sk = csk.Sketch(graph, m, d, seed)
    for k, keys in enumerate(rels):
        a = keys.shape[1]
        buf = np.zeros(n * a + 1, dtype=np.uint32)
        buf[1:] = keys.reshape(-1)
        dev = torch.from_numpy(buf.view(np.int32)).cuda()
        flat = dev[1:]  # 4-byte aligned only
        cuts = [0, 1, 64, 1000, 5000, n]
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            part = flat[lo * a:hi * a].view(hi - lo, a)
            sk.update(k, part)
    torch.cuda.synchronize()
    for k in range(graph.n_rel):
        assert np.array_equal(sk.read_sketch(k), ref[k])


@pytest.mark.parametrize("strategy", [0, 1, 2, 3, 4])
def test_adversarial_keys(strategy):
    """All tuples on one key, the all-ones key pair, and keys at the uint32 limits."""
    graph = W.chain(3)
    n, m, d, seed = 50_000, 1 << 16, 3, 21
    rng = np.random.default_rng(5)
    rels = [np.full((n, 1), 7, dtype=np.uint32),
            np.where(rng.random((n, 2)) < 0.5, 0xFFFFFFFF, 0).astype(np.uint32),
            rng.choice(np.array([0, 1, 0xFFFFFFFE, 0xFFFFFFFF], dtype=np.uint32), size=(n, 1))]
    weights = [W.turnstile_weights(n, 0.3, seed=k).numpy() for k in range(3)]
    info, co, ref = oracle_sketches(graph, rels, weights, m, d, seed)
    sk = _run_gpu(graph, rels, weights, m, d, seed, strategy=strategy, unit=True)
    for k in range(3):
        assert np.array_equal(sk.read_sketch(k), ref[k]), k
    sk.close()


def test_turnstile_insert_delete_and_reset():
    graph = W.chain(3)
    n, m, d = 5000, 1024, 5
    rels = _rels(graph, n, "zipf", 1000, config=78)
    sk = csk.Sketch(graph, m, d, 11)
    for k, keys in enumerate(rels):
        kd = to_device_keys(keys)
        w = torch.randint(-1000, 1000, (n,), dtype=torch.int64, device="cuda")
        sk.update(k, kd, w)
        sk.update(k, kd, -w)
    assert all(not sk.read_sketch(k).any() for k in range(3))
    sk.update(0, to_device_keys(rels[0]))
    assert sk.read_sketch(0).any()
    sk.reset()
    assert not sk.read_sketch(0).any()


def test_merge_is_sum():
    graph = W.star(3)
    n, m, d, seed = 3000, 2048, 5, 9
    rels = _rels(graph, n, "uniform", 500, config=79)
    a = _run_gpu(graph, [r[: n // 2] for r in rels], None, m, d, seed)
    b = _run_gpu(graph, [r[n // 2:] for r in rels], None, m, d, seed)
    a.merge_from(b)
    torch.cuda.synchronize()
    info, co, ref = oracle_sketches(graph, rels, None, m, d, seed)
    for k in range(3):
        assert np.array_equal(a.read_sketch(k), ref[k])


# --------------------------------------------------------------------------- estimate parity (Eq. 5 / Alg. 3)

INT128_EXACT = 2 ** 125   # the library represents exact results below this magnitude


def _check_estimate(graph, sk, ref_sketches, m, d, info):
    """Every repetition below 2^125 must equal the oracle's exact integer; beyond it the
    fp64 value must be within 1e-12 relative; the median must match the oracle's."""
    est = sk.estimate(reps=True)
    reps = []
    for t in range(d):
        exact = oracle.estimate_alg3(info, [ref_sketches[k][t] for k in range(graph.n_rel)], m, method="ntt")
        reps.append(exact)
        if abs(exact) < INT128_EXACT:
            assert est["rep_ints"][t] is not None, (t, est)
            assert est["rep_ints"][t] == exact, (t, est["rep_ints"][t], exact, est["rep_bounds"][t])
            assert est["rep_values"][t] == float(exact)
        else:
            assert abs(est["rep_values"][t] - exact) <= 1e-12 * abs(exact), (t, est["rep_values"][t], exact)
    med = oracle.median_lower(reps)
    if abs(med) < INT128_EXACT:
        assert est["exact"]
        assert est["value"] == float(med)
    else:
        assert abs(est["value"] - med) <= 1e-12 * abs(med)
    if -2 ** 63 <= med < 2 ** 63:
        assert est["value_i64"] == med
    return est


EST_CASES = [
    # graph, n, m, d, dist, D, s, weights
    (W.single_join(), 100_000, 1024, 5, "uniform", 10_000, 1.0, None),
    (W.chain(3), 2_000, 64, 5, "zipf", 100, 1.1, None),
    (W.chain(3), 200_000, 1 << 16, 9, "zipf", 10 ** 6, 1.1, None),
    (W.chain(4), 50_000, 8192, 5, "zipf", 10 ** 4, 1.2, "pm1"),
    (W.chain(5), 100_000, 1 << 14, 7, "zipf", 10 ** 5, 1.5, None),
    (W.star(4), 30_000, 4096, 5, "zipf", 1000, 1.2, None),
    (W.star(6), 10_000, 1024, 9, "zipf", 1000, 1.2, None),
    (W.chain(3), 3_000, 1 << 12, 5, "zipf", 10 ** 4, 1.1, "big"),
    (W.chain(4), 3_000, 1 << 10, 5, "zipf", 10 ** 4, 1.1, "huge"),
    (W.fig3_query(), 3_000, 256, 5, "zipf", 500, 1.1, None),
    (W.multiway_star(3), 2_000, 128, 3, "uniform", 50, 1.0, None),
    (W.chain(3), 100_000, 1 << 18, 3, "zipf", 10 ** 7, 1.0, None),
    (W.chain(6), 5_000, 2, 4, "uniform", 30, 1.0, None),
]


@pytest.mark.parametrize("case", range(len(EST_CASES)))
def test_estimate_exact(case):
    graph, n, m, d, dist, D, s, wk = EST_CASES[case]
    _say("estimate", case, graph.name, n, m, d, dist, s, wk)
    rels = _rels(graph, n, dist, D, config=60 + case, s=s)
    weights = None
    if wk == "pm1":
        weights = [W.turnstile_weights(n, 0.1, seed=k).numpy() for k in range(graph.n_rel)]
    elif wk == "big":
        weights = [W.random_weights(n, -2 ** 30, 2 ** 30, seed=60 + k).numpy() for k in range(graph.n_rel)]
    elif wk == "huge":
        weights = [W.random_weights(n, -2 ** 45, 2 ** 45, seed=60 + k).numpy() for k in range(graph.n_rel)]
    seed = 7 + case
    info, co, ref = oracle_sketches(graph, rels, weights, m, d, seed)
    sk = _run_gpu(graph, rels, weights, m, d, seed)
    for k in range(graph.n_rel):
        assert np.array_equal(sk.read_sketch(k), ref[k])
    est = _check_estimate(graph, sk, ref, m, d, info)
    _say("  value", est["value"], "modular reps", est["n_modular"])
    sk.close()


def test_empty_sketches_estimate_zero():
    for graph in (W.single_join(), W.chain(4), W.fig3_query()):
        sk = csk.Sketch(graph, 1024, 3, 1)
        est = sk.estimate(reps=True)
        assert est["exact"] and est["value"] == 0.0 and est["value_i64"] == 0
        assert est["rep_ints"] == [0, 0, 0]
        sk.close()


def test_estimate_prime_count_changes_between_calls():
    """The speculative modular step sizes itself from the previous estimate: a later
    estimate that needs more primes (large weights added) or fewer (the sketch reset and
    refilled small) must still be exact."""
    graph, n, m, d = W.chain(3), 4_000, 1 << 12, 5
    rels = _rels(graph, n, "zipf", 10 ** 4, config=83)
    info = oracle.analyze(graph)
    sk = csk.Sketch(graph, m, d, 9)
    big = [W.random_weights(n, -2 ** 45, 2 ** 45, seed=90 + k).numpy() for k in range(graph.n_rel)]
    for phase, weights in enumerate((None, big, None)):
        if phase == 2:
            sk.reset()
        for k in range(graph.n_rel):
            wd = None if weights is None else torch.from_numpy(weights[k]).cuda()
            sk.update(k, to_device_keys(rels[k]), wd)
        torch.cuda.synchronize()
        ref = [sk.read_sketch(k) for k in range(graph.n_rel)]
        _say("phase", phase)
        est = _check_estimate(graph, sk, ref, m, d, info)
        _say("  modular reps", est["n_modular"])
    sk.close()


def test_estimate_is_deterministic():
    graph = W.chain(4)
    n, m, d = 50_000, 1 << 15, 5
    rels = _rels(graph, n, "zipf", 10 ** 5, config=81)
    sk = _run_gpu(graph, rels, None, m, d, 5)
    a = sk.estimate(reps=True)
    b = sk.estimate(reps=True)
    assert a == b


def test_inner_product_beyond_int128_is_flagged():
    """The two-relation plan sums int64 products in 128-bit integers: when the sum of
    |products| may reach 2^127 the repetition is returned as an fp64 value flagged
    inexact (within 1e-12 of the exact sum), never as a wrapped integer.  Weights of
    1.5 * 2^62 on 13 keys over 4 buckets drive two repetitions past 2^127 (values
    computed exactly by the oracle in Python integers)."""
    graph, m, d, seed = W.single_join(), 4, 9, 3
    keys = (np.arange(13, dtype=np.uint32) * 7919).reshape(-1, 1)
    w = np.full(13, 2 ** 62 + 2 ** 61, dtype=np.int64)
    info, co, ref = oracle_sketches(graph, [keys, keys], [w, w], m, d, seed)
    sk = _run_gpu(graph, [keys, keys], [w, w], m, d, seed)
    est = sk.estimate(reps=True)
    reps = [oracle.estimate_alg3(info, [ref[0][t], ref[1][t]], m, method="ntt") for t in range(d)]
    assert sum(x >= 2 ** 127 for x in reps) >= 1
    flagged = 0
    for t, x in enumerate(reps):
        if est["rep_ints"][t] is not None:
            assert est["rep_ints"][t] == x and x < 2 ** 127, (t, x)
        else:
            flagged += 1
            assert x >= 2 ** 125
            assert abs(est["rep_values"][t] - x) <= 1e-12 * abs(x), (t, est["rep_values"][t], x)
    assert flagged >= sum(x >= 2 ** 127 for x in reps)
    med = oracle.median_lower(reps)
    assert abs(est["value"] - med) <= 1e-12 * abs(med)
    sk.close()
