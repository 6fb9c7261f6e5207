"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each compares it with an independent
route (published generator outputs, a power-sum hash instead of Horner, the explicit
sketch matrix, the paper's worked examples and closed forms, Eq. 5 by enumeration
versus Alg. 3, the theorems' expectation and variance, special cases that reduce to
the Count sketch and to the AMS multi-join estimator)."""
import json
import math
import os
import random

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _sketch_all(info, rels, m, coeffs, weights=None):
    return [oracle.create_sketch(info, k, rels[k], None if weights is None else weights[k], m, coeffs)
            for k in range(info.n_rel)]


# --------------------------------------------------------------------------- coefficient stream

def test_splitmix64_published_vectors():
    for vec in _load("splitmix64_vectors.json")["vectors"]:
        g = oracle.splitmix64(vec["seed"])
        got = [next(g) for _ in vec["outputs"]]
        assert got == [int(s, 0) for s in vec["outputs"]]


def test_coefficients_uniform_range_and_order():
    c = oracle.draw_coefficients(99, d=3, n_edges=2, n_comps=2)
    g = oracle.splitmix64(99)
    flat = []
    for t in range(3):
        flat += [x for e in range(2) for x in c.sign[t][e]]
        flat += [x for q in range(2) for x in c.bins[t][q]]
    assert flat == [next(g) >> 3 for _ in flat]   # no redraw happens for this seed
    assert all(0 <= x < oracle.P61 for x in flat)


def test_workload_uniforms_match_splitmix_stream():
    import torch
    u = W.splitmix64_at(5, torch.arange(4)).tolist()
    g = oracle.splitmix64(5)
    ref = [next(g) for _ in range(4)]
    assert [x & ((1 << 64) - 1) for x in u] == ref


# --------------------------------------------------------------------------- hashes

def test_c_horner_hash_matches_power_sum():
    rng = random.Random(1)
    for _ in range(2000):
        coef = [rng.randrange(oracle.P61) for _ in range(4)]
        x = rng.randrange(1 << 32)
        arr = np.array(coef, dtype=np.uint64)
        got = oracle.lib().or_poly_hash(arr.ctypes.data, 3, x)
        assert got == oracle.poly_value(coef, x)
        assert got == (coef[0] + coef[1] * x + coef[2] * x * x + coef[3] * x ** 3) % oracle.P61


def test_hash_edge_values():
    p = oracle.P61
    for coef in ([p - 1] * 4, [0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0]):
        for x in (0, 1, (1 << 32) - 1, 12345):
            arr = np.array(coef, dtype=np.uint64)
            assert oracle.lib().or_poly_hash(arr.ctypes.data, 3, x) == oracle.poly_value(coef, x)


def test_sign_and_bin_are_roughly_uniform():
    c = oracle.draw_coefficients(3, 1, 1, 1)
    xs = range(20000)
    signs = [oracle.sign_value(c.sign[0][0], x) for x in xs]
    assert abs(sum(signs)) < 5 * math.sqrt(len(signs))
    m = 16
    counts = np.bincount([oracle.bin_value(c.bins[0][0], x, m) for x in xs], minlength=m)
    chi2 = float(((counts - len(xs) / m) ** 2 / (len(xs) / m)).sum())
    assert chi2 < 50  # 15 dof


# --------------------------------------------------------------------------- join graph (Fig. 3)

def test_fig3_graph_analysis():
    g = _load("fig3_query.json")
    info = oracle.analyze(W.fig3_query())
    comps = {}
    for u, q in enumerate(info.psi):
        comps.setdefault(q, []).append(u)
    assert sorted(comps.values()) == g["components"]
    assert info.omega[1] == g["omega_R1"]
    assert info.gamma[1] == g["gamma_1"]
    joins = sorted(sorted(e) for e in g["R1_tuple_sign_joins"])
    used = sorted(sorted(info.edges[info.edge_of(u, v)]) for u in info.omega[1] for v in info.gamma[u])
    assert used == joins


@pytest.mark.parametrize("bad", [
    W.JoinGraph(2, (0, 1), ()),                        # not joined
    W.JoinGraph(2, (0, 0, 1), ((0, 2), (1, 2))),       # two joins between two relations: cycle
    W.JoinGraph(3, (0, 1, 2), ((0, 1), (1, 2), (0, 2))),  # triangle
    W.JoinGraph(2, (0, 0), ((0, 1),)),                 # join inside a relation
    W.JoinGraph(3, (0, 1, 2, 2), ((0, 1), (2, 3))),    # self edge inside relation 2
])
def test_invalid_graphs_rejected(bad):
    with pytest.raises(oracle.GraphError):
        oracle.analyze(bad)


# --------------------------------------------------------------------------- sketch (Alg. 2, Eq. 4, Fig. 4)

def test_fig4_worked_example():
    g = _load("fig4_worked_example.json")
    m = g["m"]
    # a two-attribute relation whose tuple (a, b) takes the worked example's hashes
    graph = W.JoinGraph(3, (0, 1, 1, 2), ((0, 1), (2, 3)))
    info = oracle.analyze(graph)
    a_key, b_key = 10, 20
    bins = {a_key: g["item_a"]["bin"], b_key: g["item_b"]["bin"]}
    signs = {a_key: g["item_a"]["sign"], b_key: g["item_b"]["sign"]}
    c = oracle.create_sketch_py(info, 1, [(a_key, b_key)], None, m, 0,
                                sign_fn=lambda e, x: signs[x], bin_fn=lambda q, x: bins[x])
    assert c == g["convolution"]
    # the same through the C accumulate path with the tuple hashes supplied
    out = np.zeros(m, dtype=np.int64)
    tb = np.array([bins[a_key] + bins[b_key]], dtype=np.uint64)
    ts = np.array([signs[a_key] * signs[b_key]], dtype=np.int32)
    tw = np.array([1], dtype=np.int64)
    oracle.lib().or_accumulate(tb.ctypes.data, ts.ctypes.data, tw.ctypes.data, 1, m, out.ctypes.data)
    assert out.tolist() == g["convolution"]
    # Def. 2.2 circular convolution and the Hadamard product of the single-item sketches
    sa, sb = g["item_a"]["sketch"], g["item_b"]["sketch"]
    conv = [sum(sa[i] * sb[(j - i) % m] for i in range(m)) for j in range(m)]
    assert conv == g["convolution"]
    assert [x * y for x, y in zip(sa, sb)] == g["hadamard"]


def _explicit_matrix_sketch(info, k, m, coeffs, t, freq, domain):
    """c = Pi vec(F) with Pi_{j,i} = S(i) 1(H(i) = j) (Sec. 2.2; Eq. 2-4), built over the
    whole tiny domain with power-sum hashes."""
    cols = info.omega[k]
    c = [0] * m
    for tup in np.ndindex(*([domain] * len(cols))):
        S, H = 1, 0
        for col, u in enumerate(cols):
            H += oracle.poly_value(coeffs.bins[t][info.psi[u]], tup[col]) % m
            for v in info.gamma[u]:
                val = oracle.poly_value(coeffs.sign[t][info.edge_of(u, v)], tup[col])
                S *= -1 if val & 1 else 1
        c[H % m] += S * freq.get(tuple(int(x) for x in tup), 0)
    return c


@pytest.mark.parametrize("graph", [W.chain(3), W.star(4), W.fig3_query(), W.chain(5)])
def test_sketch_equals_explicit_matrix(graph):
    info = oracle.analyze(graph)
    m, d, domain = 7, 3, 5
    coeffs = oracle.draw_coefficients(11, d, len(info.edges), info.n_comp)
    for k in range(info.n_rel):
        keys = W.random_small_relation(graph, k, 40, domain, seed=100 + k).numpy()
        w = W.random_weights(40, -3, 5, seed=200 + k).numpy()
        c = oracle.create_sketch(info, k, keys, w, m, coeffs)
        F = oracle.frequency_tensor(keys, w)
        for t in range(d):
            assert c[t].tolist() == _explicit_matrix_sketch(info, k, m, coeffs, t, F, domain)
            assert c[t].tolist() == oracle.create_sketch_py(info, k, keys.tolist(), w, m, t, coeffs=coeffs)


def test_linearity_and_turnstile():
    graph = W.chain(3)
    info = oracle.analyze(graph)
    m = 64
    coeffs = oracle.draw_coefficients(5, 4, len(info.edges), info.n_comp)
    keys = W.relation_keys(graph, 1, 5000, "zipf", config=9, s=1.1, D=1000).numpy()
    w = W.random_weights(5000, -2 ** 40, 2 ** 40, seed=3).numpy()
    full = oracle.create_sketch(info, 1, keys, w, m, coeffs)
    a = oracle.create_sketch(info, 1, keys[:1234], w[:1234], m, coeffs)
    b = oracle.create_sketch(info, 1, keys[1234:], w[1234:], m, coeffs)
    assert np.array_equal(full, a + b)
    perm = np.random.default_rng(0).permutation(5000)
    assert np.array_equal(full, oracle.create_sketch(info, 1, keys[perm], w[perm], m, coeffs))
    # insert then delete returns every counter to zero
    both = oracle.create_sketch(info, 1, np.concatenate([keys, keys]), np.concatenate([w, -w]), m, coeffs)
    assert not both.any()


def test_filter_rows_pins():
    """Filtered ingestion: the kept rows are exactly those a per-row check of every
    predicate accepts (brute force), and their sketch equals the sketch of all rows with
    the failing rows' Delta set to 0 (linearity: a zero change adds nothing)."""
    graph = W.chain(3)
    info = oracle.analyze(graph)
    m = 64
    coeffs = oracle.draw_coefficients(11, 3, len(info.edges), info.n_comp)
    n = 3000
    keys = W.relation_keys(graph, 1, n, "zipf", config=12, s=1.1, D=500).numpy()
    w = W.random_weights(n, -50, 50, seed=4).numpy()
    rng = np.random.default_rng(2)
    attrs = rng.integers(0, 2 ** 32, size=(n, 3), dtype=np.uint64).astype(np.uint32)
    attrs[:, 1] = rng.integers(0, 10, size=n)
    preds = [(1, 2, 6), (0, 0, 0xC0000000), (2, 0x10000000, 0xFFFFFFFF)]
    fk, fw = oracle.filter_rows(keys, w, attrs, preds)
    brute = [i for i in range(n) if all(lo <= int(attrs[i, c]) <= hi for c, lo, hi in preds)]
    assert 0 < len(brute) < n
    assert np.array_equal(fk, keys[brute]) and np.array_equal(fw, w[brute])
    zeroed = w.copy()
    mask = np.zeros(n, dtype=bool)
    mask[brute] = True
    zeroed[~mask] = 0
    assert np.array_equal(oracle.create_sketch(info, 1, fk, fw, m, coeffs),
                          oracle.create_sketch(info, 1, keys, zeroed, m, coeffs))
    # no predicate keeps everything; an empty range keeps nothing
    assert len(oracle.filter_rows(keys, None, attrs, [])[0]) == n
    assert len(oracle.filter_rows(keys, None, attrs, [(1, 5, 4)])[0]) == 0


def test_counters_wrap_mod_2_64():
    info = oracle.analyze(W.single_join())
    coeffs = oracle.draw_coefficients(1, 1, 1, 1)
    big = np.array([2 ** 62, 2 ** 62, 2 ** 62], dtype=np.int64)
    keys = np.array([[7], [7], [7]], dtype=np.uint32)
    c = oracle.create_sketch(info, 0, keys, big, 4, coeffs)
    s = oracle.sign_value(coeffs.sign[0][0], 7)
    j = oracle.bin_value(coeffs.bins[0][0], 7, 4)
    assert c[0, j] == oracle.wrap_int64(3 * s * 2 ** 62)


def test_null_weights_equal_plus_one():
    info = oracle.analyze(W.chain(2))
    coeffs = oracle.draw_coefficients(8, 2, 1, 1)
    keys = W.relation_keys(W.chain(2), 0, 1000, "uniform", config=9, D=50).numpy()
    a = oracle.create_sketch(info, 0, keys, None, 32, coeffs)
    b = oracle.create_sketch(info, 0, keys, np.ones(1000, dtype=np.int64), 32, coeffs)
    assert np.array_equal(a, b)


# --------------------------------------------------------------------------- estimate (Eq. 5, Alg. 3)

def _random_sketches(info, m, seed, lo=-9, hi=9):
    rng = np.random.default_rng(seed)
    return [rng.integers(lo, hi + 1, size=m).astype(np.int64) for _ in range(info.n_rel)]


@pytest.mark.parametrize("graph", [W.single_join(), W.chain(3), W.chain(4), W.star(4), W.fig3_query(),
                                   W.multiway_star(3), W.chain(5)])
@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6, 8])
def test_eq5_equals_alg3_all_roots(graph, m):
    info = oracle.analyze(graph)
    c = _random_sketches(info, m, seed=m * 7 + info.n_rel)
    ref = oracle.estimate_eq5(info, c, m)
    for root in range(info.n_attr):
        assert oracle.estimate_alg3(info, c, m, root=root, method="direct") == ref
        assert oracle.estimate_alg3(info, c, m, root=root, method="ntt") == ref


def test_alg3_ntt_equals_direct_large_values():
    info = oracle.analyze(W.chain(4))
    m = 32
    c = _random_sketches(info, m, seed=3, lo=-2 ** 62, hi=2 ** 62)
    assert oracle.estimate_alg3(info, c, m, method="ntt") == oracle.estimate_alg3(info, c, m, method="direct")


@pytest.mark.parametrize("m", [24, 100])
def test_alg3_modular_equals_direct_any_m(m):
    """m not a power of two: the modular route (correlations by Def. 3.1 modulo each
    prime, Chinese remaindering) against exact integer vectors, with values large enough
    to need several primes."""
    for graph in (W.chain(4), W.fig3_query(), W.multiway_star(3)):
        info = oracle.analyze(graph)
        c = _random_sketches(info, m, seed=m + info.n_rel, lo=-2 ** 40, hi=2 ** 40)
        assert oracle.estimate_alg3(info, c, m, method="ntt") == oracle.estimate_alg3(info, c, m, method="direct")


@pytest.mark.parametrize("graph", [W.single_join(), W.chain(3), W.chain(4), W.star(4), W.fig3_query(),
                                   W.multiway_star(3), W.chain(5)])
@pytest.mark.parametrize("m", [1, 2, 3, 5, 6, 8])
def test_sparse_alg3_equals_eq5_all_roots(graph, m):
    """The sparse exact evaluation against Eq. 5 by enumeration, with zeros planted in the
    counters (the ring skips them), for every root."""
    info = oracle.analyze(graph)
    c = _random_sketches(info, m, seed=m * 11 + info.n_rel)
    for k, v in enumerate(c):
        v[(k + np.arange(m)) % 3 == 0] = 0
    ref = oracle.estimate_eq5(info, c, m)
    for root in range(info.n_attr):
        assert oracle.estimate_sparse(info, c, m, root=root) == ref


@pytest.mark.parametrize("m", [97, 1 << 10, 1000])
def test_sparse_alg3_equals_dense_on_sparse_sketches(m):
    """Sketches of few tuples at larger m (the regime the sparse ring serves): equal to the
    dense modular route (NTT for powers of two, Def. 3.1 term by term otherwise), with
    values near 2^62 that need several primes there."""
    for graph in (W.chain(3), W.chain(5), W.star(4), W.fig3_query()):
        info = oracle.analyze(graph)
        rng = np.random.default_rng(m + info.n_rel)
        c = []
        for _ in range(info.n_rel):
            v = np.zeros(m, dtype=np.int64)
            idx = rng.choice(m, size=min(m, 40), replace=False)
            v[idx] = rng.integers(-2 ** 62, 2 ** 62, size=len(idx))
            c.append(v)
        assert oracle.estimate_sparse(info, c, m) == oracle.estimate_alg3(info, c, m, method="ntt")


def test_sparse_reversed_correlation_is_detected():
    """Planted mistake in the sparse ring (operands of Def. 3.1 swapped): Eq. 5 catches it."""

    class Reversed(oracle._SparseRing):
        def correlate(self, a, x):
            return super().correlate(x, a)

    info = oracle.analyze(W.chain(3))
    m = 7
    c = _random_sketches(info, m, seed=5)
    ref = oracle.estimate_eq5(info, c, m)
    ring = Reversed(m)
    assert ring.total(oracle._combine_sketches(0, set(), info, c, ring)) != ref


def test_fig3_closed_form():
    info = oracle.analyze(W.fig3_query())
    for m in (3, 5, 8):
        c = _random_sketches(info, m, seed=m)
        closed = sum(c[0][j0] * c[2][j0] * c[1][(j0 + j1) % m] * c[3][j1]
                     for j0 in range(m) for j1 in range(m))
        assert oracle.estimate_eq5(info, c, m) == closed
        assert oracle.estimate_alg3(info, c, m, method="direct") == closed


def test_reversed_correlation_is_detected():
    """The correlation direction matters: swapping the operands of Def. 3.1 changes the
    chain estimate, so the Eq. 5 comparison above pins the direction (planted mistake)."""

    class Reversed(oracle._ExactRing):
        def correlate(self, a, x):
            return super().correlate(x, a)

    info = oracle.analyze(W.chain(3))
    m = 8
    c = _random_sketches(info, m, seed=4)
    ring = Reversed(m)
    wrong = ring.total(oracle._combine_sketches(0, set(), info, c, ring))
    assert wrong != oracle.estimate_eq5(info, c, m)


def test_dropped_sign_is_detected():
    """Planted mistake: a sketch that forgets the second join of attribute 1 in Fig. 3
    differs from the explicit-matrix sketch."""
    graph = W.fig3_query()
    info = oracle.analyze(graph)
    m, domain = 7, 5
    coeffs = oracle.draw_coefficients(11, 1, len(info.edges), info.n_comp)
    keys = W.random_small_relation(graph, 1, 40, domain, seed=101).numpy()
    F = oracle.frequency_tensor(keys)
    ref = _explicit_matrix_sketch(info, 1, m, coeffs, 0, F, domain)
    e_drop = info.edge_of(1, 3)
    wrong = oracle.create_sketch_py(
        info, 1, keys.tolist(), None, m, 0,
        sign_fn=lambda e, x: 1 if e == e_drop else oracle.sign_value(coeffs.sign[0][e], x),
        coeffs=coeffs)
    assert wrong != ref


def test_m1_reduces_to_ams_multijoin():
    """With one bin, the sketch is Eq. 1's single AMS counter and X = prod_k c_k."""
    graph = W.fig3_query()
    info = oracle.analyze(graph)
    coeffs = oracle.draw_coefficients(17, 2, len(info.edges), info.n_comp)
    rels = [W.random_small_relation(graph, k, 30, 6, seed=k).numpy() for k in range(info.n_rel)]
    sk = _sketch_all(info, rels, 1, coeffs)
    for t in range(2):
        for k in range(info.n_rel):
            eq1 = 0
            for tup in rels[k].tolist():
                s = 1
                for col, u in enumerate(info.omega[k]):
                    for v in info.gamma[u]:
                        s *= oracle.sign_value(coeffs.sign[t][info.edge_of(u, v)], tup[col])
                eq1 += s
            assert sk[k][t, 0] == eq1
        X = oracle.estimate_alg3(info, [s[t] for s in sk], 1)
        assert X == math.prod(int(s[t, 0]) for s in sk)


def test_two_relations_is_count_sketch_inner_product():
    info = oracle.analyze(W.single_join())
    m = 16
    c = _random_sketches(info, m, seed=9, lo=-1000, hi=1000)
    assert oracle.estimate_alg3(info, c, m) == int(np.dot(c[0].astype(object), c[1].astype(object)))


def test_chain_spectral_identity_numpy_fft():
    """For a chain, X = (1/m) sum_f prod_k C_k[f] with alternating conjugation, where
    C_k is numpy's FFT of c_k; checks the oracle from the frequency side."""
    info = oracle.analyze(W.chain(5))
    m = 16
    c = _random_sketches(info, m, seed=21, lo=-50, hi=50)
    F = [np.fft.fft(x.astype(np.float64)) for x in c]
    prod = np.ones(m, dtype=np.complex128)
    for k, Ck in enumerate(F):
        prod *= np.conj(Ck) if k % 2 == 0 else Ck
    spectral = prod.sum().real / m
    assert abs(spectral - oracle.estimate_alg3(info, c, m)) < 1e-6 * max(1.0, abs(spectral))


def test_l1_bound_holds():
    for graph in (W.chain(4), W.star(5), W.fig3_query(), W.multiway_star(4)):
        info = oracle.analyze(graph)
        for seed in range(5):
            c = _random_sketches(info, 8, seed=seed)
            assert abs(oracle.estimate_eq5(info, c, 8)) <= oracle.l1_bound(c)


def test_ntt_convolution_matches_direct():
    rng = np.random.default_rng(0)
    for n in (1, 2, 8, 64, 256):
        p = oracle.ntt_primes(n)[0]
        g = oracle.primitive_root(p)
        a = rng.integers(0, p, size=n).astype(np.uint64)
        b = rng.integers(0, p, size=n).astype(np.uint64)
        fast = oracle.ntt((oracle.ntt(a, p, g) * oracle.ntt(b, p, g)) % np.uint64(p), p, g, inverse=True)
        direct = [sum(int(a[i]) * int(b[(j - i) % n]) for i in range(n)) % p for j in range(n)]
        assert fast.tolist() == direct
        assert oracle.ntt(oracle.ntt(a, p, g), p, g, inverse=True).tolist() == a.tolist()


def test_crt_centered():
    primes = oracle.ntt_primes(1024)[:3]
    for x in (0, 1, -1, 123456789012345678901234, -98765432109876543210):
        assert oracle.crt_centered([x % p for p in primes], primes) == x


def test_median_lower():
    assert oracle.median_lower([5, 1, 3]) == 3
    assert oracle.median_lower([4, 1, 3, 2]) == 2
    assert oracle.median_lower([7]) == 7


# --------------------------------------------------------------------------- ground truth and Thm. 3.1

@pytest.mark.parametrize("graph", [W.chain(3), W.star(3), W.fig3_query()])
def test_join_size_definitions_agree(graph):
    info = oracle.analyze(graph)
    freqs = []
    for k in range(info.n_rel):
        keys = W.random_small_relation(graph, k, 12, 3, seed=k).numpy()
        freqs.append(oracle.frequency_tensor(keys))
    assert oracle.join_size(info, freqs) == oracle.join_size_bruteforce(info, freqs)


def test_single_join_size_is_frequency_inner_product():
    graph = W.single_join()
    info = oracle.analyze(graph)
    a = W.random_small_relation(graph, 0, 200, 10, seed=1).numpy()
    b = W.random_small_relation(graph, 1, 300, 10, seed=2).numpy()
    fa, fb = np.bincount(a[:, 0], minlength=10), np.bincount(b[:, 0], minlength=10)
    J = oracle.join_size(info, [oracle.frequency_tensor(a), oracle.frequency_tensor(b)])
    assert J == int(np.dot(fa, fb))


@pytest.mark.parametrize("graph,m", [(W.chain(3), 16), (W.star(3), 16), (W.fig3_query(), 8), (W.single_join(), 8)])
def test_unbiased_and_variance_bound(graph, m):
    """Thm. 3.1: E[X] = join size, Var(X) <= 3^(r-1)/m prod ||F_k||^2, over S seeds with
    one repetition each (the median is biased, so single repetitions are used)."""
    info = oracle.analyze(graph)
    rels = [W.random_small_relation(graph, k, 60, 4, seed=300 + k).numpy() for k in range(info.n_rel)]
    freqs = [oracle.frequency_tensor(r) for r in rels]
    J = oracle.join_size(info, freqs)
    V = oracle.variance_bound(info, freqs, m)
    S = 1500
    xs = []
    for s in range(S):
        coeffs = oracle.draw_coefficients(1000 + s, 1, len(info.edges), info.n_comp)
        sk = _sketch_all(info, rels, m, coeffs)
        xs.append(oracle.estimate_alg3(info, [c[0] for c in sk], m, method="direct"))
    mean = sum(xs) / S
    var = sum((x - mean) ** 2 for x in xs) / (S - 1)
    assert abs(mean - J) <= 5 * math.sqrt(V / S), (mean, J, V)
    assert var <= 1.3 * V, (var, V)


# --------------------------------------------------------------------------- AMS multi-join baseline (Eq. 1)

def test_ams_coefficient_stream_order():
    """With one counter, repetition 0's AMS sign polynomials are the first draws of the
    stream, exactly where Alg. 1's sign polynomials of repetition 0 are."""
    info = oracle.analyze(W.fig3_query())
    E = len(info.edges)
    ams = oracle.draw_ams_coefficients(23, 1, 1, E)
    cs = oracle.draw_coefficients(23, 1, E, info.n_comp)
    assert np.array_equal(ams[0, 0], cs.sign_array()[0])


@pytest.mark.parametrize("graph", [W.chain(3), W.fig3_query(), W.multiway_star(3)])
def test_ams_sketch_equals_definition(graph):
    """Eq. 1 counter by counter with the power-sum hash in Python integers."""
    info = oracle.analyze(graph)
    m, d = 3, 2
    coef = oracle.draw_ams_coefficients(5, d, m, len(info.edges))
    for k in range(info.n_rel):
        keys = W.random_small_relation(graph, k, 25, 6, seed=40 + k).numpy()
        w = W.random_weights(25, -4, 4, seed=60 + k).numpy()
        got = oracle.create_ams_sketch(info, k, keys, w, m, coef)
        for t in range(d):
            for j in range(m):
                ref = 0
                for tup, wt in zip(keys.tolist(), w.tolist()):
                    s = 1
                    for col, u in enumerate(info.omega[k]):
                        for v in info.gamma[u]:
                            s *= oracle.sign_value(coef[t, j, info.edge_of(u, v)].tolist(), tup[col])
                    ref += s * wt
                assert got[t, j] == ref, (k, t, j)


def test_ams_one_counter_is_count_sketch_one_bin():
    """A Count sketch with m = 1 has one counter per repetition holding Eq. 1's sum: fed
    the same sign polynomials, Alg. 2 and Eq. 1 must agree (two independent routines)."""
    graph = W.chain(4)
    info = oracle.analyze(graph)
    d = 3
    cs = oracle.draw_coefficients(31, d, len(info.edges), info.n_comp)
    ams = cs.sign_array().reshape(d, 1, len(info.edges), 4)
    for k in range(info.n_rel):
        keys = W.random_small_relation(graph, k, 200, 20, seed=k).numpy()
        w = W.turnstile_weights(200, 0.2, seed=k).numpy()
        a = oracle.create_sketch(info, k, keys, w, 1, cs)
        b = oracle.create_ams_sketch(info, k, keys, w, 1, ams)
        assert np.array_equal(a, b)


def test_ams_estimate_definition_and_linearity():
    graph = W.chain(3)
    info = oracle.analyze(graph)
    m, d = 5, 3
    coef = oracle.draw_ams_coefficients(8, d, m, len(info.edges))
    rels = [W.random_small_relation(graph, k, 60, 8, seed=k).numpy() for k in range(3)]
    sk = [oracle.create_ams_sketch(info, k, rels[k], None, m, coef) for k in range(3)]
    nums, med = oracle.estimate_ams(sk)
    for t in range(d):
        assert nums[t] == sum(int(sk[0][t, j]) * int(sk[1][t, j]) * int(sk[2][t, j]) for j in range(m))
    assert med == sorted(nums)[(d - 1) // 2]
    # insert then delete half of relation 1: the sketch of the rest
    keys = rels[1]
    w = np.concatenate([np.ones(60, dtype=np.int64), -np.ones(30, dtype=np.int64)])
    both = oracle.create_ams_sketch(info, 1, np.concatenate([keys, keys[:30]]), w, m, coef)
    rest = oracle.create_ams_sketch(info, 1, keys[30:], None, m, coef)
    assert np.array_equal(both, rest)


def test_ams_unbiased_within_variance_bound():
    """Thm. 2.3: E[X] is the join size and Var(X) <= 3^(r-1)/m prod_k ||F_k||_2^2.  Over
    400 independent seeds the mean of X must lie within 5 standard errors of the join
    size computed from the frequency tables."""
    graph = W.chain(3)
    info = oracle.analyze(graph)
    m = 4
    rels = [W.random_small_relation(graph, k, 40, 5, seed=k).numpy() for k in range(3)]
    freqs = [oracle.frequency_tensor(r) for r in rels]
    J = oracle.join_size(info, freqs)
    var_bound = 3 ** (info.n_rel - 1) / m * math.prod(sum(v * v for v in f.values()) for f in freqs)
    xs = []
    for seed in range(400):
        coef = oracle.draw_ams_coefficients(1000 + seed, 1, m, len(info.edges))
        sk = [oracle.create_ams_sketch(info, k, rels[k], None, m, coef) for k in range(3)]
        nums, _ = oracle.estimate_ams(sk)
        xs.append(nums[0] / m)
    mean = sum(xs) / len(xs)
    assert abs(mean - J) <= 5 * math.sqrt(var_bound / len(xs)), (mean, J, var_bound)
    var = sum((x - mean) ** 2 for x in xs) / (len(xs) - 1)
    assert var <= 1.5 * var_bound, (var, var_bound)


# --------------------------------------------------------------------------- per-attribute sketches (Sec. 3.4)

def test_attr_sketch_single_join_equals_query_sketch():
    """For the one-join query, the component's hash functions are the join's: the
    per-attribute sketches and the stream order coincide with Alg. 2's sketches of the
    query (two independent routes to the same counters)."""
    graph = W.single_join()
    info = oracle.analyze(graph)
    m, d = 64, 3
    sign, bins = oracle.draw_attr_coefficients(77, d, info.n_comp)
    co = oracle.draw_coefficients(77, d, len(info.edges), info.n_comp)
    assert np.array_equal(sign, co.sign_array()) and np.array_equal(bins, co.bin_array())
    for k in range(2):
        keys = W.random_small_relation(graph, k, 500, 40, seed=k).numpy()
        w = W.turnstile_weights(500, 0.2, seed=k).numpy()
        a = oracle.create_attr_sketch(keys[:, 0], w, m, sign[:, 0], bins[:, 0])
        assert np.array_equal(a, oracle.create_sketch(info, k, keys, w, m, co))


def test_attr_sketch_definition_and_pairwise_estimate():
    """Counter by counter from the power-sum hashes, and the pairwise estimate against
    the inner-product definition; E[X] over seeds is the join size."""
    m, d = 8, 2
    x = W.uniform_keys(300, 12, seed=3).numpy().astype(np.uint32)
    y = W.uniform_keys(200, 12, seed=4).numpy().astype(np.uint32)
    sign, bins = oracle.draw_attr_coefficients(5, d, 1)
    a = oracle.create_attr_sketch(x, None, m, sign[:, 0], bins[:, 0])
    for t in range(d):
        ref = [0] * m
        for v in x.tolist():
            ref[oracle.bin_value(bins[t, 0].tolist(), v, m)] += oracle.sign_value(sign[t, 0].tolist(), v)
        assert a[t].tolist() == ref
    b = oracle.create_attr_sketch(y, None, m, sign[:, 0], bins[:, 0])
    reps, med = oracle.estimate_pairwise(a, b)
    assert reps == [int(np.dot(a[t].astype(object), b[t].astype(object))) for t in range(d)]
    fx, fy = oracle.frequency_tensor(x.reshape(-1, 1)), oracle.frequency_tensor(y.reshape(-1, 1))
    J = sum(c * fy.get(k, 0) for k, c in fx.items())
    est = []
    for seed in range(300):
        sg, bn = oracle.draw_attr_coefficients(900 + seed, 1, 1)
        a1 = oracle.create_attr_sketch(x, None, m, sg[:, 0], bn[:, 0])
        b1 = oracle.create_attr_sketch(y, None, m, sg[:, 0], bn[:, 0])
        est.append(oracle.estimate_pairwise(a1, b1)[1])
    var_bound = 3 / m * sum(v * v for v in fx.values()) * sum(v * v for v in fy.values())
    assert abs(sum(est) / len(est) - J) <= 5 * math.sqrt(var_bound / len(est))
