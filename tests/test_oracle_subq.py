"""Pins of the oracle's sub-query sketches (Sec. 3.4) against the paper's worked example,
the attribute-sketch definition, a brute-force evaluation, closed-form sharing counts and
unbiasedness (Thm. 3.1).  CPU only."""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _keys(graph, k, n, domain, seed):
    return W.random_small_relation(graph, k, n, domain, seed=seed).numpy()


def _signature(sq, i):
    return (sq.relations[i], tuple(sq.columns[i]))


def test_fig3_example_renumbering_and_reuse():
    """Fig. 3's query: attribute 1 is joined with 0 and with 3.  The sub-queries {0,1}
    and {1,3} each join attribute 1 once, so its sketch is the same in both (the reuse
    Sec. 3.4 describes); in the sub-query holding both joins, attribute 1 takes the two
    joins' own sign polynomials."""
    g = W.fig3_query()   # joins: 0 = (0,1), 1 = (1,3), 2 = (2,4); components {0,1,3} = 0, {2,4} = 1
    a = oracle.subquery(g, [0])
    b = oracle.subquery(g, [1])
    both = oracle.subquery(g, [0, 1])
    assert a.relations == [0, 1] and b.relations == [1, 2] and both.relations == [0, 1, 2]
    assert a.graph.n_rel == 2 and a.graph.attr_rel == (0, 1) and a.graph.edges == ((0, 1),)
    assert both.graph.attr_rel == (0, 1, 2) and both.graph.edges == ((0, 1), (1, 2))
    # relation 1's sketch: column 0 (attribute 1), component 0, the shared sign
    assert a.columns[1] == [(0, 0, (("comp", 0),))]
    assert b.columns[0] == [(0, 0, (("comp", 0),))]
    assert _signature(a, 1) == _signature(b, 0)
    # two joins in component 0: per-join signs, attribute 1 signed by both
    assert both.columns == [[(0, 0, (("join", 0),))], [(0, 0, (("join", 0), ("join", 1)))],
                            [(0, 0, (("join", 1),))]]
    # joins of different components: each component has one join, shared signs
    c = oracle.subquery(g, [0, 2])
    assert c.columns[1] == [(0, 0, (("comp", 0),)), (1, 1, (("comp", 1),))]


def test_disconnected_joins_are_refused():
    with pytest.raises(oracle.GraphError):
        oracle.subquery(W.chain(4), [0, 2])
    with pytest.raises(oracle.GraphError):
        oracle.subquery(W.chain(4), [])


def test_draw_prefix_is_the_attribute_sketch_draw():
    info = oracle.analyze(W.fig3_query())
    cs, bn, js = oracle.draw_subq_coefficients(77, 4, info.n_comp, len(info.edges))
    sa, ba = oracle.draw_attr_coefficients(77, 4, info.n_comp)
    assert np.array_equal(cs, sa) and np.array_equal(bn, ba)
    assert js.shape == (4, 3, 4) and int(js.max()) < oracle.P61


@pytest.mark.parametrize("graph", [W.fig3_query(), W.chain(4), W.multiway_star(4)])
def test_pairwise_subquery_is_the_attribute_sketch_inner_product(graph):
    """A one-join sub-query: each relation's sketch is its attribute's sketch with the
    component's hash functions, and the estimate is their inner product (Eq. 5, r = 2)."""
    info = oracle.analyze(graph)
    m, d = 13, 3
    cs, bn, js = oracle.draw_subq_coefficients(5, d, info.n_comp, len(info.edges))
    rels = [_keys(graph, k, 80, 6, 10 + k) for k in range(info.n_rel)]
    for e in range(len(info.edges)):
        sq = oracle.subquery(graph, [e])
        sks = []
        for i, k in enumerate(sq.relations):
            (c, q, signs), = sq.columns[i]
            assert signs == (("comp", q),)
            got = oracle.create_subq_sketch(info, sq.columns[i], rels[k], None, m, cs, bn, js)
            ref = oracle.create_attr_sketch(rels[k][:, c], None, m, cs[:, q], bn[:, q])
            assert np.array_equal(got, ref)
            sks.append(got)
        reps, med = oracle.estimate(oracle.analyze(sq.graph), sks, m)
        reps2, med2 = oracle.estimate_pairwise(sks[0], sks[1])
        assert reps == reps2 and med == med2


def test_subquery_sketch_equals_brute_force_definition():
    """Counter by counter from the definition: bucket = sum of the listed columns' bin
    values mod m, sign = product of the listed sign polynomials' signs, in Python
    integers with the power-sum hash."""
    graph = W.fig3_query()
    info = oracle.analyze(graph)
    m, d = 7, 2
    cs, bn, js = oracle.draw_subq_coefficients(9, d, info.n_comp, len(info.edges))
    rels = [_keys(graph, k, 30, 5, 50 + k) for k in range(info.n_rel)]
    w = [W.random_weights(30, -3, 3, seed=70 + k).numpy() for k in range(info.n_rel)]
    for joins in ([0, 1], [0, 1, 2], [1, 2], [2]):
        sq = oracle.subquery(graph, joins)
        for i, k in enumerate(sq.relations):
            got = oracle.create_subq_sketch(info, sq.columns[i], rels[k], w[k], m, cs, bn, js)
            for t in range(d):
                ref = [0] * m
                for tup, wt in zip(rels[k].tolist(), w[k].tolist()):
                    j, s = 0, 1
                    for c, q, signs in sq.columns[i]:
                        x = int(tup[c])
                        j += oracle.poly_value([int(v) for v in bn[t, q]], x)
                        for kind, idx in signs:
                            coef = cs[t, idx] if kind == "comp" else js[t, idx]
                            s *= oracle.sign_value([int(v) for v in coef], x)
                    ref[j % m] += s * int(wt)
                assert got[t].tolist() == ref, (joins, k, t)


def _n_targets(graph):
    sigs = set()
    for mask in W.connected_subqueries(graph):
        sq = oracle.subquery(graph, [e for e in range(len(graph.edges)) if (mask >> e) & 1])
        for i in range(len(sq.relations)):
            sigs.add(_signature(sq, i))
    return len(sigs)


@pytest.mark.parametrize("r", [3, 4, 5, 6, 7])
def test_chain_subchains_share_sketches(r):
    """All connected sub-chains of an r-chain need 3r - 4 distinct sketches: the end
    relations one each (their one column), every middle relation three (left column,
    right column, both), against r(r-1)(r+4)/6 relation sketches built separately."""
    assert _n_targets(W.chain(r)) == 3 * r - 4
    n_sub = len(W.connected_subqueries(W.chain(r)))
    assert n_sub == r * (r - 1) // 2
    assert sum(len(oracle.subquery(W.chain(r), [e for e in range(r - 1) if (mk >> e) & 1]).relations)
               for mk in W.connected_subqueries(W.chain(r))) == r * (r - 1) * (r + 4) // 6


def test_star_and_multiway_counts():
    """star(5): the centre's sketch for every non-empty set of its four columns (15) and
    one per leaf (4).  multiway_star(4), one component of four attributes: the centre
    once with the shared sign (one join) and once per set of two or three joins (4);
    each leaf once with the shared sign and once with its join's own sign."""
    assert _n_targets(W.star(5)) == 15 + 4
    assert _n_targets(W.multiway_star(4)) == (1 + 4) + 3 * 2


def _unbiased_stats(graph, joins, m, S, force_shared=False):
    info = oracle.analyze(graph)
    sq = oracle.subquery(graph, joins)
    sub_info = oracle.analyze(sq.graph)
    cols = sq.columns
    if force_shared:  # a planted mistake: one shared polynomial for every join of a component
        cols = [[(c, q, (("comp", q),)) for c, q, _ in cl] for cl in cols]
    rels = [_keys(graph, k, 60, 4, 300 + k) for k in sq.relations]
    freqs = [oracle.frequency_tensor(r[:, [c for c, _, _ in cl]]) for r, cl in zip(rels, cols)]
    J = oracle.join_size(sub_info, freqs)
    V = oracle.variance_bound(sub_info, freqs, m)
    xs = []
    for s in range(S):
        cs, bn, js = oracle.draw_subq_coefficients(2000 + s, 1, info.n_comp, len(info.edges))
        sks = [oracle.create_subq_sketch(info, cl, r, None, m, cs, bn, js) for r, cl in zip(rels, cols)]
        xs.append(oracle.estimate_alg3(sub_info, [c[0] for c in sks], m, method="direct"))
    mean = sum(xs) / S
    return mean, J, V


@pytest.mark.parametrize("graph,joins,m", [(W.multiway_star(3), [0, 1], 8), (W.fig3_query(), [0, 1, 2], 8),
                                           (W.chain(4), [1, 2], 16)])
def test_subquery_estimate_unbiased(graph, joins, m):
    """Thm. 3.1 for a sub-query under the reuse assignment: the mean over S seeds (one
    repetition each) is the sub-query's exact join size within 5 standard errors."""
    S = 1200
    mean, J, V = _unbiased_stats(graph, joins, m, S)
    assert abs(mean - J) <= 5 * math.sqrt(V / S), (mean, J, V)


def test_shared_sign_on_a_twice_joined_attribute_is_biased():
    """The planted mistake the assignment avoids: with one shared sign polynomial for
    both joins at the centre of multiway_star(3), the centre's sign is s(x)^2 = 1 and
    the estimate's mean leaves the join size by far more than 5 standard errors."""
    S = 1200
    mean, J, V = _unbiased_stats(W.multiway_star(3), [0, 1], 8, S, force_shared=True)
    assert abs(mean - J) > 5 * math.sqrt(V / S), (mean, J, V)
