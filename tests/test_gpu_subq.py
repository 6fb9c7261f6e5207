"""Sub-query sketches (Sec. 3.4) on the GPU against the oracle, through the C ABI: one
pass per base relation fills every distinct sketch (target); every target is
bit-identical to the oracle's sketch of each (sub-query, relation) it serves, targets are
shared exactly where the oracle's hash assignment makes two sketches equal, and every
sub-query's per-repetition estimates and median equal the oracle's exact integers."""
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


def _joins(mask):
    return [e for e in range(32) if (mask >> e) & 1]


CASES = [
    # graph, sub-query masks (None: every connected one), n, m, d, weights, Zipf domain
    (W.chain(5), None, (1 << 20) + 4097, 1 << 18, 3, None, 10 ** 4),   # 513 blocks, ragged tail
    (W.chain(5), None, 3000, 1 << 18, 5, "pm1", 10 ** 4),
    (W.multiway_star(4), None, 20_000, 1000, 5, "pm1", 10 ** 4),        # a component of four attributes
    (W.star(5), None, 5000, 1 << 14, 2, None, 10 ** 4),                 # 15 sketches of the centre
    (W.fig3_query(), None, 10_000, 3 << 10, 4, "small", 10 ** 4),        # general weights: atomics
    (W.fig3_query(), None, 80, (3 << 14) + 5, 3, "small", 40),           # three ranges, odd m
    (W.chain(3), [1, 1, 3], 5, 2, 1, None, 10 ** 4),                     # duplicate masks, m = 2
    (W.chain(4), None, 70_000, 1 << 20, 2, None, 10 ** 4),              # 64 bucket ranges
    (W.chain(3), None, 700_000, 1 << 16, 64, "pm1", 10 ** 4),           # d = 64: two chunks
    (W.chain(4), [0b111], 0, 1 << 12, 3, None, 10 ** 4),                # no tuples
]


def _oracle_reps(sub_info, sks, m, d):
    """Exact per-repetition estimates: inner products for one join, number-theoretic
    transforms for powers of two and small m, the sparse ring otherwise (small inputs)."""
    if sub_info.n_rel == 2:
        return oracle.estimate_pairwise(sks[0], sks[1])[0]
    if m & (m - 1) == 0 or m <= 4096:
        return [oracle.estimate_alg3(sub_info, [c[t] for c in sks], m, method="ntt") for t in range(d)]
    return [oracle.estimate_sparse(sub_info, [c[t] for c in sks], m) for t in range(d)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_subquery_targets_and_estimates(case):
    graph, masks, n, m, d, wk, D = CASES[case]
    masks = W.connected_subqueries(graph) if masks is None else masks
    _say("subq", case, graph.name, len(masks), n, m, d, wk)
    info = oracle.analyze(graph)
    rels = [keys_u32(W.relation_keys(graph, k, max(n, 1), "zipf", config=410 + case, s=1.0, D=D))[:n]
            for k in range(graph.n_rel)]
    weights = None
    if wk == "pm1":
        weights = [W.turnstile_weights(n, 0.3, seed=k).numpy() for k in range(graph.n_rel)]
    elif wk == "small":
        weights = [W.random_weights(n, -5, 5, seed=k).numpy() for k in range(graph.n_rel)]
    seed = 500 + case
    cs_, bn, js = oracle.draw_subq_coefficients(seed, d, info.n_comp, len(info.edges))
    sq = csk.SubQueries(graph, masks, m, d, seed)
    gc, gb, gj = sq.coefficients()
    assert np.array_equal(gc, cs_) and np.array_equal(gb, bn) and np.array_equal(gj, js)
    for k in range(graph.n_rel):
        wd = None if weights is None else torch.from_numpy(weights[k]).cuda()
        sq.update(k, to_device_keys(rels[k]), wd, unit_weights=(wk == "pm1"))
    torch.cuda.synchronize()
    nt, tof = sq.layout()
    subs = [oracle.subquery(graph, _joins(mk)) for mk in masks]
    # the oracle's sketch of every distinct (relation, columns and signs)
    ref = {}
    target_sig = {}
    for qi, s in enumerate(subs):
        for i, k in enumerate(s.relations):
            sig = (k, tuple(s.columns[i]))
            if sig not in ref:
                ref[sig] = oracle.create_subq_sketch(info, s.columns[i], rels[k],
                                                     None if weights is None else weights[k], m, cs_, bn, js)
            t = int(tof[qi, k])
            assert t >= 0
            # a target serves exactly one signature
            assert target_sig.setdefault(t, sig) == sig, (qi, k)
        for k in range(graph.n_rel):
            if k not in s.relations:
                assert tof[qi, k] == -1
    assert nt == len(ref) == len(target_sig)
    for t, sig in target_sig.items():
        assert np.array_equal(sq.read_target(t), ref[sig]), (t, sig[0])
    # estimates
    alls = sq.estimate_all()
    for qi, s in enumerate(subs):
        sks = [ref[(k, tuple(s.columns[i]))] for i, k in enumerate(s.relations)]
        sub_info = oracle.analyze(s.graph)
        reps = _oracle_reps(sub_info, sks, m, d)
        med = oracle.median_lower(reps)
        _say("  sub-query", qi, s.joins, "oracle done")
        got = sq.estimate(qi, reps=True)
        assert got["exact"] and got["rep_ints"] == reps, (qi, s.joins)
        assert got["value"] == float(med)
        assert alls[qi]["exact"] and alls[qi]["value"] == float(med)
    sq.close()


def test_pairwise_subqueries_equal_attribute_sketches():
    """With the same seed, a one-join sub-query's sketches are the per-attribute sketches
    (both draw the component's sign and bin polynomials first)."""
    graph = W.chain(4)
    n, m, d = 200_000, 1 << 16, 5
    rels = [keys_u32(W.relation_keys(graph, k, n, "zipf", config=431, s=1.1, D=10 ** 5)) for k in range(graph.n_rel)]
    info = oracle.analyze(graph)
    masks = [1 << e for e in range(len(graph.edges))]
    sq = csk.SubQueries(graph, masks, m, d, 11)
    ak = csk.AttrSketches(graph, m, d, 11)
    for k in range(graph.n_rel):
        sq.update(k, to_device_keys(rels[k]))
        ak.update(k, to_device_keys(rels[k]))
    torch.cuda.synchronize()
    nt, tof = sq.layout()
    assert nt == graph.n_attr
    for qi, mk in enumerate(masks):
        (u, v), = [graph.edges[e] for e in _joins(mk)]
        for a in (u, v):
            k = info.attr_rel[a]
            assert np.array_equal(sq.read_target(int(tof[qi, k])), ak.read_sketch(a))
        e1 = sq.estimate(qi, reps=True)
        e2 = ak.estimate_join(u, v, reps=True)
        assert e1["rep_ints"] == e2["rep_ints"] and e1["value"] == e2["value"]
    sq.close()
    ak.close()


def test_update_order_and_reset():
    """Two calls per relation equal one call on the concatenation; reset zeroes."""
    graph = W.chain(5)
    m, d = 1 << 15, 4
    masks = W.connected_subqueries(graph)
    a = csk.SubQueries(graph, masks, m, d, 3)
    b = csk.SubQueries(graph, masks, m, d, 3)
    for k in range(graph.n_rel):
        keys = keys_u32(W.relation_keys(graph, k, 50_001, "zipf", config=432, s=1.2, D=1000))
        a.update(k, to_device_keys(keys))
        b.update(k, to_device_keys(keys[:20_000]))
        b.update(k, to_device_keys(keys[20_000:]))
    torch.cuda.synchronize()
    nt, _ = a.layout()
    for t in range(nt):
        assert np.array_equal(a.read_target(t), b.read_target(t))
    a.reset()
    torch.cuda.synchronize()
    for t in range(nt):
        assert not a.read_target(t).any()
    a.close()
    b.close()


@pytest.mark.parametrize("graph,masks", [
    (W.chain(4), [0b101]),          # not connected
    (W.chain(4), [0]),              # empty
    (W.chain(4), [0b1000]),         # names no join of the graph
    (W.star(6), None),              # 31 sketches of the centre relation
])
def test_refusals(graph, masks):
    masks = W.connected_subqueries(graph) if masks is None else masks
    with pytest.raises(csk.CsError) as e:
        csk.SubQueries(graph, masks, 1024, 2, 1)
    assert e.value.status == csk.CS_EINVAL
