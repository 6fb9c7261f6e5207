"""Per-attribute sketches (Sec. 3.4 reuse) on the GPU against the oracle, through the C
ABI: every attribute's counters bit-identical, pairwise join estimates exact."""
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


CASES = [
    # graph, n, m, d, weights
    (W.chain(4), 50_000, 1 << 16, 5, None),     # 16-bit counter kernels
    (W.fig3_query(), 20_000, 1000, 3, "pm1"),   # attribute 1 joined twice; m not a power of two
    (W.star(4), 30_000, 1 << 18, 3, "big"),     # three-column centre relation
    (W.chain(3), 1, 64, 2, None),
    (W.chain(3), 300_000, 1 << 20, 3, "pm1"),   # partition strategy
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_attr_sketches_and_pairwise_estimates(case):
    graph, n, m, d, wk = CASES[case]
    _say("attr", case, graph.name, n, m, d, wk)
    info = oracle.analyze(graph)
    rels = [keys_u32(W.relation_keys(graph, k, n, "zipf", config=330 + case, s=1.1, D=10 ** 4))
            for k in range(graph.n_rel)]
    weights = None
    if wk == "pm1":
        weights = [W.turnstile_weights(n, 0.1, seed=k).numpy() for k in range(graph.n_rel)]
    elif wk == "big":
        weights = [W.random_weights(n, -2 ** 40, 2 ** 40, seed=k).numpy() for k in range(graph.n_rel)]
    seed = 90 + case
    sign, bins = oracle.draw_attr_coefficients(seed, d, info.n_comp)
    ak = csk.AttrSketches(graph, m, d, seed)
    gs, gb = ak.coefficients()
    assert np.array_equal(gs, sign) and np.array_equal(gb, bins)
    for k in range(graph.n_rel):
        wd = None if weights is None else torch.from_numpy(weights[k]).cuda()
        ak.update(k, to_device_keys(rels[k]), wd, unit_weights=(wk == "pm1"))
    torch.cuda.synchronize()
    ref = {}
    for k in range(graph.n_rel):
        for c, u in enumerate(info.omega[k]):
            q = info.psi[u]
            ref[u] = oracle.create_attr_sketch(rels[k][:, c], None if weights is None else weights[k], m,
                                               sign[:, q], bins[:, q])
            assert np.array_equal(ak.read_sketch(u), ref[u]), (k, u)
    for (u, v) in info.edges:
        est = ak.estimate_join(u, v, reps=True)
        reps, med = oracle.estimate_pairwise(ref[u], ref[v])
        if all(abs(x) < 2 ** 120 for x in reps):
            assert est["exact"] and est["rep_ints"] == reps
            assert est["value"] == float(med)
    ak.close()


def test_attr_single_join_matches_query_sketch():
    """For one join the per-attribute sketches are the query's sketches (same draw)."""
    graph = W.single_join()
    n, m, d = 40_000, 4096, 5
    rels = [keys_u32(W.relation_keys(graph, k, n, "zipf", config=341, s=1.2, D=5000)) for k in range(2)]
    ak = csk.AttrSketches(graph, m, d, 7)
    sk = csk.Sketch(graph, m, d, 7)
    for k in range(2):
        ak.update(k, to_device_keys(rels[k]))
        sk.update(k, to_device_keys(rels[k]))
    torch.cuda.synchronize()
    for k in range(2):
        assert np.array_equal(ak.read_sketch(k), sk.read_sketch(k))
    a = ak.estimate_join(0, 1)
    b = sk.estimate()
    assert a["value"] == b["value"] and a["value_i64"] == b["value_i64"]
    ak.close()
    sk.close()


def test_attr_rejects_bad_pairs():
    graph = W.fig3_query()
    ak = csk.AttrSketches(graph, 64, 2, 1)
    info = oracle.analyze(graph)
    other = next(v for v in range(graph.n_attr) if info.psi[v] != info.psi[0])
    for u, v in ((0, 0), (0, other), (0, graph.n_attr)):
        with pytest.raises(csk.CsError) as e:
            ak.estimate_join(u, v)
        assert e.value.status == csk.CS_EINVAL
    ak.reset()
    torch.cuda.synchronize()
    assert not ak.read_sketch(0).any()
    ak.close()
