"""Batched mode through the C ABI: one persistent update launch and one batched
estimate must give exactly what the plain per-query calls give (and the oracle)."""
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


def _make_inputs(specs, s=1.2, D=10 ** 5, weights_kind=None):
    """Device keys (and weights) for every relation of every query spec."""
    data = []
    for qi, sp in enumerate(specs):
        rels = []
        for k in range(sp.graph.n_rel):
            n = sp.n_per_rel[k]
            keys = keys_u32(W.relation_keys(sp.graph, k, n, "zipf", config=400 + qi, s=s, D=D))
            w = None
            if weights_kind == "pm1":
                w = W.turnstile_weights(n, 0.1, seed=qi * 16 + k).numpy()
            elif weights_kind == "big":
                w = W.random_weights(n, -2 ** 40, 2 ** 40, seed=qi * 16 + k).numpy()
            rels.append((keys, w))
        data.append(rels)
    return data


def _plain(specs, data, unit=False):
    out = []
    for sp, rels in zip(specs, data):
        sk = csk.Sketch(sp.graph, sp.m, sp.d, sp.sketch_seed)
        for k, (keys, w) in enumerate(rels):
            sk.update(k, to_device_keys(keys), None if w is None else torch.from_numpy(w).cuda(), unit_weights=unit)
        out.append(sk)
    torch.cuda.synchronize()
    return out


def _batched_items(specs, data, unit=False):
    sks, items, keep = [], [], []
    for sp, rels in zip(specs, data):
        sk = csk.Sketch(sp.graph, sp.m, sp.d, sp.sketch_seed)
        sks.append(sk)
        for k, (keys, w) in enumerate(rels):
            kd = to_device_keys(keys)
            wd = None if w is None else torch.from_numpy(w).cuda()
            keep.append((kd, wd))
            items.append((sk, k, kd, wd, unit))
    return sks, items, keep


@pytest.mark.parametrize("weights_kind", [None, "pm1", "big"])
def test_batched_update_equals_plain(weights_kind):
    specs = W.batched_queries(40, seed=11 + (weights_kind is not None), m_log2=(10, 16),
                              n_range=(50, 60_000))
    specs.append(W.QuerySpec(W.fig3_query(), 512, 5, (3000, 4000, 100, 2000), 99))
    specs.append(W.QuerySpec(W.single_join(), 1 << 16, 9, (200_000, 150_000), 98))
    # LDS segment tasks off the one-join fast hash: an attribute in two joins, and m not
    # a power of two
    specs.append(W.QuerySpec(W.fig3_query(), 512, 5, (40_001, 30_002, 20_003, 50_000), 95))
    specs.append(W.QuerySpec(W.chain(3), 1000, 5, (50_001, 60_002, 40_003), 94))
    _say("batch", weights_kind, len(specs), "queries")
    data = _make_inputs(specs, weights_kind=weights_kind)
    unit = weights_kind == "pm1"
    plain = _plain(specs, data, unit=unit)
    sks, items, keep = _batched_items(specs, data, unit=unit)
    b = csk.Batch()
    b.update(items)
    torch.cuda.synchronize()
    st = b.stats()
    _say("  tasks", st)
    assert st["tasks_atomic"] > 0 and st["tasks_segment"] > 0
    for qi, (sp, a, p) in enumerate(zip(specs, sks, plain)):
        for k in range(sp.graph.n_rel):
            assert np.array_equal(a.read_sketch(k), p.read_sketch(k)), (qi, k)
    # a few queries against the oracle directly
    for qi in (0, len(specs) - 4, len(specs) - 3, len(specs) - 2, len(specs) - 1):
        sp = specs[qi]
        rels = [r[0] for r in data[qi]]
        ws = None if weights_kind is None else [r[1] for r in data[qi]]
        info, co, ref = oracle_sketches(sp.graph, rels, ws, sp.m, sp.d, sp.sketch_seed)
        for k in range(sp.graph.n_rel):
            assert np.array_equal(sks[qi].read_sketch(k), ref[k]), (qi, k)
    b.close()


def test_graph_capture_replay():
    """A captured batch replayed several times adds its tuples once per replay; every
    replay is checked, with eager work and synchronisation in between."""
    specs = W.batched_queries(12, seed=5, m_log2=(10, 14), n_range=(100, 40_000))
    data = _make_inputs(specs)
    plain = _plain(specs, data)
    ref = [[p.read_sketch(k) for k in range(sp.graph.n_rel)] for sp, p in zip(specs, plain)]
    sks, items, keep = _batched_items(specs, data)
    b = csk.Batch()
    b.capture(items)
    for rep in range(1, 4):
        b.replay()
        torch.cuda.synchronize()
        junk = torch.ones(1 << 20, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        assert float(junk) == float(1 << 20)
        for qi, sp in enumerate(specs):
            for k in range(sp.graph.n_rel):
                assert np.array_equal(sks[qi].read_sketch(k), ref[qi][k] * rep), (rep, qi, k)
    b.close()


def test_batched_estimate_equals_plain():
    specs = W.batched_queries(30, seed=21, m_log2=(10, 16), n_range=(100, 50_000), r_range=(2, 6))
    specs.append(W.QuerySpec(W.fig3_query(), 256, 5, (3000, 4000, 100, 2000), 97))
    specs.append(W.QuerySpec(W.multiway_star(4), 128, 3, (500, 400, 300, 200), 96))
    data = _make_inputs(specs, weights_kind="big")
    plain = _plain(specs, data)
    b = csk.Batch()
    got = b.estimate(plain, reps=True)
    for qi, (sp, sk) in enumerate(zip(specs, plain)):
        ref = sk.estimate(reps=True)
        assert got[qi] == ref, (qi, got[qi], ref)
    # and the oracle for a handful
    for qi in (0, 7, len(specs) - 2, len(specs) - 1):
        sp = specs[qi]
        info = oracle.analyze(sp.graph)
        refs = [sk_ for sk_ in (plain[qi].read_sketch(k) for k in range(sp.graph.n_rel))]
        reps, med = oracle.estimate(info, refs, sp.m, method="ntt")
        if all(abs(x) < 2 ** 125 for x in reps):
            assert got[qi]["rep_ints"] == reps, qi
    b.close()
