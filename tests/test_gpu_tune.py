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


def _arch_of_table(path):
    for line in open(path).read().splitlines()[1:]:
        if line.strip():
            return line.split()[0]
    raise AssertionError("empty tuning table")


def test_batch_tuner_keeps_counters_and_plans_with_its_choice(tmp_path):
    """cs_tune_batch_update: every candidate's counters equal the global-atomic run's
    (none rejected), the chosen class entries are stored, and a batch planned with them
    gives exactly the per-query path's sketches."""
    from tests.test_gpu_batch import _batched_items, _make_inputs, _plain
    csk.tune_clear()
    specs = W.batched_queries(48, seed=21, m_log2=(10, 16), n_range=(50, 200_000))
    _say("batch tuner", len(specs), "queries")
    data = _make_inputs(specs)
    plain = _plain(specs, data)
    sks, items, keep = _batched_items(specs, data)
    b = csk.Batch()
    rep = b.tune(items)
    _say("  report", rep)
    assert rep["classes"] >= 1 and rep["rejected"] == 0
    assert rep["tuned_ms"] > 0 and rep["rule_ms"] > 0
    assert csk.tune_count() == rep["classes"]
    path = tmp_path / "tuned.txt"
    csk.tune_save(str(path))
    codes = {int(l.split()[7]) for l in path.read_text().splitlines()[1:]}
    assert codes <= {csk.TUNE_BATCH_ATOMIC, csk.TUNE_BATCH_SEGMENT, csk.TUNE_BATCH_SORT}
    # the handles' counters were not touched by tuning
    for sk in sks:
        for k in range(sk.graph.n_rel):
            assert not sk.read_sketch(k).any()
    b.update(items)
    torch.cuda.synchronize()
    for qi, (sp, a, p) in enumerate(zip(specs, sks, plain)):
        for k in range(sp.graph.n_rel):
            assert np.array_equal(a.read_sketch(k), p.read_sketch(k)), (qi, k)
    ests = b.estimate(sks)
    for e, p in zip(ests, plain):
        assert e["value"] == p.estimate()["value"]
    b.close()
    csk.tune_clear()


@pytest.mark.parametrize("weights", ["unit", "general"])
def test_sort_reduce_tasks_give_the_per_query_sketches(weights, tmp_path):
    """Every class of a batch forced to sort-reduce tasks through the tuning table: the
    batch plans only sort-reduce tasks, and the sketches (Zipf-skewed keys, so runs of
    equal counters in every wavefront) equal the per-query path's counter for counter,
    for unit and for general int64 weights (up to +-2^40)."""
    from tests.test_gpu_batch import _batched_items, _make_inputs, _plain
    csk.tune_clear()
    specs = W.batched_queries(24, seed=23, m_log2=(10, 16), n_range=(50, 150_000))
    _say("sort-reduce", weights, len(specs), "queries")
    data = _make_inputs(specs, weights_kind="big" if weights == "general" else None)
    plain = _plain(specs, data)
    sks, items, keep = _batched_items(specs, data)
    b = csk.Batch()
    rep = b.tune(items)
    assert rep["rejected"] == 0
    path = tmp_path / "tuned.txt"
    csk.tune_save(str(path))
    lines = path.read_text().splitlines()
    forced = [lines[0]]
    for line in lines[1:]:
        f = line.split()
        f[7], f[8] = str(csk.TUNE_BATCH_SORT), "16"
        forced.append(" ".join(f))
    fpath = tmp_path / "forced.txt"
    fpath.write_text("\n".join(forced) + "\n")
    csk.tune_clear()
    csk.tune_load(str(fpath))
    b.update(items)
    torch.cuda.synchronize()
    st = b.stats()
    assert st["tasks_sort_reduce"] > 0 and st["tasks_atomic"] == 0 and st["tasks_segment"] == 0, st
    for qi, (sp, a, p) in enumerate(zip(specs, sks, plain)):
        for k in range(sp.graph.n_rel):
            assert np.array_equal(a.read_sketch(k), p.read_sketch(k)), (qi, k)
    b.close()
    csk.tune_clear()


SPLIT_CASES = [
    # graph, m, d, n per relation (the transform length is m, or 2^ceil(log2(2m - 1)))
    (W.chain(4), 1 << 16, 3, 20_000),     # spectral plan, 2^16
    (W.chain(4), 1 << 18, 2, 3000),       # spectral plan, 2^18
    (W.fig3_query(), 1 << 14, 3, 3000),   # general plan, 2^14
    (W.chain(3), 3000, 3, 5000),          # general plan, zero-padded 2^13
]


@pytest.mark.parametrize("case", range(len(SPLIT_CASES)))
def test_every_transform_split_gives_the_exact_estimate(case, tmp_path):
    """cs_tune_transform runs every legal split with identical spectra; then each split,
    forced through the tuning table, gives the oracle's exact per-repetition estimates."""
    import oracle
    graph, m, d, n = SPLIT_CASES[case]
    L = (m - 1).bit_length() if m & (m - 1) == 0 else (2 * m - 2).bit_length()
    csk.tune_clear()
    rep = csk.tune_transform(L, n_vec=8)
    _say("split", case, graph.name, m, "length 2^%d" % L, rep)
    assert all(c["valid"] == 1 for c in rep["candidates"])
    splits = [c["split"] for c in rep["candidates"]]
    assert len(splits) >= 2
    path = tmp_path / "t.txt"
    csk.tune_save(str(path))
    arch = _arch_of_table(path)
    rels = [keys_u32(W.relation_keys(graph, k, n, "zipf", config=890 + case, s=1.1, D=10 ** 4))
            for k in range(graph.n_rel)]
    info, co, ref = oracle_sketches(graph, rels, None, m, d, 77)
    want = [oracle.estimate_alg3(info, [c[t] for c in ref], m, method="ntt") for t in range(d)]
    sk = csk.Sketch(graph, m, d, 77)
    for k in range(graph.n_rel):
        sk.update(k, to_device_keys(rels[k]))
    for S in splits:
        f = tmp_path / ("s%d.txt" % S)
        f.write_text("csketch-tune 1\n%s %d 0 0 0 0 0 %d %d 0 0.1\n" % (arch, 1 << L, csk.TUNE_TRANSFORM_SPLIT, S))
        csk.tune_clear()
        csk.tune_load(str(f))
        got = sk.estimate(reps=True)
        assert got["exact"] and got["rep_ints"] == want, (S, got["rep_ints"], want)
    sk.close()
    csk.tune_clear()
