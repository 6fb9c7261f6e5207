"""Serving loop through the C ABI: every estimate served in a mixed, concurrent trace
equals the estimate of the same query computed alone from exactly the updates that were
submitted before it; admission control by sketch memory."""
import random
import sys

import numpy as np
import pytest
import torch

import workloads as W
from tests.helpers import keys_u32, to_device_keys

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2402_15953_amd as csk


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pools(specs, pool_n):
    pools = []
    for qi, sp in enumerate(specs):
        rels = []
        for k in range(sp.graph.n_rel):
            keys = keys_u32(W.relation_keys(sp.graph, k, pool_n, "zipf", config=700 + qi, s=1.1, D=10 ** 5))
            rels.append(to_device_keys(keys))
        pools.append(rels)
    return pools


def _trace(specs, pool_n, n_req, seed, est_frac=0.2, del_frac=0.1, max_len=20_000):
    """(kind, qid, rel, off, len, sign) requests; deletes re-send a slice inserted earlier."""
    rng = random.Random(seed)
    inserted = {}
    out = []
    for _ in range(n_req):
        q = rng.randrange(len(specs))
        if rng.random() < est_frac:
            out.append(("E", q, 0, 0, 0, 0))
            continue
        k = rng.randrange(specs[q].graph.n_rel)
        prev = inserted.get((q, k), [])
        if prev and rng.random() < del_frac:
            off, ln = prev.pop(rng.randrange(len(prev)))
            out.append(("U", q, k, off, ln, -1))
        else:
            ln = rng.randint(1, max_len)
            off = rng.randrange(0, pool_n - ln + 1)
            inserted.setdefault((q, k), []).append((off, ln))
            out.append(("U", q, k, off, ln, +1))
    return out


def test_served_estimates_equal_alone():
    specs = W.batched_queries(10, seed=31, m_log2=(10, 14), d_choices=(5, 9), n_range=(10, 100))
    pool_n = 60_000
    pools = _pools(specs, pool_n)
    ones = torch.ones(pool_n, dtype=torch.int64, device="cuda")
    minus = -ones
    srv = csk.Server(n_streams=3, max_batch_items=64)
    qids = [srv.add_query(sp.graph, sp.m, sp.d, sp.sketch_seed) for sp in specs]
    trace = _trace(specs, pool_n, 400, seed=1)
    tickets = {}
    history = {q: [] for q in range(len(specs))}
    est_history = {}
    for i, (kind, q, k, off, ln, sign) in enumerate(trace):
        if kind == "U":
            keys = pools[q][k][off:off + ln]
            w = (ones if sign > 0 else minus)[off:off + ln]
            t = srv.submit_update(qids[q], k, keys, w, unit_weights=True)
            history[q].append((k, off, ln, sign))
        else:
            t = srv.submit_estimate(qids[q])
            est_history[t] = (q, list(history[q]))
        tickets[t] = (kind, q)
        if i % 97 == 0:
            srv.drain()
    srv.drain()
    comps = srv.poll(10_000)
    assert len(comps) == len(trace)
    assert all(c["status"] == 0 for c in comps)
    st = srv.stats()
    _say("server stats", st)
    assert st["update_launches"] < sum(1 for r in trace if r[0] == "U")   # updates were batched
    n_checked = 0
    for c in comps:
        if c["kind"] != 1:
            continue
        q, hist = est_history[c["ticket"]]
        sp = specs[q]
        alone = csk.Sketch(sp.graph, sp.m, sp.d, sp.sketch_seed)
        for (k, off, ln, sign) in hist:
            alone.update(k, pools[q][k][off:off + ln], (ones if sign > 0 else minus)[off:off + ln],
                         unit_weights=True)
        ref = alone.estimate()
        assert c["estimate"] == ref, (c["ticket"], q, c["estimate"], ref)
        alone.close()
        n_checked += 1
    _say("estimates checked", n_checked)
    assert n_checked > 40
    lat = sorted(c["done_us"] - c["submit_us"] for c in comps)
    assert lat[0] >= 0
    srv.close()


def test_admission_by_memory():
    g = W.chain(3)
    per = csk.sketch_bytes(g, 1 << 14, 9)
    srv = csk.Server(memory_budget=2 * per + 10)
    a = srv.add_query(g, 1 << 14, 9, 1)
    b = srv.add_query(g, 1 << 14, 9, 2)
    with pytest.raises(csk.CsError) as e:
        srv.add_query(g, 1 << 14, 9, 3)
    assert e.value.status == csk.CS_EBUSY
    srv.remove_query(a)
    c = srv.add_query(g, 1 << 14, 9, 4)   # fits again
    assert srv.stats()["live_queries"] == 2
    srv.close()
    del b, c


def test_queue_limit():
    g = W.single_join()
    srv = csk.Server(max_pending=4)
    q = srv.add_query(g, 1024, 5, 1)
    keys = torch.zeros(1 << 20, 1, dtype=torch.int32, device="cuda")
    n_ok, busy = 0, 0
    for _ in range(64):
        try:
            srv.submit_update(q, 0, keys)
            n_ok += 1
        except csk.CsError as e:
            assert e.status == csk.CS_EBUSY
            busy += 1
    srv.drain()
    assert n_ok >= 4
    comps = srv.poll()
    assert len(comps) == n_ok
    sk = srv.sketch(q)
    assert int(np.abs(sk.read_sketch(0)).sum(axis=1)[0]) == n_ok * (1 << 20)
    srv.close()


def test_update_order_across_streams():
    """A query updated by a large batch on one update stream and then by a tiny batch on
    another: its next estimate must include both (the second launch waits for the first)."""
    g = W.chain(3)
    m, d = 1 << 16, 9
    big_n, tiny_n = 1 << 23, 17
    keys = [to_device_keys(keys_u32(W.relation_keys(g, k, big_n, "zipf", config=760, s=1.1, D=10 ** 6)))
            for k in range(g.n_rel)]
    srv = csk.Server(n_streams=2, max_batch_items=1)
    q = srv.add_query(g, m, d, 11)
    alone = csk.Sketch(g, m, d, 11)
    for rnd in range(2):
        for k in range(g.n_rel):
            srv.submit_update(q, k, keys[k])                   # one epoch, stream A
            srv.submit_update(q, k, keys[k][:tiny_n])          # next epoch, stream B
            alone.update(k, keys[k])
            alone.update(k, keys[k][:tiny_n])
        t = srv.submit_estimate(q)
        srv.drain()
        comps = {c["ticket"]: c for c in srv.poll(1000)}
        assert comps[t]["status"] == 0
        assert comps[t]["estimate"] == alone.estimate(), rnd
    for k in range(g.n_rel):
        assert np.array_equal(srv.sketch(q).read_sketch(k), alone.read_sketch(k)), k
    alone.close()
    srv.close()


def test_remove_query_while_others_flow():
    """Removing one query waits only for its own requests; later submissions for it are
    refused; the other query's estimates still equal the same query computed alone."""
    g = W.chain(3)
    n = 1 << 16
    keys = [to_device_keys(keys_u32(W.relation_keys(g, k, n, "zipf", config=761, s=1.1, D=10 ** 5)))
            for k in range(g.n_rel)]
    srv = csk.Server(n_streams=2, max_batch_items=4)
    a = srv.add_query(g, 1 << 12, 5, 1)
    b = srv.add_query(g, 1 << 12, 5, 2)
    alone = csk.Sketch(g, 1 << 12, 5, 2)
    for k in range(g.n_rel):
        srv.submit_update(a, k, keys[k])
        srv.submit_update(b, k, keys[k])
        alone.update(k, keys[k])
    srv.remove_query(a)
    with pytest.raises(csk.CsError) as e:
        srv.submit_update(a, 0, keys[0])
    assert e.value.status == csk.CS_EINVAL
    with pytest.raises(csk.CsError):
        srv.remove_query(a)
    t = srv.submit_estimate(b)
    srv.drain()
    comps = {c["ticket"]: c for c in srv.poll(1000)}
    assert comps[t]["status"] == 0 and comps[t]["estimate"] == alone.estimate()
    assert srv.stats()["live_queries"] == 1
    alone.close()
    srv.close()
