"""Parity at the full workload sizes, in the launch configuration the benchmark times.

* chain-3, 1e7 tuples per relation, Zipf(1.1) over 1e6, m = 2^16, d = 9: every counter
  and every repetition's estimate against the oracle.
* 5-chain, 96 calls of 2^20 tuples per relation, Zipf(s) over 1e7, m = 2^18, d = 15:
  at s = 1.0 every counter, all 15 repetitions and the median; at s = 0.5 and 1.5 one
  sampled repetition (all its counters, and its estimate) against the oracle.
* 4096 uneven chain/star queries in one batched update and one batched estimate:
  sampled queries against the oracle (all repetitions).
* 256 live queries (m = 2^14..2^18, d = 9) in the serving loop: sampled queries' served
  estimates against the same query computed alone, and against the oracle.

The oracle runs on the host in parallel threads (one call per relation); its inputs are
the generator's keys, never anything the GPU computed."""
import random
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2402_15953_amd as csk

INT128_EXACT = 2 ** 125


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _host_u32(t: torch.Tensor) -> np.ndarray:
    a = t.cpu().numpy().view(np.uint32)
    return a.reshape(a.shape[0], -1)


def _oracle_rep_sketches(graph, host_keys, host_w, m, d, seed, reps):
    """Oracle sketches of every relation restricted to repetitions `reps`: [k] -> int64
    [len(reps)][m].  Coefficients come from the full d-repetition draw; the oracle is run
    on the sub-table of the sampled repetitions."""
    info = oracle.analyze(graph)
    co = oracle.draw_coefficients(seed, d, len(info.edges), info.n_comp)
    sub = oracle.Coefficients(len(reps), co.n_edges, co.n_comps, [co.sign[t] for t in reps],
                              [co.bins[t] for t in reps])
    with ThreadPoolExecutor(max_workers=min(8, graph.n_rel)) as ex:
        futs = [ex.submit(oracle.create_sketch, info, k, host_keys[k],
                          None if host_w is None else host_w[k], m, sub) for k in range(graph.n_rel)]
        return info, [f.result() for f in futs]


def _oracle_sketches_chunked(graph, host_keys, m, d, seed, workers=16, pieces=16):
    """Oracle sketches (every repetition) of relations too large for one thread: each
    relation's tuples are cut into pieces, each piece sketched by the oracle, and the
    pieces' sketches summed modulo 2^64 -- a sketch is linear in its input (Sec. 2.2,
    pinned by the oracle's linearity tests)."""
    info = oracle.analyze(graph)
    co = oracle.draw_coefficients(seed, d, len(info.edges), info.n_comp)
    jobs = []
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for k in range(graph.n_rel):
            n = host_keys[k].shape[0]
            step = (n + pieces - 1) // pieces
            for i0 in range(0, n, step):
                jobs.append((k, ex.submit(oracle.create_sketch, info, k, host_keys[k][i0:i0 + step], None, m, co)))
        out = [np.zeros((d, m), dtype=np.int64) for _ in range(graph.n_rel)]
        for k, f in jobs:
            out[k] += f.result()   # int64 addition wraps like the counters
    return info, out


def _check_rep(est, t, exact):
    """Repetition t of a GPU estimate against the oracle's exact integer."""
    if abs(exact) < INT128_EXACT:
        assert est["rep_ints"][t] == exact, (t, est["rep_ints"][t], exact, est["rep_bounds"][t])
        assert est["rep_values"][t] == float(exact)
    else:
        assert abs(est["rep_values"][t] - exact) <= 1e-12 * abs(exact), (t, est["rep_values"][t], exact)


def _check_median(est, reps_exact):
    med = oracle.median_lower(reps_exact)
    if abs(med) < INT128_EXACT:
        assert est["exact"] and est["value"] == float(med)
    else:
        assert abs(est["value"] - med) <= 1e-12 * abs(med)
    if -2 ** 63 <= med < 2 ** 63:
        assert est["value_i64"] == med


@pytest.mark.timeout(400)
def test_chain3_full_size():
    graph, n, m, d, seed = W.chain(3), 10_000_000, 1 << 16, 9, 7
    _say("chain3 full", n, m, d)
    dev = torch.device("cuda", 0)
    keys = [W.relation_keys(graph, k, n, "zipf", config=2, s=1.1, D=10 ** 6, device=dev).to(torch.int32).contiguous()
            for k in range(graph.n_rel)]
    stream = torch.cuda.Stream()
    sk = csk.Sketch(graph, m, d, seed)
    with torch.cuda.stream(stream):
        for k in range(graph.n_rel):
            sk.update(k, keys[k], None, stream=stream)
        est = sk.estimate(stream=stream, reps=True)
    torch.cuda.synchronize()
    host = [_host_u32(kk) for kk in keys]
    del keys
    info, ref = _oracle_rep_sketches(graph, host, None, m, d, seed, list(range(d)))
    for k in range(graph.n_rel):
        assert np.array_equal(sk.read_sketch(k), ref[k]), k
    reps = [oracle.estimate_alg3(info, [ref[k][t] for k in range(graph.n_rel)], m, method="ntt") for t in range(d)]
    for t in range(d):
        _check_rep(est, t, reps[t])
    _check_median(est, reps)
    _say("  estimate", est["value"], "exact", est["exact"])
    sk.close()


@pytest.mark.timeout(900)
def test_chain5_full_size_all_repetitions():
    """5-chain at Zipf(1.0): every counter of every repetition, all 15 repetitions'
    exact estimates and their median against the oracle."""
    graph, m, d, seed, s = W.chain(5), 1 << 18, 15, 8, 1.0
    n_call, calls = 1 << 20, 96
    n = n_call * calls
    _say("chain5 full, all repetitions", s, n, m, d)
    dev = torch.device("cuda", 0)
    keys = [W.relation_keys(graph, k, n, "zipf", config=3, s=s, D=10 ** 7, device=dev).to(torch.int32).contiguous()
            for k in range(graph.n_rel)]
    stream = torch.cuda.Stream()
    sk = csk.Sketch(graph, m, d, seed)
    with torch.cuda.stream(stream):
        for c in range(calls):
            for k in range(graph.n_rel):
                sk.update(k, keys[k][c * n_call:(c + 1) * n_call], None, stream=stream)
        est = sk.estimate(stream=stream, reps=True)
    torch.cuda.synchronize()
    host = [_host_u32(kk) for kk in keys]
    del keys
    _say("  oracle sketches")
    info, ref = _oracle_sketches_chunked(graph, host, m, d, seed)
    del host
    for k in range(graph.n_rel):
        assert np.array_equal(sk.read_sketch(k), ref[k]), k
    _say("  oracle estimates")
    with ThreadPoolExecutor(max_workers=8) as ex:
        reps = list(ex.map(lambda t: oracle.estimate_alg3(info, [ref[k][t] for k in range(graph.n_rel)], m,
                                                          method="ntt"), range(d)))
    for t in range(d):
        _check_rep(est, t, reps[t])
    _check_median(est, reps)
    _say("  median", est["value"], "exact", est["exact"])
    sk.close()


@pytest.mark.timeout(400)
@pytest.mark.parametrize("s,t", [(0.5, 0), (1.5, 14)])
def test_chain5_full_size_sampled_repetition(s, t):
    graph, m, d, seed = W.chain(5), 1 << 18, 15, 8
    n_call, calls = 1 << 20, 96
    n = n_call * calls
    _say("chain5 full", s, "repetition", t, n, m, d)
    dev = torch.device("cuda", 0)
    keys = [W.relation_keys(graph, k, n, "zipf", config=3, s=s, D=10 ** 7, device=dev).to(torch.int32).contiguous()
            for k in range(graph.n_rel)]
    stream = torch.cuda.Stream()
    sk = csk.Sketch(graph, m, d, seed)
    with torch.cuda.stream(stream):
        for c in range(calls):
            for k in range(graph.n_rel):
                sk.update(k, keys[k][c * n_call:(c + 1) * n_call], None, stream=stream)
        est = sk.estimate(stream=stream, reps=True)
    torch.cuda.synchronize()
    host = [_host_u32(kk) for kk in keys]
    del keys
    info, ref = _oracle_rep_sketches(graph, host, None, m, d, seed, [t])
    del host
    for k in range(graph.n_rel):
        assert np.array_equal(sk.read_sketch(k)[t], ref[k][0]), k
    exact = oracle.estimate_alg3(info, [ref[k][0] for k in range(graph.n_rel)], m, method="ntt")
    _check_rep(est, t, exact)
    _say("  repetition", t, "estimate", exact, "median", est["value"])
    sk.close()


def _sample_queries(specs, count, seed):
    """Largest total input, most relations, largest sketch, smallest input, then random."""
    idx = {max(range(len(specs)), key=lambda i: sum(specs[i].n_per_rel)),
           max(range(len(specs)), key=lambda i: (specs[i].graph.n_rel, sum(specs[i].n_per_rel))),
           max(range(len(specs)), key=lambda i: (specs[i].m * specs[i].d, -sum(specs[i].n_per_rel))),
           min(range(len(specs)), key=lambda i: sum(specs[i].n_per_rel))}
    rng = random.Random(seed)
    while len(idx) < count:
        idx.add(rng.randrange(len(specs)))
    return sorted(idx)


@pytest.mark.timeout(600)
def test_batched_4096_queries_full_size_sampled():
    specs = W.batched_queries(4096, seed=4)
    dev = torch.device("cuda", 0)
    _say("batched full", len(specs), "queries", sum(sum(sp.n_per_rel) for sp in specs), "tuples")
    keys = [[W.relation_keys(sp.graph, k, sp.n_per_rel[k], "zipf", config=4000 + qi, s=1.2, D=10 ** 6,
                             device=dev).to(torch.int32).contiguous() for k in range(sp.graph.n_rel)]
            for qi, sp in enumerate(specs)]
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    sks = [csk.Sketch(sp.graph, sp.m, sp.d, sp.sketch_seed) for sp in specs]
    b = csk.Batch()
    items = [(sk_, k, kk, None, False) for sk_, ks in zip(sks, keys) for k, kk in enumerate(ks)]
    b.capture(items, stream=stream)
    b.replay(stream=stream)
    torch.cuda.synchronize()
    ests = b.estimate(sks, stream=stream, reps=True)
    sample = _sample_queries(specs, 10, seed=3)
    _say("  sampled", sample)
    for qi in sample:
        sp = specs[qi]
        host = [_host_u32(kk) for kk in keys[qi]]
        info, ref = _oracle_rep_sketches(sp.graph, host, None, sp.m, sp.d, sp.sketch_seed, list(range(sp.d)))
        for k in range(sp.graph.n_rel):
            assert np.array_equal(sks[qi].read_sketch(k), ref[k]), (qi, k)
        reps = [oracle.estimate_alg3(info, [ref[k][t] for k in range(sp.graph.n_rel)], sp.m, method="ntt")
                for t in range(sp.d)]
        for t in range(sp.d):
            _check_rep(ests[qi], t, reps[t])
        _check_median(ests[qi], reps)
    b.close()
    for sk_ in sks:
        sk_.close()


@pytest.mark.timeout(600)
def test_serving_256_queries_full_size_sampled():
    specs = W.batched_queries(256, seed=5, m_log2=(14, 18), d_choices=(9,), n_range=(1, 2))
    pool = 1 << 18
    dev = torch.device("cuda", 0)
    pools = [[W.relation_keys(sp.graph, k, pool, "zipf", config=5000 + qi, s=1.1, D=10 ** 6,
                              device=dev).to(torch.int32).contiguous() for k in range(sp.graph.n_rel)]
             for qi, sp in enumerate(specs)]
    ones = torch.ones(pool, dtype=torch.int64, device=dev)
    minus = -ones
    torch.cuda.synchronize()
    srv = csk.Server(n_streams=3, max_batch_items=1024)
    qids = [srv.add_query(sp.graph, sp.m, sp.d, sp.sketch_seed) for sp in specs]
    _say("serving full", len(specs), "queries", srv.stats()["used_bytes"], "counter bytes")
    rng = random.Random(9)
    inserted, history, est_of = {}, {q: [] for q in range(len(specs))}, {}
    n_req = 3000
    for i in range(n_req):
        q = rng.randrange(len(specs))
        if rng.random() < 0.2:
            tk = srv.submit_estimate(qids[q])
            est_of[tk] = (q, len(history[q]))
            continue
        k = rng.randrange(specs[q].graph.n_rel)
        prev = inserted.get((q, k), [])
        if prev and rng.random() < 0.1:
            off, ln = prev.pop(rng.randrange(len(prev)))
            sign = -1
        else:
            ln = 1 << rng.randint(10, 18)
            off = rng.randrange(0, pool - ln + 1)
            inserted.setdefault((q, k), []).append((off, ln))
            sign = 1
        srv.submit_update(qids[q], k, pools[q][k][off:off + ln], (ones if sign > 0 else minus)[off:off + ln],
                          unit_weights=True)
        history[q].append((k, off, ln, sign))
        if i % 256 == 255:
            srv.drain()
    srv.drain()
    comps = srv.poll(1 << 13)
    assert len(comps) == n_req and all(c["status"] == 0 for c in comps)
    served = {}
    for c in comps:
        if c["kind"] == 1:
            q, h = est_of[c["ticket"]]
            served.setdefault(q, []).append((h, c["estimate"]))
    sample = sorted(served, key=lambda q: -len(served[q]))[:6]
    _say("  sampled", sample)
    for q in sample:
        sp = specs[q]
        alone = csk.Sketch(sp.graph, sp.m, sp.d, sp.sketch_seed)
        done = 0
        for h, value in sorted(served[q], key=lambda e: e[0]):
            for (k, off, ln, sign) in history[q][done:h]:
                alone.update(k, pools[q][k][off:off + ln], (ones if sign > 0 else minus)[off:off + ln],
                             unit_weights=True)
            done = h
            assert value == alone.estimate(), (q, h)
        alone.close()
    # the last served estimate of two sampled queries against the oracle
    for q in sample[:2]:
        sp = specs[q]
        h, value = max(served[q], key=lambda e: e[0])
        host_k = [[] for _ in range(sp.graph.n_rel)]
        host_w = [[] for _ in range(sp.graph.n_rel)]
        for (k, off, ln, sign) in history[q][:h]:
            host_k[k].append(_host_u32(pools[q][k][off:off + ln]))
            host_w[k].append(np.full(ln, sign, dtype=np.int64))
        cols = [len(sp.graph.columns(k)) for k in range(sp.graph.n_rel)]
        keys_np = [np.concatenate(host_k[k]) if host_k[k] else np.zeros((0, cols[k]), np.uint32)
                   for k in range(sp.graph.n_rel)]
        w_np = [np.concatenate(host_w[k]) if host_w[k] else np.zeros(0, np.int64) for k in range(sp.graph.n_rel)]
        info, ref = _oracle_rep_sketches(sp.graph, keys_np, w_np, sp.m, sp.d, sp.sketch_seed, list(range(sp.d)))
        reps = [oracle.estimate_alg3(info, [ref[k][t] for k in range(sp.graph.n_rel)], sp.m, method="ntt")
                for t in range(sp.d)]
        med = oracle.median_lower(reps)
        if abs(med) < INT128_EXACT:
            assert value["exact"] and value["value"] == float(med), (q, value, med)
        else:
            assert abs(value["value"] - med) <= 1e-12 * abs(med)
        if -2 ** 63 <= med < 2 ** 63:
            assert value["value_i64"] == med
    srv.close()
