"""Asynchronous estimate through the C ABI: the cs_estimate_t the device publishes into
pinned host memory or device memory equals the synchronous estimate of the same
counters (Eq. 5, median over repetitions), stream-ordered with updates, with no host
round trip in the call."""
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


def _pinned():
    return torch.zeros(csk.ESTIMATE_BYTES, dtype=torch.uint8, pin_memory=True)


def _fields(e):
    return {k: e[k] for k in ("value", "exact", "value_i64", "d", "n_modular")}


CASES = [
    # graph, n, m, d, weights
    (W.chain(3), 100_000, 1 << 16, 9, None),      # fp64 estimate certified exact
    (W.chain(3), 40_000, 1 << 12, 5, "big"),      # repetitions need the modular step
    (W.single_join(), 50_000, 1 << 14, 5, None),  # inner-product plan
    (W.star(4), 20_000, 1 << 10, 3, "pm1"),
]


def _weights(kind, graph, n):
    if kind is None:
        return None
    if kind == "pm1":
        return [W.turnstile_weights(n, 0.1, seed=k).numpy() for k in range(graph.n_rel)]
    return [W.random_weights(n, -2 ** 30, 2 ** 30, seed=60 + k).numpy() for k in range(graph.n_rel)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_async_matches_sync(case):
    graph, n, m, d, wk = CASES[case]
    _say("async", case, graph.name, n, m, d, wk)
    rels = [keys_u32(W.relation_keys(graph, k, n, "zipf", config=700 + case, s=1.1, D=10 ** 4))
            for k in range(graph.n_rel)]
    weights = _weights(wk, graph, n)
    sk = csk.Sketch(graph, m, d, 50 + case)
    for k in range(graph.n_rel):
        w = None if weights is None else torch.from_numpy(weights[k]).cuda()
        sk.update(k, to_device_keys(rels[k]), w)
    # first estimate on a fresh handle: the speculative modular step takes 5 primes
    host = _pinned()
    dev = torch.zeros(csk.ESTIMATE_BYTES, dtype=torch.uint8, device="cuda")
    sk.estimate_async(host.data_ptr())
    sk.estimate_async(dev.data_ptr())
    torch.cuda.synchronize()
    a = csk.read_estimate(host)
    b = csk.read_estimate(dev.cpu())
    ref = sk.estimate()
    assert _fields(a) == _fields(ref) == _fields(b)
    if ref["exact"] and m <= 1 << 14:
        info, _, sk_ref = oracle_sketches(graph, rels, weights, m, d, 50 + case)
        _, med = oracle.estimate(info, sk_ref, m)
        assert ref["value"] == float(med)
    # after a synchronous estimate the speculative step takes exactly what it needed
    sk.estimate_async(host.data_ptr())
    torch.cuda.synchronize()
    assert _fields(csk.read_estimate(host)) == _fields(ref)
    sk.close()


def test_async_is_stream_ordered_with_updates():
    """update, estimate, update, estimate, all enqueued before one synchronisation: each
    published estimate is that of the counters at its point in the stream."""
    graph = W.chain(3)
    n, m, d = 60_000, 1 << 14, 5
    rels = [keys_u32(W.relation_keys(graph, k, n, "zipf", config=710, s=1.2, D=10 ** 4)) for k in range(3)]
    sk = csk.Sketch(graph, m, d, 9)
    half = csk.Sketch(graph, m, d, 9)
    stream = torch.cuda.Stream()
    bufs = [_pinned() for _ in range(3)]
    kd = [to_device_keys(r) for r in rels]
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        sk.estimate_async(bufs[0].data_ptr(), stream=stream)
        for k in range(3):
            sk.update(k, kd[k][: n // 2], stream=stream)
        sk.estimate_async(bufs[1].data_ptr(), stream=stream)
        for k in range(3):
            sk.update(k, kd[k][n // 2:], stream=stream)
        sk.estimate_async(bufs[2].data_ptr(), stream=stream)
    stream.synchronize()
    for k in range(3):
        half.update(k, kd[k][: n // 2])
    torch.cuda.synchronize()
    e0, e1, e2 = (csk.read_estimate(b) for b in bufs)
    assert e0["exact"] and e0["value"] == 0.0 and e0["value_i64"] == 0
    assert _fields(e1) == _fields(half.estimate())
    assert _fields(e2) == _fields(sk.estimate())
    sk.close()
    half.close()


def test_async_refuses_general_plan():
    graph = W.chain(3)
    sk = csk.Sketch(graph, 1000, 3, 1)
    assert sk.info()["plan"] == csk.PLAN_GENERAL
    dev = torch.zeros(csk.ESTIMATE_BYTES, dtype=torch.uint8, device="cuda")
    with pytest.raises(csk.CsError) as e:
        sk.estimate_async(dev.data_ptr())
    assert e.value.status == csk.CS_EINVAL
    torch.cuda.synchronize()
    assert not dev.cpu().any()
    assert sk.estimate()["exact"]
    sk.close()


def test_async_refuses_pageable_destination():
    """A destination the device cannot write (pageable host memory) is refused before
    anything is enqueued; the handle keeps working."""
    graph = W.chain(3)
    sk = csk.Sketch(graph, 1 << 12, 3, 2)
    page = np.zeros(csk.ESTIMATE_BYTES, dtype=np.uint8)
    with pytest.raises(csk.CsError) as e:
        sk.estimate_async(page.ctypes.data)
    assert e.value.status == csk.CS_EINVAL
    assert not page.any()
    host = _pinned()
    sk.estimate_async(host.data_ptr())
    torch.cuda.synchronize()
    assert csk.read_estimate(host)["exact"]
    sk.close()
